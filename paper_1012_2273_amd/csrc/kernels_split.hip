// kernels_split.hip -- the split step of the three-term bfloat16 product:
// every binary32 x becomes hi = bf16(x) and lo = bf16(x - hi), both rounded
// to nearest even by the gfx950 conversion instruction. x - hi is exact in
// binary32 (the low 16 significand bits of x, at most), so hi + lo carries
// 16 significand bits of x.
//
// Both kernels are bound by HBM bandwidth: 4 bytes read and 4 bytes written
// per element. The transposing variant stages a 64 x 64 tile through LDS
// so that reads along the input rows and writes along the output rows are
// both coalesced.
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "internal.h"

namespace g355 {

__device__ __forceinline__ void split1(float x, uint16_t &h, uint16_t &l) {
  const __bf16 hb = (__bf16)x;
  const float r = x - (float)hb;
  h = __builtin_bit_cast(uint16_t, hb);
  l = __builtin_bit_cast(uint16_t, (__bf16)r);
}

// Same orientation: (rows x cols) -> (rows x cols_pad), zeros in [cols,
// cols_pad). One thread per 4 consecutive elements of a plane row; VEC: X
// rows and planes are 16/8-byte aligned.
template <bool VEC>
__global__ void __launch_bounds__(256)
split_rows_kernel(int64_t rows, int64_t cols, const float *__restrict__ X, int64_t ldx,
                  uint16_t *__restrict__ hi, uint16_t *__restrict__ lo, int64_t ldo,
                  int64_t cols_pad) {
  const int64_t cq = (cols_pad + 3) / 4;
  const int64_t total = rows * cq;
  for (int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; t < total;
       t += (int64_t)gridDim.x * blockDim.x) {
    const int64_t r = t / cq, c = (t - r * cq) * 4;
    const float *src = X + r * ldx + c;
    uint16_t *dh = hi + r * ldo + c, *dl = lo + r * ldo + c;
    if (VEC && c + 4 <= cols) {
      const float4 v = *reinterpret_cast<const float4 *>(src);
      uint16_t h0, h1, h2, h3, l0, l1, l2, l3;
      split1(v.x, h0, l0); split1(v.y, h1, l1); split1(v.z, h2, l2); split1(v.w, h3, l3);
      *reinterpret_cast<uint2 *>(dh) = make_uint2(h0 | ((uint32_t)h1 << 16), h2 | ((uint32_t)h3 << 16));
      *reinterpret_cast<uint2 *>(dl) = make_uint2(l0 | ((uint32_t)l1 << 16), l2 | ((uint32_t)l3 << 16));
    } else {
      for (int e = 0; e < 4 && c + e < cols_pad; ++e) {
        if (c + e < cols) {
          split1(src[e], dh[e], dl[e]);
        } else {
          dh[e] = 0;
          dl[e] = 0;
        }
      }
    }
  }
}

// Transposing: (rows x cols) -> planes of (cols x rows_pad): out[c][r],
// zeros for r in [rows, rows_pad).
__global__ void __launch_bounds__(256)
split_transpose_kernel(int64_t rows, int64_t cols, const float *__restrict__ X, int64_t ldx,
                       uint16_t *__restrict__ hi, uint16_t *__restrict__ lo, int64_t ldo,
                       int64_t rows_pad) {
  constexpr int T = 64, PITCH = T + 2;
  __shared__ uint16_t sh[2][T][PITCH];
  const int64_t tiles_c = (cols + T - 1) / T;
  const int64_t r0 = (int64_t)(blockIdx.x / tiles_c) * T;
  const int64_t c0 = (int64_t)(blockIdx.x % tiles_c) * T;
  const int tid = threadIdx.x;
#pragma unroll
  for (int i = 0; i < T * T / 256; ++i) {
    const int idx = tid + i * 256;
    const int r = idx / T, c = idx % T;
    uint16_t h = 0, l = 0;
    if (r0 + r < rows && c0 + c < cols) split1(X[(r0 + r) * ldx + c0 + c], h, l);
    sh[0][r][c] = h;
    sh[1][r][c] = l;
  }
  __syncthreads();
#pragma unroll
  for (int i = 0; i < T * T / 256; ++i) {
    const int idx = tid + i * 256;
    const int oc = idx / T, orr = idx % T;      // output row = input column
    if (c0 + oc < cols && r0 + orr < rows_pad) {
      hi[(c0 + oc) * ldo + r0 + orr] = sh[0][orr][oc];
      lo[(c0 + oc) * ldo + r0 + orr] = sh[1][orr][oc];
    }
  }
}

// Both operands of the split product in one launch. Workgroups [0, na)
// split 64 x 64 tiles of A into row-major planes (rows x cols_a_pad, zero
// padding); workgroups [na, na + nb) split 64 x 64 tiles of B and write the
// planes transposed (cols_b x rows_b_pad, zero padding), staging each tile
// through LDS so that both the binary32 reads and the 16-byte plane writes
// are coalesced. VEC: 16-byte aligned inputs with row pitches that are
// multiples of 4 elements.
struct SplitJob {
  const float *X; int64_t ldx, rows, cols, pad;   // pad: padded plane row length
  uint16_t *hi, *lo; int64_t ldo;
  int64_t tiles_c;                                // 64-wide tiles across cols (A) / pad rows (B)
};

template <bool VEC>
__device__ __forceinline__ void load4(const float *X, int64_t ldx, int64_t rows, int64_t cols,
                                      int64_t r, int64_t c, float v[4]) {
  if (r < rows && VEC && c + 4 <= cols) {
    const float4 f = *reinterpret_cast<const float4 *>(X + r * ldx + c);
    v[0] = f.x; v[1] = f.y; v[2] = f.z; v[3] = f.w;
  } else {
#pragma unroll
    for (int e = 0; e < 4; ++e) v[e] = (r < rows && c + e < cols) ? X[r * ldx + c + e] : 0.0f;
  }
}

template <bool VEC>
__global__ void __launch_bounds__(256)
split_pair_kernel(SplitJob a, SplitJob b, int64_t na) {
  constexpr int T = 64, PITCH = T + 8;
  __shared__ __attribute__((aligned(16))) uint16_t sh[2][T][PITCH];
  const int tid = threadIdx.x;
  if ((int64_t)blockIdx.x < na) {
    // A: plane[r][c] for c < pad (zeros past cols)
    const int64_t r0 = (int64_t)(blockIdx.x / a.tiles_c) * T, c0 = (int64_t)(blockIdx.x % a.tiles_c) * T;
#pragma unroll
    for (int i = 0; i < 4; ++i) {
      const int idx = tid + 256 * i;
      const int64_t r = r0 + idx / 16, c = c0 + (idx % 16) * 4;
      if (r >= a.rows || c >= a.pad) continue;
      float v[4];
      load4<VEC>(a.X, a.ldx, a.rows, a.cols, r, c, v);
      uint16_t h[4], l[4];
#pragma unroll
      for (int e = 0; e < 4; ++e) split1(v[e], h[e], l[e]);
      uint16_t *dh = a.hi + r * a.ldo + c, *dl = a.lo + r * a.ldo + c;
      if (c + 4 <= a.pad) {   // planes: 8-byte aligned rows (pad, ldo multiples of 8)
        *reinterpret_cast<uint2 *>(dh) = make_uint2(h[0] | ((uint32_t)h[1] << 16), h[2] | ((uint32_t)h[3] << 16));
        *reinterpret_cast<uint2 *>(dl) = make_uint2(l[0] | ((uint32_t)l[1] << 16), l[2] | ((uint32_t)l[3] << 16));
      } else {
        for (int e = 0; c + e < a.pad; ++e) { dh[e] = h[e]; dl[e] = l[e]; }
      }
    }
    return;
  }
  // B: input tile rows r0.. (K), cols c0.. (N); planes out[c][r], r < pad
  const int64_t bid = (int64_t)blockIdx.x - na;
  const int64_t r0 = (bid / b.tiles_c) * T, c0 = (bid % b.tiles_c) * T;
#pragma unroll
  for (int i = 0; i < 4; ++i) {
    const int idx = tid + 256 * i;
    const int rr = idx / 16, cc = (idx % 16) * 4;
    float v[4];
    load4<VEC>(b.X, b.ldx, b.rows, b.cols, r0 + rr, c0 + cc, v);
#pragma unroll
    for (int e = 0; e < 4; ++e) split1(v[e], sh[0][rr][cc + e], sh[1][rr][cc + e]);
  }
  __syncthreads();
#pragma unroll
  for (int i = 0; i < 4; ++i) {
    const int v = tid + 256 * i;                 // 1024 vectors of 8 = 2 planes x 64 rows x 8
    const int pl = v / 512, oc = (v % 512) / 8, rv = (v % 8) * 8;
    const int64_t orow = c0 + oc, ocol = r0 + rv;
    if (orow >= b.cols || ocol >= b.pad) continue;
    uint32_t w[4];
#pragma unroll
    for (int j = 0; j < 4; ++j)
      w[j] = sh[pl][rv + 2 * j][oc] | ((uint32_t)sh[pl][rv + 2 * j + 1][oc] << 16);
    uint16_t *dst = (pl == 0 ? b.hi : b.lo) + orow * b.ldo + ocol;
    *reinterpret_cast<uint4 *>(dst) = make_uint4(w[0], w[1], w[2], w[3]);
  }
}

hipError_t launch_split_pair(int64_t m, int64_t n, int64_t k, const float *A, int64_t lda,
                             const float *B, int64_t ldb, uint16_t *ahi, uint16_t *alo,
                             uint16_t *bhi, uint16_t *blo, int64_t kp, int64_t ldp,
                             hipStream_t stream) {
  if (m <= 0 || n <= 0 || k <= 0) return hipSuccess;
  if (kp % 8 != 0 || ldp % 8 != 0 || ldp < kp || ((uintptr_t)bhi % 16) || ((uintptr_t)blo % 16) ||
      ((uintptr_t)ahi % 8) || ((uintptr_t)alo % 8))
    return hipErrorInvalidValue;
  SplitJob a{A, lda, m, k, kp, ahi, alo, ldp, (kp + 63) / 64};
  SplitJob b{B, ldb, k, n, kp, bhi, blo, ldp, (n + 63) / 64};
  const int64_t na = ((m + 63) / 64) * a.tiles_c;
  const int64_t nb = ((kp + 63) / 64) * b.tiles_c;
  if (na + nb > 0x7fffffff) return hipErrorInvalidValue;
  const bool vec = ((uintptr_t)A % 16 == 0) && (lda % 4 == 0) && ((uintptr_t)B % 16 == 0) &&
                   (ldb % 4 == 0);
  if (vec)
    hipLaunchKernelGGL(split_pair_kernel<true>, dim3((unsigned)(na + nb)), dim3(256), 0, stream, a,
                       b, na);
  else
    hipLaunchKernelGGL(split_pair_kernel<false>, dim3((unsigned)(na + nb)), dim3(256), 0, stream, a,
                       b, na);
  return hipGetLastError();
}

hipError_t launch_split(int64_t rows, int64_t cols, const float *X, int64_t ldx, bool transpose,
                        uint16_t *hi, uint16_t *lo, int64_t ldo, int64_t out_pad,
                        hipStream_t stream) {
  if (rows <= 0 || cols <= 0) return hipSuccess;
  if (transpose) {
    const int64_t tiles = ((out_pad + 63) / 64) * ((cols + 63) / 64);
    if (tiles > 0x7fffffff) return hipErrorInvalidValue;
    hipLaunchKernelGGL(split_transpose_kernel, dim3((unsigned)tiles), dim3(256), 0, stream,
                       rows, cols, X, ldx, hi, lo, ldo, out_pad);
  } else {
    const bool vec = ((uintptr_t)X % 16 == 0) && (ldx % 4 == 0) && ((uintptr_t)hi % 8 == 0) &&
                     ((uintptr_t)lo % 8 == 0) && (ldo % 4 == 0);
    const int64_t work = rows * ((out_pad + 3) / 4);
    int64_t blocks = (work + 255) / 256;
    if (blocks > 65536) blocks = 65536;
    if (vec)
      hipLaunchKernelGGL(split_rows_kernel<true>, dim3((unsigned)blocks), dim3(256), 0, stream,
                         rows, cols, X, ldx, hi, lo, ldo, out_pad);
    else
      hipLaunchKernelGGL(split_rows_kernel<false>, dim3((unsigned)blocks), dim3(256), 0, stream,
                         rows, cols, X, ldx, hi, lo, ldo, out_pad);
  }
  return hipGetLastError();
}

}  // namespace g355
