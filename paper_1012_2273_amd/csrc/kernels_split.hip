// kernels_split.hip -- the split step of the split products: every binary32
// x becomes NP bfloat16 planes, each rounded to nearest even by the gfx950
// conversion instruction:
//   two planes:   hi = bf16(x), lo = bf16(x - hi)
//   three planes: hi = bf16(x), mid = bf16(x - hi), lo = bf16((x - hi) - mid)
// Every difference is exact in binary32 (it is the part of x below the
// planes already taken), so hi + lo carries 16 significand bits of x and
// hi + mid + lo all 24.
//
// The kernels are bound by HBM bandwidth: 4 bytes read and 2 NP bytes
// written per element. The transposing variants stage a 64 x 64 tile
// through LDS so that reads along the input rows and writes along the
// output rows are both coalesced.
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "gemm_tile.hpp"
#include "internal.h"

namespace g355 {

// Plane pointers of one split operand.
template <int NP> struct Planes { uint16_t *p[NP]; };

// Same orientation: (rows x cols) -> (rows x cols_pad), zeros in [cols,
// cols_pad). One thread per 4 consecutive elements of a plane row; VEC: X
// rows 16-byte and planes 8-byte aligned.
template <bool VEC, int NP>
__global__ void __launch_bounds__(256)
split_rows_kernel(int64_t rows, int64_t cols, const float *__restrict__ X, int64_t ldx,
                  Planes<NP> out, int64_t ldo, int64_t cols_pad) {
  const int64_t cq = (cols_pad + 3) / 4;
  const int64_t total = rows * cq;
  for (int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; t < total;
       t += (int64_t)gridDim.x * blockDim.x) {
    const int64_t r = t / cq, c = (t - r * cq) * 4;
    const float *src = X + r * ldx + c;
    if (VEC && c + 4 <= cols) {
      const float4 v = *reinterpret_cast<const float4 *>(src);
      uint16_t s0[NP], s1[NP], s2[NP], s3[NP];
      split_x<NP>(v.x, s0); split_x<NP>(v.y, s1); split_x<NP>(v.z, s2); split_x<NP>(v.w, s3);
#pragma unroll
      for (int p = 0; p < NP; ++p)
        *reinterpret_cast<uint2 *>(out.p[p] + r * ldo + c) =
            make_uint2(s0[p] | ((uint32_t)s1[p] << 16), s2[p] | ((uint32_t)s3[p] << 16));
    } else {
      for (int e = 0; e < 4 && c + e < cols_pad; ++e) {
        uint16_t s[NP];
        if (c + e < cols) {
          split_x<NP>(src[e], s);
        } else {
#pragma unroll
          for (int p = 0; p < NP; ++p) s[p] = 0;
        }
#pragma unroll
        for (int p = 0; p < NP; ++p) out.p[p][r * ldo + c + e] = s[p];
      }
    }
  }
}

// Transposing: (rows x cols) -> planes of (cols x rows_pad): out[c][r],
// zeros for r in [rows, rows_pad).
template <int NP>
__global__ void __launch_bounds__(256)
split_transpose_kernel(int64_t rows, int64_t cols, const float *__restrict__ X, int64_t ldx,
                       Planes<NP> out, int64_t ldo, int64_t rows_pad) {
  constexpr int T = 64, PITCH = T + 2;
  __shared__ uint16_t sh[NP][T][PITCH];
  const int64_t tiles_c = (cols + T - 1) / T;
  const int64_t r0 = (int64_t)(blockIdx.x / tiles_c) * T;
  const int64_t c0 = (int64_t)(blockIdx.x % tiles_c) * T;
  const int tid = threadIdx.x;
#pragma unroll
  for (int i = 0; i < T * T / 256; ++i) {
    const int idx = tid + i * 256;
    const int r = idx / T, c = idx % T;
    uint16_t s[NP];
#pragma unroll
    for (int p = 0; p < NP; ++p) s[p] = 0;
    if (r0 + r < rows && c0 + c < cols) split_x<NP>(X[(r0 + r) * ldx + c0 + c], s);
#pragma unroll
    for (int p = 0; p < NP; ++p) sh[p][r][c] = s[p];
  }
  __syncthreads();
#pragma unroll
  for (int i = 0; i < T * T / 256; ++i) {
    const int idx = tid + i * 256;
    const int oc = idx / T, orr = idx % T;      // output row = input column
    if (c0 + oc < cols && r0 + orr < rows_pad) {
#pragma unroll
      for (int p = 0; p < NP; ++p) out.p[p][(c0 + oc) * ldo + r0 + orr] = sh[p][orr][oc];
    }
  }
}

// Both operands of a split product in one launch. Workgroups [0, na) split
// 64 x 64 tiles of A into row-major planes (rows x pad, zero padding);
// workgroups [na, na + nb) split 64 x 64 tiles of B and write the planes
// transposed (cols x pad, zero padding), staging each tile through LDS so
// that both the binary32 reads and the 16-byte plane writes are coalesced.
// VEC: 16-byte aligned inputs with row pitches that are multiples of 4
// elements.
template <int NP> struct SplitJob {
  const float *X; int64_t ldx, rows, cols, pad;   // pad: padded plane row length
  Planes<NP> out; int64_t ldo;
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

template <bool VEC, int NP>
__global__ void __launch_bounds__(256)
split_pair_kernel(SplitJob<NP> a, SplitJob<NP> b, int64_t na) {
  // 132-byte rows: the transposed reads below take one column of rows
  // rv, rv + 8, ..., rv + 56 in 8 neighbouring lanes, which a 132-byte pitch
  // spreads over 8 different 32-byte bank windows (a 144-byte pitch put them
  // in two: 82% of the LDS cycles were bank conflicts)
  constexpr int T = 64, PITCH = T + 2;
  __shared__ __attribute__((aligned(16))) uint16_t sh[NP][T][PITCH];
  const int tid = threadIdx.x;
  if ((int64_t)blockIdx.x < na) {
    // A: plane[r][c] for c < pad (zeros past cols)
    const int64_t r0 = (int64_t)(blockIdx.x / a.tiles_c) * T, c0 = (int64_t)(blockIdx.x % a.tiles_c) * T;
    // all four loads first, so that four are in flight per lane (one at a
    // time left the kernel waiting on memory latency)
    float v[4][4];
#pragma unroll
    for (int i = 0; i < 4; ++i) {
      const int idx = tid + 256 * i;
      const int64_t r = r0 + idx / 16, c = c0 + (idx % 16) * 4;
      load4<VEC>(a.X, a.ldx, a.rows, a.cols, r, c, v[i]);
    }
#pragma unroll
    for (int i = 0; i < 4; ++i) {
      const int idx = tid + 256 * i;
      const int64_t r = r0 + idx / 16, c = c0 + (idx % 16) * 4;
      if (r >= a.rows || c >= a.pad) continue;
      uint16_t s[4][NP];
#pragma unroll
      for (int e = 0; e < 4; ++e) split_x<NP>(v[i][e], s[e]);
#pragma unroll
      for (int p = 0; p < NP; ++p) {
        uint16_t *d = a.out.p[p] + r * a.ldo + c;
        if (c + 4 <= a.pad) {   // planes: 8-byte aligned rows (pad, ldo multiples of 8)
          *reinterpret_cast<uint2 *>(d) =
              make_uint2(s[0][p] | ((uint32_t)s[1][p] << 16), s[2][p] | ((uint32_t)s[3][p] << 16));
        } else {
          for (int e = 0; c + e < a.pad; ++e) d[e] = s[e][p];
        }
      }
    }
    return;
  }
  // B: input tile rows r0.. (K), cols c0.. (N); planes out[c][r], r < pad
  const int64_t bid = (int64_t)blockIdx.x - na;
  const int64_t r0 = (bid / b.tiles_c) * T, c0 = (bid % b.tiles_c) * T;
  float v[4][4];
#pragma unroll
  for (int i = 0; i < 4; ++i) {
    const int idx = tid + 256 * i;
    load4<VEC>(b.X, b.ldx, b.rows, b.cols, r0 + idx / 16, c0 + (idx % 16) * 4, v[i]);
  }
#pragma unroll
  for (int i = 0; i < 4; ++i) {
    const int idx = tid + 256 * i;
    const int rr = idx / 16, cc = (idx % 16) * 4;
#pragma unroll
    for (int e = 0; e < 4; ++e) {
      uint16_t s[NP];
      split_x<NP>(v[i][e], s);
#pragma unroll
      for (int p = 0; p < NP; ++p) sh[p][rr][cc + e] = s[p];
    }
  }
  __syncthreads();
  // NP planes x 64 rows x 8 vectors of 8 elements, 256 threads
#pragma unroll
  for (int i = 0; i < 2 * NP; ++i) {
    const int v = tid + 256 * i;
    const int pl = v / 512, oc = (v % 512) / 8, rv = (v % 8) * 8;
    const int64_t orow = c0 + oc, ocol = r0 + rv;
    if (orow >= b.cols || ocol >= b.pad) continue;
    uint32_t w[4];
#pragma unroll
    for (int j = 0; j < 4; ++j)
      w[j] = sh[pl][rv + 2 * j][oc] | ((uint32_t)sh[pl][rv + 2 * j + 1][oc] << 16);
    uint16_t *dst = b.out.p[pl] + orow * b.ldo + ocol;
    *reinterpret_cast<uint4 *>(dst) = make_uint4(w[0], w[1], w[2], w[3]);
  }
}

template <int NP>
static hipError_t launch_pair(int64_t m, int64_t n, int64_t k, const float *A, int64_t lda,
                              const float *B, int64_t ldb, uint16_t *const *ap,
                              uint16_t *const *bp, int64_t kp, int64_t ldp, hipStream_t stream) {
  SplitJob<NP> a{A, lda, m, k, kp, {}, ldp, (kp + 63) / 64};
  SplitJob<NP> b{B, ldb, k, n, kp, {}, ldp, (n + 63) / 64};
  for (int p = 0; p < NP; ++p) {
    a.out.p[p] = ap[p];
    b.out.p[p] = bp[p];
  }
  const int64_t na = ((m + 63) / 64) * a.tiles_c;
  const int64_t nb = ((kp + 63) / 64) * b.tiles_c;
  if (na + nb > 0x7fffffff) return hipErrorInvalidValue;
  const bool vec = ((uintptr_t)A % 16 == 0) && (lda % 4 == 0) && ((uintptr_t)B % 16 == 0) &&
                   (ldb % 4 == 0);
  if (vec)
    hipLaunchKernelGGL((split_pair_kernel<true, NP>), dim3((unsigned)(na + nb)), dim3(256), 0,
                       stream, a, b, na);
  else
    hipLaunchKernelGGL((split_pair_kernel<false, NP>), dim3((unsigned)(na + nb)), dim3(256), 0,
                       stream, a, b, na);
  return hipGetLastError();
}

hipError_t launch_split_pair(int np, int64_t m, int64_t n, int64_t k, const float *A, int64_t lda,
                             const float *B, int64_t ldb, uint16_t *const *ap, uint16_t *const *bp,
                             int64_t kp, int64_t ldp, hipStream_t stream) {
  if (m <= 0 || n <= 0 || k <= 0) return hipSuccess;
  if (np != 2 && np != 3) return hipErrorInvalidValue;
  if (kp % 8 != 0 || ldp % 8 != 0 || ldp < kp) return hipErrorInvalidValue;
  for (int p = 0; p < np; ++p)
    if (((uintptr_t)bp[p] % 16) || ((uintptr_t)ap[p] % 8)) return hipErrorInvalidValue;
  return np == 2 ? launch_pair<2>(m, n, k, A, lda, B, ldb, ap, bp, kp, ldp, stream)
                 : launch_pair<3>(m, n, k, A, lda, B, ldb, ap, bp, kp, ldp, stream);
}

template <int NP>
static hipError_t launch_one_split(int64_t rows, int64_t cols, const float *X, int64_t ldx,
                                   bool transpose, uint16_t *const *planes, int64_t ldo,
                                   int64_t out_pad, hipStream_t stream) {
  Planes<NP> out;
  bool aligned = true;
  for (int p = 0; p < NP; ++p) {
    out.p[p] = planes[p];
    aligned = aligned && ((uintptr_t)planes[p] % 8 == 0);
  }
  if (transpose) {
    const int64_t tiles = ((out_pad + 63) / 64) * ((cols + 63) / 64);
    if (tiles > 0x7fffffff) return hipErrorInvalidValue;
    hipLaunchKernelGGL((split_transpose_kernel<NP>), dim3((unsigned)tiles), dim3(256), 0, stream,
                       rows, cols, X, ldx, out, ldo, out_pad);
  } else {
    const bool vec = ((uintptr_t)X % 16 == 0) && (ldx % 4 == 0) && aligned && (ldo % 4 == 0);
    const int64_t work = rows * ((out_pad + 3) / 4);
    int64_t blocks = (work + 255) / 256;
    if (blocks > 65536) blocks = 65536;
    if (vec)
      hipLaunchKernelGGL((split_rows_kernel<true, NP>), dim3((unsigned)blocks), dim3(256), 0,
                         stream, rows, cols, X, ldx, out, ldo, out_pad);
    else
      hipLaunchKernelGGL((split_rows_kernel<false, NP>), dim3((unsigned)blocks), dim3(256), 0,
                         stream, rows, cols, X, ldx, out, ldo, out_pad);
  }
  return hipGetLastError();
}

hipError_t launch_split(int np, int64_t rows, int64_t cols, const float *X, int64_t ldx,
                        bool transpose, uint16_t *const *planes, int64_t ldo, int64_t out_pad,
                        hipStream_t stream) {
  if (rows <= 0 || cols <= 0) return hipSuccess;
  if (np == 2) return launch_one_split<2>(rows, cols, X, ldx, transpose, planes, ldo, out_pad, stream);
  if (np == 3) return launch_one_split<3>(rows, cols, X, ldx, transpose, planes, ldo, out_pad, stream);
  return hipErrorInvalidValue;
}

}  // namespace g355
