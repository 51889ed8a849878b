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
