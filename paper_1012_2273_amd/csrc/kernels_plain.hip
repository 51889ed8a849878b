// kernels_plain.hip -- single-product kernels: one workgroup per output tile.
#include "gemm_tile.hpp"
#include "gemm_tile_dma.hpp"
#include "internal.h"

namespace g355 {

template <int P, class S, bool TA, bool TB, bool VEC>
__global__ void __launch_bounds__(S::NT)
gemm_plain_kernel(GemmArgs g, int tiles_m, int tiles_n, int group_m) {
  __shared__ __attribute__((aligned(16))) char smem[lds_bytes<P, S>()];
  int tm, tn;
  tile_of(blockIdx.x, gridDim.x, tiles_m, tiles_n, group_m, tm, tn);
  gemm_tile<P, S, TA, TB, VEC>(g, (int64_t)tm * S::BM, (int64_t)tn * S::BN, smem);
}

// Direct-to-LDS variant (16-byte aligned operands, shapes that split evenly
// into 1 KiB transfers per wave).
template <int P, class S, bool TA, bool TB>
__global__ void __launch_bounds__(S::NT)
gemm_plain_dma_kernel(GemmArgs g, int tiles_m, int tiles_n, int group_m) {
  __shared__ __attribute__((aligned(16))) char smem[lds_bytes_dma<P, S, TA, TB>()];
  int tm, tn;
  tile_of(blockIdx.x, gridDim.x, tiles_m, tiles_n, group_m, tm, tn);
  gemm_tile_dma<P, S, TA, TB>(g, (int64_t)tm * S::BM, (int64_t)tn * S::BN, smem);
}

template <int P, class S, bool TA, bool TB, bool VEC>
static hipError_t launch_one(const GemmArgs &a, hipStream_t stream) {
  const int64_t tiles_m = (a.M + S::BM - 1) / S::BM;
  const int64_t tiles_n = (a.N + S::BN - 1) / S::BN;
  const int64_t tiles = tiles_m * tiles_n;
  if (tiles <= 0) return hipSuccess;
  if (tiles > 0x7fffffff) return hipErrorInvalidValue;
  // 4 tile rows per raster group keeps an XCD's tiles within few rows of A
  const int group_m = 4;
  if constexpr (VEC && dma_ok<P, S, TA, TB>()) {
    hipLaunchKernelGGL((gemm_plain_dma_kernel<P, S, TA, TB>), dim3((unsigned)tiles), dim3(S::NT),
                       0, stream, a, (int)tiles_m, (int)tiles_n, group_m);
  } else {
    hipLaunchKernelGGL((gemm_plain_kernel<P, S, TA, TB, VEC>), dim3((unsigned)tiles), dim3(S::NT),
                       0, stream, a, (int)tiles_m, (int)tiles_n, group_m);
  }
  return hipGetLastError();
}

template <int P, class S, bool TA, bool TB>
static hipError_t by_vec(bool vec, const GemmArgs &a, hipStream_t s) {
  return vec ? launch_one<P, S, TA, TB, true>(a, s) : launch_one<P, S, TA, TB, false>(a, s);
}

template <int P, class S>
static hipError_t by_layout(int layout, bool vec, const GemmArgs &a, hipStream_t s) {
  if constexpr (!shape_ok<P, S>()) {
    return hipErrorInvalidValue;   // not offered for this precision (the host never picks it)
  } else if constexpr (P == PREC_SPLIT) {
    // the split planes are always written K-contiguous and 16-byte aligned
    if (layout != LAYOUT_NT || !vec) return hipErrorInvalidValue;
    return launch_one<P, S, false, true, true>(a, s);
  } else {
    switch (layout) {
      case LAYOUT_NN: return by_vec<P, S, false, false>(vec, a, s);
      case LAYOUT_NT: return by_vec<P, S, false, true>(vec, a, s);
      case LAYOUT_TN: return by_vec<P, S, true, false>(vec, a, s);
    }
    return hipErrorInvalidValue;
  }
}

using S128x128 = Shape<128, 128, 2, 2>;
using S128x64 = Shape<128, 64, 2, 2>;
using S64x64 = Shape<64, 64, 2, 2>;
using S32x32 = Shape<32, 32, 2, 2>;
using S128x128w8 = Shape<128, 128, 4, 2>;
using S128x128k2 = Shape<128, 128, 2, 2, 2>;
using S128x64k2 = Shape<128, 64, 2, 2, 2>;
using S64x64k2 = Shape<64, 64, 2, 2, 2>;
using S32x32k2 = Shape<32, 32, 2, 2, 2>;
using S128x256w8 = Shape<128, 256, 2, 4, 1, 32>;

template <int P>
static hipError_t by_cfg(int layout, int cfg, bool vec, const GemmArgs &a, hipStream_t s) {
  switch (cfg) {
    case CFG_128x128: return by_layout<P, S128x128>(layout, vec, a, s);
    case CFG_128x64: return by_layout<P, S128x64>(layout, vec, a, s);
    case CFG_64x64: return by_layout<P, S64x64>(layout, vec, a, s);
    case CFG_32x32: return by_layout<P, S32x32>(layout, vec, a, s);
    case CFG_128x128_W8: return by_layout<P, S128x128w8>(layout, vec, a, s);
    case CFG_128x128_K2: return by_layout<P, S128x128k2>(layout, vec, a, s);
    case CFG_128x64_K2: return by_layout<P, S128x64k2>(layout, vec, a, s);
    case CFG_64x64_K2: return by_layout<P, S64x64k2>(layout, vec, a, s);
    case CFG_32x32_K2: return by_layout<P, S32x32k2>(layout, vec, a, s);
    case CFG_128x256_W8:
      if constexpr (P == PREC_BF16 || P == PREC_SPLIT) {
        return by_layout<P, S128x256w8>(layout, vec, a, s);
      } else {
        return hipErrorInvalidValue;   // 16-bit only (the host never picks it)
      }
  }
  return hipErrorInvalidValue;
}

hipError_t launch_plain(int prec, int layout, int cfg, bool vec, const GemmArgs &a,
                        hipStream_t stream) {
  switch (prec) {
    case PREC_F64: return by_cfg<PREC_F64>(layout, cfg, vec, a, stream);
    case PREC_F32: return by_cfg<PREC_F32>(layout, cfg, vec, a, stream);
    case PREC_BF16: return by_cfg<PREC_BF16>(layout, cfg, vec, a, stream);
    case PREC_SPLIT: return by_cfg<PREC_SPLIT>(layout, cfg, vec, a, stream);
  }
  return hipErrorInvalidValue;
}

}  // namespace g355
