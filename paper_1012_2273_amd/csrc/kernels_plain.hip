// kernels_plain.hip -- single-product kernels: one workgroup per output tile.
#include "gemm_tile.hpp"
#include "gemm_tile_dma.hpp"
#include "internal.h"

namespace g355 {

template <int P, class S, bool TA, bool TB, int VW>
__global__ void __launch_bounds__(S::NT)
gemm_plain_kernel(GemmArgs g, int tiles_m, int tiles_n, int group_m) {
  __shared__ __attribute__((aligned(16))) char smem[lds_bytes<P, S>()];
  int tm, tn;
  tile_of(blockIdx.x, gridDim.x, tiles_m, tiles_n, group_m, tm, tn);
  gemm_tile<P, S, TA, TB, VW>(g, (int64_t)tm * S::BM, (int64_t)tn * S::BN, smem);
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

template <int P, class S, bool TA, bool TB, int VW>
static hipError_t launch_one(const GemmArgs &a, hipStream_t stream) {
  const int64_t tiles_m = (a.M + S::BM - 1) / S::BM;
  const int64_t tiles_n = (a.N + S::BN - 1) / S::BN;
  const int64_t tiles = tiles_m * tiles_n;
  if (tiles <= 0) return hipSuccess;
  if (tiles > 0x7fffffff) return hipErrorInvalidValue;
  // 4 tile rows per raster group keeps an XCD's tiles within few rows of A
  const int group_m = 4;
  if constexpr (VW == 16 && dma_ok<P, S, TA, TB>()) {
    hipLaunchKernelGGL((gemm_plain_dma_kernel<P, S, TA, TB>), dim3((unsigned)tiles), dim3(S::NT),
                       0, stream, a, (int)tiles_m, (int)tiles_n, group_m);
  } else {
    hipLaunchKernelGGL((gemm_plain_kernel<P, S, TA, TB, VW>), dim3((unsigned)tiles), dim3(S::NT),
                       0, stream, a, (int)tiles_m, (int)tiles_n, group_m);
  }
  return hipGetLastError();
}

// One instantiation of the single-product kernel pair (precision, shape,
// operand layout, vector width in bytes), handed to a visitor.
template <int P, class S, bool TA, bool TB, int VW> struct KTag {};

template <int P, class S, bool TA, bool TB, int VW> static int occupancy_one() {
  int per = 0;
  hipError_t e;
  if constexpr (VW == 16 && dma_ok<P, S, TA, TB>())
    e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&per, gemm_plain_dma_kernel<P, S, TA, TB>, S::NT, 0);
  else
    e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&per, gemm_plain_kernel<P, S, TA, TB, VW>, S::NT, 0);
  return e == hipSuccess ? per : 0;
}

// Visitors return an int >= 0, or -1 for a combination that is not offered.
// vw: the widest vector loads the operands allow (16 or 8 bytes, 0 for
// elements); 8-byte vectors are instantiated for 2- and 4-byte elements only.
template <int P, class S, bool TA, bool TB, class F> static int by_width(int vw, F &f) {
  if (vw == 16) return f(KTag<P, S, TA, TB, 16>{});
  if constexpr (sizeof(typename Traits<P>::E) < 8) {
    if (vw == 8) return f(KTag<P, S, TA, TB, 8>{});
  }
  return f(KTag<P, S, TA, TB, 0>{});
}

template <int P, class S, class F> static int by_layout(int layout, int vw, F &f) {
  if constexpr (!shape_ok<P, S>()) {
    return -1;   // not offered for this precision (the host never picks it)
  } else if constexpr (P == PREC_SPLIT || P == PREC_SPLIT3) {
    // the split planes are always written K-contiguous and 16-byte aligned
    if (layout != LAYOUT_NT || vw != 16) return -1;
    return f(KTag<P, S, false, true, 16>{});
  } else if constexpr (P == PREC_FSPLIT || P == PREC_FSPLIT3) {
    // binary32 operands as given, direct-to-LDS only (the caller falls back
    // to the split step and the plane product otherwise)
    if constexpr (!dma_ok<P, S, false, false>()) {
      return -1;
    } else {
      if (layout != LAYOUT_NN || vw != 16) return -1;
      return f(KTag<P, S, false, false, 16>{});
    }
  } else {
    switch (layout) {
      case LAYOUT_NN: return by_width<P, S, false, false>(vw, f);
      case LAYOUT_NT: return by_width<P, S, false, true>(vw, f);
      case LAYOUT_TN: return by_width<P, S, true, false>(vw, f);
    }
    return -1;
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
using S64x64k4 = Shape<64, 64, 2, 2, 4, 32>;   // 1024 threads
using S128x256w8 = Shape<128, 256, 2, 4, 1, 32>;

template <int P, class F> static int by_cfg(int layout, int cfg, int vw, F &f) {
  switch (cfg) {
    case CFG_128x128: return by_layout<P, S128x128>(layout, vw, f);
    case CFG_128x64: return by_layout<P, S128x64>(layout, vw, f);
    case CFG_64x64: return by_layout<P, S64x64>(layout, vw, f);
    case CFG_32x32: return by_layout<P, S32x32>(layout, vw, f);
    case CFG_128x128_W8: return by_layout<P, S128x128w8>(layout, vw, f);
    case CFG_128x128_K2: return by_layout<P, S128x128k2>(layout, vw, f);
    case CFG_128x64_K2: return by_layout<P, S128x64k2>(layout, vw, f);
    case CFG_64x64_K2: return by_layout<P, S64x64k2>(layout, vw, f);
    case CFG_32x32_K2: return by_layout<P, S32x32k2>(layout, vw, f);
    case CFG_64x64_K4:
      if constexpr (P == PREC_F64)
        return by_layout<P, S64x64k4>(layout, vw, f);
      else
        return -1;   // binary64 only (the host never picks it)
    case CFG_128x256_W8:
      if constexpr (P == PREC_BF16 || P == PREC_SPLIT || P == PREC_SPLIT3 || P == PREC_FSPLIT ||
                    P == PREC_FSPLIT3)
        return by_layout<P, S128x256w8>(layout, vw, f);
      else
        return -1;   // bfloat16-MFMA products only (the host never picks it)
  }
  return -1;
}

template <class F> static int visit(int prec, int layout, int cfg, int vw, F &f) {
  switch (prec) {
    case PREC_F64: return by_cfg<PREC_F64>(layout, cfg, vw, f);
    case PREC_F32: return by_cfg<PREC_F32>(layout, cfg, vw, f);
    case PREC_BF16: return by_cfg<PREC_BF16>(layout, cfg, vw, f);
    case PREC_SPLIT: return by_cfg<PREC_SPLIT>(layout, cfg, vw, f);
    case PREC_SPLIT3: return by_cfg<PREC_SPLIT3>(layout, cfg, vw, f);
    case PREC_FSPLIT: return by_cfg<PREC_FSPLIT>(layout, cfg, vw, f);
    case PREC_FSPLIT3: return by_cfg<PREC_FSPLIT3>(layout, cfg, vw, f);
  }
  return -1;
}

hipError_t launch_plain(int prec, int layout, int cfg, int vw, const GemmArgs &a,
                        hipStream_t stream) {
  auto f = [&]<int P, class S, bool TA, bool TB, int VW>(KTag<P, S, TA, TB, VW>) -> int {
    return (int)launch_one<P, S, TA, TB, VW>(a, stream);
  };
  const int r = visit(prec, layout, cfg, vw, f);
  return r < 0 ? hipErrorInvalidValue : (hipError_t)r;
}

int plain_occupancy(int prec, int layout, int cfg, int vw) {
  auto f = []<int P, class S, bool TA, bool TB, int VW>(KTag<P, S, TA, TB, VW>) -> int {
    return occupancy_one<P, S, TA, TB, VW>();
  };
  const int r = visit(prec, layout, cfg, vw, f);
  return r < 0 ? 0 : r;
}

bool plain_offered(int prec, int layout, int cfg, int vw) {
  auto f = []<int P, class S, bool TA, bool TB, int VW>(KTag<P, S, TA, TB, VW>) -> int { return 0; };
  return visit(prec, layout, cfg, vw, f) >= 0;
}

}  // namespace g355
