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

// K split over workgroups: blockIdx.y takes K-indices [y kc, (y + 1) kc) of
// the product; chunk 0 writes its partial product to C, chunk y > 0 to plane
// y - 1 of the workspace (M x N, row pitch N). kc is a multiple of every
// K-tile depth and of 16 bytes, so only the last chunk has a ragged K-tile
// and every chunk's operand base keeps the alignment of the whole operand.
template <int P, class S, bool TA, bool TB, int VW>
__global__ void __launch_bounds__(S::NT)
gemm_ksplit_kernel(GemmArgs g, int tiles_m, int tiles_n, int group_m, int64_t kc, void *ws) {
  using E = typename Traits<P>::E;
  using O = typename Traits<P>::Out;
  constexpr bool DMA = VW == 16 && dma_ok<P, S, TA, TB>();
  __shared__ __attribute__((aligned(16))) char smem[DMA ? lds_bytes_dma<P, S, TA, TB>()
                                                        : lds_bytes<P, S>()];
  const int64_t y = blockIdx.y, k0 = y * kc;
  g.A = (const E *)g.A + k0 * (TA ? g.lda : 1);
  g.B = (const E *)g.B + k0 * (TB ? 1 : g.ldb);
  g.K = g.K - k0 < kc ? g.K - k0 : kc;
  if (y > 0) {
    g.C = (O *)ws + (y - 1) * g.M * g.N;
    g.ldc = g.N;
  }
  int tm, tn;
  tile_of(blockIdx.x, gridDim.x, tiles_m, tiles_n, group_m, tm, tn);
  if constexpr (DMA)
    gemm_tile_dma<P, S, TA, TB>(g, (int64_t)tm * S::BM, (int64_t)tn * S::BN, smem);
  else
    gemm_tile<P, S, TA, TB, VW>(g, (int64_t)tm * S::BM, (int64_t)tn * S::BN, smem);
}

// C += plane 0 + plane 1 + ... + plane (parts - 1), added in that order
// (the K chunks' order), one thread per output column, rows strided over
// blockIdx.y. The planes are loaded eight at a time before they are added,
// so eight loads per lane are in flight (one at a time left the kernel
// latency-bound at a fifth of HBM bandwidth); the additions keep their order.
template <class O>
__global__ void __launch_bounds__(256)
ksplit_sum_kernel(O *C, int64_t ldc, const O *W, int64_t m, int64_t n, int parts) {
  const int64_t c = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (c >= n) return;
  const int64_t mn = m * n;
  for (int64_t r = blockIdx.y; r < m; r += gridDim.y) {
    const O *w = W + r * n + c;
    O acc = C[r * ldc + c];
    int p = 0;
    for (; p + 8 <= parts; p += 8) {
      O v[8];
#pragma unroll
      for (int j = 0; j < 8; ++j) v[j] = w[(int64_t)(p + j) * mn];
#pragma unroll
      for (int j = 0; j < 8; ++j) acc += v[j];
    }
    for (; p < parts; ++p) acc += w[(int64_t)p * mn];
    C[r * ldc + c] = acc;
  }
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
  if constexpr (P == PREC_LSPLIT || P == PREC_LSPLIT3) {
    // binary32 operands as given (NN, 16-byte rows), split by the loader
    // waves: shapes with loader waves only
    if constexpr (S::LDW == 0 || S::KS != 2) {
      return -1;
    } else {
      if (layout != LAYOUT_NN || vw != 16) return -1;
      if constexpr (dma_ok<P, S, false, false>()) return f(KTag<P, S, false, false, 16>{});
      return -1;
    }
  } else if constexpr (S::LDW > 0 && (P == PREC_SPLIT || P == PREC_SPLIT3)) {
    // shapes with loader waves exist on the direct-to-LDS path only
    if (layout != LAYOUT_NT || vw != 16) return -1;
    if constexpr (dma_ok<P, S, false, true>()) return f(KTag<P, S, false, true, 16>{});
    return -1;
  } else if constexpr (S::LDW > 0 && (P == PREC_FSPLIT || P == PREC_FSPLIT3)) {
    if (layout != LAYOUT_NN || vw != 16) return -1;
    if constexpr (dma_ok<P, S, false, false>()) return f(KTag<P, S, false, false, 16>{});
    return -1;
  } else if constexpr ((P == PREC_BF16 && S::KS > 1) || S::LDW > 0 || S::BM * S::BN >= 256 * 256) {
    // 16-bit K-split tiles exist on the direct-to-LDS path only (64-deep
    // K-tiles; the register path's 32-deep tiles do not split), and so do
    // the shapes with loader waves and the 256 x 256 tile
    if (vw != 16) return -1;
    switch (layout) {
      case LAYOUT_NN:
        if constexpr (dma_ok<P, S, false, false>()) return f(KTag<P, S, false, false, 16>{});
        return -1;
      case LAYOUT_NT:
        if constexpr (dma_ok<P, S, false, true>()) return f(KTag<P, S, false, true, 16>{});
        return -1;
      case LAYOUT_TN:
        if constexpr (dma_ok<P, S, true, false>()) return f(KTag<P, S, true, false, 16>{});
        return -1;
    }
    return -1;
  } else if constexpr (!shape_ok<P, S>()) {
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
using S256x256w8 = Shape<256, 256, 2, 4, 1, 32>;
#ifndef G355_LDW
#define G355_LDW 4
#endif
#ifndef G355_LD_SHAPE
#define G355_LD_SHAPE 128, 128, 2, 2, 2, 0, G355_LDW
#endif
using S128x128k2ld = Shape<G355_LD_SHAPE>;   // + loader waves

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
    case CFG_128x128_K2_LD: return by_layout<P, S128x128k2ld>(layout, vw, f);
    case CFG_128x256_W8:
      if constexpr (P == PREC_BF16 || P == PREC_SPLIT || P == PREC_SPLIT3 || P == PREC_FSPLIT ||
                    P == PREC_FSPLIT3 || P == PREC_LSPLIT || P == PREC_LSPLIT3)
        return by_layout<P, S128x256w8>(layout, vw, f);
      else
        return -1;   // bfloat16-MFMA products only (the host never picks it)
    case CFG_256x256_W8:
      // bf16 and the two-way split (whose three planes would not leave two
      // stages of the ring: the three-way products stay off it, in both forms)
      if constexpr (P == PREC_BF16 || P == PREC_SPLIT || P == PREC_FSPLIT)
        return by_layout<P, S256x256w8>(layout, vw, f);
      else
        return -1;
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
    case PREC_LSPLIT: return by_cfg<PREC_LSPLIT>(layout, cfg, vw, f);
    case PREC_LSPLIT3: return by_cfg<PREC_LSPLIT3>(layout, cfg, vw, f);
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

// The K split is instantiated for NN products of the plain precisions on
// the shapes that hold one or two workgroups per CU.
template <int P, class S, bool TA, bool TB> constexpr bool ksplit_offered() {
  return (P == PREC_F64 || P == PREC_F32 || P == PREC_BF16) && !TA && !TB &&
         (std::is_same_v<S, S128x128> || std::is_same_v<S, S128x128w8> ||
          std::is_same_v<S, S128x64> || std::is_same_v<S, S64x64>);
}

bool ksplit_offered(int prec, int layout, int cfg, int vw) {
  auto f = []<int P, class S, bool TA, bool TB, int VW>(KTag<P, S, TA, TB, VW>) -> int {
    return ksplit_offered<P, S, TA, TB>() ? 0 : -1;
  };
  return visit(prec, layout, cfg, vw, f) >= 0;
}

hipError_t launch_ksplit(int prec, int layout, int cfg, int vw, const GemmArgs &a, int parts,
                         int64_t kc, void *ws, hipStream_t stream) {
  auto f = [&]<int P, class S, bool TA, bool TB, int VW>(KTag<P, S, TA, TB, VW>) -> int {
    if constexpr (!ksplit_offered<P, S, TA, TB>()) {
      return -1;
    } else {
      const int64_t tiles_m = (a.M + S::BM - 1) / S::BM;
      const int64_t tiles_n = (a.N + S::BN - 1) / S::BN;
      const int64_t tiles = tiles_m * tiles_n;
      if (tiles <= 0 || parts < 1) return (int)hipSuccess;
      if (tiles > 0x7fffffff || parts > 65535) return (int)hipErrorInvalidValue;
      hipLaunchKernelGGL((gemm_ksplit_kernel<P, S, TA, TB, VW>), dim3((unsigned)tiles, (unsigned)parts),
                         dim3(S::NT), 0, stream, a, (int)tiles_m, (int)tiles_n, 4, kc, ws);
      return (int)hipGetLastError();
    }
  };
  const int r = visit(prec, layout, cfg, vw, f);
  return r < 0 ? hipErrorInvalidValue : (hipError_t)r;
}

hipError_t launch_ksplit_sum(int prec, void *C, int64_t ldc, const void *W, int64_t m, int64_t n,
                             int parts, hipStream_t stream) {
  if (m <= 0 || n <= 0 || parts <= 0) return hipSuccess;
  const int64_t gx = (n + 255) / 256, gy = m < 4096 ? m : 4096;
  if (gx > 0x7fffffff) return hipErrorInvalidValue;
  const dim3 grid((unsigned)gx, (unsigned)gy);
  if (prec == PREC_F64)
    hipLaunchKernelGGL(ksplit_sum_kernel<double>, grid, dim3(256), 0, stream, (double *)C, ldc,
                       (const double *)W, m, n, parts);
  else
    hipLaunchKernelGGL(ksplit_sum_kernel<float>, grid, dim3(256), 0, stream, (float *)C, ldc,
                       (const float *)W, m, n, parts);
  return hipGetLastError();
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
