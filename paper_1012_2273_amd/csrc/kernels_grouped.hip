// kernels_grouped.hip -- one persistent launch for many independent products.
//
// The paper divides one product among workers by rows of A (Section 3.1.1,
// Algorithm 2). On one GPU the unit of work is an output tile instead: the
// host planner lists every tile of every problem, largest work first, each
// with the tile shape the tuned policy gives its size class; a persistent
// grid pulls items from that list through one atomic counter until it is
// exhausted. Every workgroup exits once the counter passes the item count.
#include "gemm_tile.hpp"
#include "gemm_tile_dma.hpp"
#include "internal.h"

namespace g355 {

// The grouped shapes: 512 threads, two waves per output position each
// taking half of every K-tile (the same shapes single launches offer under
// the same ids, so a problem's tiles are computed bit for bit as a single
// launch of that shape would compute them).
using G128x128 = Shape<128, 128, 2, 2, 2>;
using G128x64 = Shape<128, 64, 2, 2, 2>;
using G64x64 = Shape<64, 64, 2, 2, 2>;
using G32x32 = Shape<32, 32, 2, 2, 2>;
constexpr int GNT = 512;

template <int P, class S> __host__ __device__ constexpr int item_lds() {
  constexpr int reg = lds_bytes<P, S>();
  if constexpr (dma_ok<P, S, false, false>()) {
    constexpr int dma = lds_bytes_dma<P, S, false, false>();
    return dma > reg ? dma : reg;
  } else {
    return reg;
  }
}
template <int P> __host__ __device__ constexpr int grouped_lds() {
  constexpr int a = item_lds<P, G128x128>(), b = item_lds<P, G128x64>();
  constexpr int c = item_lds<P, G64x64>(), d = item_lds<P, G32x32>();
  constexpr int ab = a > b ? a : b, cd = c > d ? c : d;
  return ab > cd ? ab : cd;
}

// Same path choice as a single launch: direct-to-LDS when the operands allow
// 16-byte transfers and the shape's K-tile splits into whole 1 KiB transfers
// per loader wave, else registers.
// Problems with and without 16-byte operands go to two kernels (VEC), which
// keeps each kernel's register allocation to the paths it runs.
template <int P, class S, bool VEC>
__device__ __forceinline__ void run_item(const GemmArgs &g, const WorkItem &w, char *smem) {
  const int64_t m0 = (int64_t)w.tm * S::BM, n0 = (int64_t)w.tn * S::BN;
  if constexpr (VEC && dma_ok<P, S, false, false>())
    gemm_tile_dma<P, S, false, false>(g, m0, n0, smem);
  else
    gemm_tile<P, S, false, false, VEC ? 16 : 0>(g, m0, n0, smem);
}

template <int P, bool VEC>
__global__ void __launch_bounds__(GNT)
gemm_grouped_kernel(const GroupedProblem *__restrict__ probs, const WorkItem *__restrict__ items,
                    int32_t n_items, uint32_t *__restrict__ counter) {
  __shared__ __attribute__((aligned(16))) char smem[grouped_lds<P>()];
  __shared__ int32_t s_item;
  for (;;) {
    if (threadIdx.x == 0) s_item = (int32_t)atomicAdd(counter, 1u);
    __syncthreads();
    const int32_t it = s_item;
    __syncthreads();
    if (it >= n_items) break;
    const WorkItem w = items[it];
    const GroupedProblem pb = probs[w.prob];
    GemmArgs g;
    g.M = pb.M; g.N = pb.N; g.K = pb.K;
    g.A = pb.A; g.lda = pb.lda;
    g.B = pb.B; g.ldb = pb.ldb;
    g.A2 = nullptr; g.B2 = nullptr;
    g.C = pb.C; g.ldc = pb.ldc;
    switch (w.cfg) {
      case CFG_128x128_K2: run_item<P, G128x128, VEC>(g, w, smem); break;
      case CFG_128x64_K2: run_item<P, G128x64, VEC>(g, w, smem); break;
      case CFG_64x64_K2: run_item<P, G64x64, VEC>(g, w, smem); break;
      default: run_item<P, G32x32, VEC>(g, w, smem); break;
    }
    __syncthreads();   // the next item's prologue reuses the LDS
  }
}

__global__ void counter_reset_kernel(uint32_t *counter) {
  if (threadIdx.x == 0 && blockIdx.x == 0) {
    counter[0] = 0u;
    counter[kCounterStride] = 0u;
  }
}

hipError_t launch_counter_reset(uint32_t *counter, hipStream_t stream) {
  hipLaunchKernelGGL(counter_reset_kernel, dim3(1), dim3(64), 0, stream, counter);
  return hipGetLastError();
}

template <int P>
static hipError_t launch_pair(const GroupedProblem *probs, const WorkItem *items, int32_t n_vec,
                              int32_t n_scalar, uint32_t *counter, int grid, hipStream_t stream) {
  if (n_vec > 0) {
    hipLaunchKernelGGL((gemm_grouped_kernel<P, true>), dim3(grid), dim3(GNT), 0, stream, probs,
                       items, n_vec, counter);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
  }
  if (n_scalar > 0) {
    hipLaunchKernelGGL((gemm_grouped_kernel<P, false>), dim3(grid), dim3(GNT), 0, stream, probs,
                       items + n_vec, n_scalar, counter + kCounterStride);
    return hipGetLastError();
  }
  return hipSuccess;
}

hipError_t launch_grouped(int prec, const GroupedProblem *probs, const WorkItem *items,
                          int32_t n_vec, int32_t n_scalar, uint32_t *counter, int grid,
                          hipStream_t stream) {
  if (grid <= 0) return hipSuccess;
  switch (prec) {
    case PREC_F64:
      return launch_pair<PREC_F64>(probs, items, n_vec, n_scalar, counter, grid, stream);
    case PREC_F32:
      return launch_pair<PREC_F32>(probs, items, n_vec, n_scalar, counter, grid, stream);
  }
  return hipErrorInvalidValue;
}

int grouped_max_grid(int prec) {
  int dev = 0, cus = 0, per = 0;
  if (hipGetDevice(&dev) != hipSuccess) return 0;
  if (hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess)
    return 0;
  // the two kernels may differ; size the grid for the one fewer fit
  int per2 = 0;
  hipError_t e = hipErrorInvalidValue, e2 = hipErrorInvalidValue;
  if (prec == PREC_F64) {
    e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&per, gemm_grouped_kernel<PREC_F64, true>, GNT, 0);
    e2 = hipOccupancyMaxActiveBlocksPerMultiprocessor(&per2, gemm_grouped_kernel<PREC_F64, false>, GNT, 0);
  } else if (prec == PREC_F32) {
    e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&per, gemm_grouped_kernel<PREC_F32, true>, GNT, 0);
    e2 = hipOccupancyMaxActiveBlocksPerMultiprocessor(&per2, gemm_grouped_kernel<PREC_F32, false>, GNT, 0);
  }
  if (e != hipSuccess || e2 != hipSuccess) return cus;
  per = per < per2 ? per : per2;
  if (per <= 0) per = 1;
  return cus * per;
}

}  // namespace g355
