// kernels_grouped.hip -- one persistent launch for many independent products.
//
// The paper divides one product among workers by rows of A (Section 3.1.1,
// Algorithm 2). On one GPU the unit of work is an output tile instead: the
// host planner lists every tile of every problem, largest work first, each
// with the tile shape the tuned policy gives its size class; a persistent
// grid pulls items from that list through one atomic counter until it is
// exhausted. Every workgroup exits once the counter passes the item count.
#include "gemm_tile.hpp"
#include "internal.h"

namespace g355 {

using S128x128 = Shape<128, 128, 2, 2>;
using S128x64 = Shape<128, 64, 2, 2>;
using S64x64 = Shape<64, 64, 2, 2>;
using S32x32 = Shape<32, 32, 2, 2>;

template <int P> __host__ __device__ constexpr int grouped_lds() {
  // the largest configuration bounds the shared buffer
  return lds_bytes<P, S128x128>();
}

template <int P, class S>
__device__ __forceinline__ void run_item(const GemmArgs &g, const WorkItem &w, bool vec,
                                         char *smem) {
  if (vec)
    gemm_tile<P, S, false, false, true>(g, (int64_t)w.tm * S::BM, (int64_t)w.tn * S::BN, smem);
  else
    gemm_tile<P, S, false, false, false>(g, (int64_t)w.tm * S::BM, (int64_t)w.tn * S::BN, smem);
}

template <int P>
__global__ void __launch_bounds__(256)
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
      case CFG_128x128: run_item<P, S128x128>(g, w, pb.vec != 0, smem); break;
      case CFG_128x64: run_item<P, S128x64>(g, w, pb.vec != 0, smem); break;
      case CFG_64x64: run_item<P, S64x64>(g, w, pb.vec != 0, smem); break;
      default: run_item<P, S32x32>(g, w, pb.vec != 0, smem); break;
    }
  }
}

__global__ void counter_reset_kernel(uint32_t *counter) {
  if (threadIdx.x == 0 && blockIdx.x == 0) *counter = 0u;
}

hipError_t launch_counter_reset(uint32_t *counter, hipStream_t stream) {
  hipLaunchKernelGGL(counter_reset_kernel, dim3(1), dim3(64), 0, stream, counter);
  return hipGetLastError();
}

hipError_t launch_grouped(int prec, const GroupedProblem *probs, const WorkItem *items,
                          int32_t n_items, uint32_t *counter, int grid, hipStream_t stream) {
  if (grid <= 0) return hipSuccess;
  switch (prec) {
    case PREC_F64:
      hipLaunchKernelGGL(gemm_grouped_kernel<PREC_F64>, dim3(grid), dim3(256), 0, stream, probs,
                         items, n_items, counter);
      break;
    case PREC_F32:
      hipLaunchKernelGGL(gemm_grouped_kernel<PREC_F32>, dim3(grid), dim3(256), 0, stream, probs,
                         items, n_items, counter);
      break;
    default: return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

int grouped_max_grid(int prec) {
  int dev = 0, cus = 0, per = 0;
  if (hipGetDevice(&dev) != hipSuccess) return 0;
  if (hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess)
    return 0;
  hipError_t e = hipErrorInvalidValue;
  if (prec == PREC_F64)
    e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&per, gemm_grouped_kernel<PREC_F64>, 256, 0);
  else if (prec == PREC_F32)
    e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&per, gemm_grouped_kernel<PREC_F32>, 256, 0);
  if (e != hipSuccess || per <= 0) per = 1;
  return cus * per;
}

}  // namespace g355
