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
// taking half of every K-tile, and the 8-wave 128 x 128 tile (the same
// shapes single launches offer under the same ids, so a problem's tiles are
// computed bit for bit as a single launch of that shape would compute them).
using G128x128 = Shape<128, 128, 2, 2, 2>;
using G128x64 = Shape<128, 64, 2, 2, 2>;
using G64x64 = Shape<64, 64, 2, 2, 2>;
using G32x32 = Shape<32, 32, 2, 2, 2>;
using G128x128w8 = Shape<128, 128, 4, 2, 1>;
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
  constexpr int e = item_lds<P, G128x128w8>();
  constexpr int ab = a > b ? a : b, cd = c > d ? c : d, abcd = ab > cd ? ab : cd;
  return abcd > e ? abcd : e;
}

// Same path choice as a single launch: direct-to-LDS when the operands allow
// 16-byte transfers and the shape's K-tile splits into whole 1 KiB transfers
// per loader wave, else registers.
// Problems with 16-byte operands (their own, or the plan's packed copies)
// and the rest run in different kernels (VEC), which keeps each kernel's
// register allocation to the paths it runs.
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
      case CFG_128x128_W8: run_item<P, G128x128w8, VEC>(g, w, smem); break;
      default: run_item<P, G32x32, VEC>(g, w, smem); break;
    }
    __syncthreads();   // the next item's prologue reuses the LDS
  }
}

__global__ void counter_reset_kernel(uint32_t *counter) {
  if (threadIdx.x < kQueues && blockIdx.x == 0) counter[threadIdx.x * kCounterStride] = 0u;
}

hipError_t launch_counter_reset(uint32_t *counter, hipStream_t stream) {
  hipLaunchKernelGGL(counter_reset_kernel, dim3(1), dim3(64), 0, stream, counter);
  return hipGetLastError();
}

hipError_t launch_grouped(int prec, bool vec, const GroupedProblem *probs, const WorkItem *items,
                          int32_t n_items, uint32_t *counter, int grid, hipStream_t stream) {
  if (grid <= 0 || n_items <= 0) return hipSuccess;
  const dim3 g(grid), b(GNT);
  if (prec == PREC_F64 && vec)
    hipLaunchKernelGGL((gemm_grouped_kernel<PREC_F64, true>), g, b, 0, stream, probs, items, n_items, counter);
  else if (prec == PREC_F64)
    hipLaunchKernelGGL((gemm_grouped_kernel<PREC_F64, false>), g, b, 0, stream, probs, items, n_items, counter);
  else if (prec == PREC_F32 && vec)
    hipLaunchKernelGGL((gemm_grouped_kernel<PREC_F32, true>), g, b, 0, stream, probs, items, n_items, counter);
  else if (prec == PREC_F32)
    hipLaunchKernelGGL((gemm_grouped_kernel<PREC_F32, false>), g, b, 0, stream, probs, items, n_items, counter);
  else
    return hipErrorInvalidValue;
  return hipGetLastError();
}

// The operand copy that lets a problem whose rows are not 16-byte multiples
// use the direct-to-LDS kernel. Block b copies kPackRows destination rows of
// one job (found by binary search over the jobs' first blocks); a grid
// smaller than the block count walks the blocks in strides. Each wave copies
// whole rows: lane l gathers the V elements of 16-byte destination vectors
// l, l + 64, ... with element loads (a wave reads 64 V consecutive elements)
// and stores each vector at once. Memory-bound: rows * cols elements read,
// drows * dcols written per job.
template <typename E>
__global__ void __launch_bounds__(256)
pack_kernel(const PackJob *__restrict__ jobs, int32_t n_jobs, int64_t nblocks) {
  constexpr int V = 16 / (int)sizeof(E);
  typedef E Vec __attribute__((ext_vector_type(V)));
  const int wave = (int)(threadIdx.x / 64), lane = (int)(threadIdx.x % 64);
  for (int64_t b = blockIdx.x; b < nblocks; b += gridDim.x) {
    int32_t lo = 0, hi = n_jobs - 1;
    while (lo < hi) {
      const int32_t mid = (lo + hi + 1) / 2;
      if (jobs[mid].first_block <= b) lo = mid; else hi = mid - 1;
    }
    const PackJob j = jobs[lo];
    const int64_t r0 = (b - j.first_block) * kPackRows;
    for (int rr = wave; rr < kPackRows && r0 + rr < j.drows; rr += 4) {
      const int64_t r = r0 + rr;
      const bool in = r < j.rows;
      const E *s = reinterpret_cast<const E *>(j.src) + (in ? r * j.sld : 0);
      E *d = reinterpret_cast<E *>(j.dst) + r * j.dld;
      for (int64_t c = (int64_t)lane * V; c < j.dcols; c += 64 * V) {
        Vec v;
#pragma unroll
        for (int e = 0; e < V; ++e) v[e] = (in && c + e < j.cols) ? s[c + e] : (E)0;
        *reinterpret_cast<Vec *>(d + c) = v;
      }
    }
  }
}

hipError_t launch_pack(int prec, const PackJob *jobs, int32_t n_jobs, int64_t blocks, int grid,
                       hipStream_t stream) {
  if (n_jobs <= 0 || blocks <= 0) return hipSuccess;
  const int64_t g = grid <= 0 || grid > blocks ? blocks : grid;
  if (g > 0x7fffffffLL) return hipErrorInvalidValue;
  if (prec == PREC_F64)
    hipLaunchKernelGGL(pack_kernel<double>, dim3((uint32_t)g), dim3(256), 0, stream, jobs,
                       n_jobs, blocks);
  else if (prec == PREC_F32)
    hipLaunchKernelGGL(pack_kernel<float>, dim3((uint32_t)g), dim3(256), 0, stream, jobs,
                       n_jobs, blocks);
  else
    return hipErrorInvalidValue;
  return hipGetLastError();
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
