// internal.h -- host-side declarations shared by the library's translation
// units (not part of the public ABI).
#pragma once

#include <hip/hip_runtime.h>
#include <stddef.h>
#include <stdint.h>

#include <string>

namespace g355 {

struct GemmArgs;

// Tile configurations the kernels are instantiated for; the id is the
// value the tuner and the grouped planner store. The K-split ones (512 threads: two waves per output
// position, each taking half of every K-tile) are the ones the persistent
// grouped kernel offers; every configuration runs as a single product.
// 128x256w8 is offered to the bfloat16-MFMA products only (8 waves of 64 x 64
// outputs with 32-deep K-tiles, 25% fewer operand bytes per flop than
// 128 x 128); 64x64k4 to binary64 only (16 waves: four per output position,
// each taking a quarter of every 32-deep K-tile). 128x128k2ld is 128x128k2
// plus loader waves that issue every operand transfer (direct-to-LDS only).
// 256x256w8 (8 waves of 128 x 64 outputs, 32-deep K-tiles, direct-to-LDS
// only) is offered to the bfloat16-MFMA products: a third fewer operand
// bytes per flop than 128 x 256.
enum TileCfg : int {
  CFG_128x128 = 0, CFG_128x64 = 1, CFG_64x64 = 2, CFG_32x32 = 3,
  CFG_128x128_W8 = 4, CFG_128x128_K2 = 5, CFG_128x64_K2 = 6, CFG_64x64_K2 = 7,
  CFG_32x32_K2 = 8, CFG_128x256_W8 = 9, CFG_64x64_K4 = 10, CFG_128x128_K2_LD = 11,
  CFG_256x256_W8 = 12, CFG_COUNT = 13
};
constexpr int kGroupedCfgs[5] = {CFG_128x128_K2, CFG_128x64_K2, CFG_64x64_K2, CFG_32x32_K2,
                                 CFG_128x128_W8};
bool cfg_grouped(int cfg);
struct CfgInfo { int bm, bn; const char *name; };
const CfgInfo &cfg_info(int id);
bool cfg_supported(int prec, int cfg);

// Operand layout of one launch: TA -> op(A) = A^T stored K x M;
// TB -> op(B) = B^T stored N x K.
enum Layout : int { LAYOUT_NN = 0, LAYOUT_NT = 1, LAYOUT_TN = 2 };

// Launch one single-product kernel (grid = all tiles of C).
// prec: a Prec value (gemm_tile.hpp). Returns hipSuccess or the launch error.
hipError_t launch_plain(int prec, int layout, int cfg, int vw, const GemmArgs &a,
                        hipStream_t stream);
// Workgroups of that kernel one CU holds at once (0 if not offered or unknown).
int plain_occupancy(int prec, int layout, int cfg, int vw);
// Whether a kernel exists for that combination.
bool plain_offered(int prec, int layout, int cfg, int vw);
// K split over workgroups (binary64, binary32, bf16): `parts` chunks of kc
// K-indices, chunk 0 into C, chunk y > 0 into plane y - 1 of ws (M x N
// outputs each, row pitch N); then C += the planes in chunk order.
bool ksplit_offered(int prec, int layout, int cfg, int vw);
hipError_t launch_ksplit(int prec, int layout, int cfg, int vw, const GemmArgs &a, int parts,
                         int64_t kc, void *ws, hipStream_t stream);
hipError_t launch_ksplit_sum(int prec, void *C, int64_t ldc, const void *W, int64_t m, int64_t n,
                             int parts, hipStream_t stream);

// Split kernels (np = 2: hi, lo; np = 3: hi, mid, lo). X (rows x cols, ldx)
// -> np 16-bit planes. Plane rows are written up to `out_pad` >= their
// length (cols, or rows when transposed), the padding with zeros.
hipError_t launch_split(int np, int64_t rows, int64_t cols, const float *X, int64_t ldx,
                        bool transpose, uint16_t *const *planes, int64_t ldo, int64_t out_pad,
                        hipStream_t stream);

// Both operands of a split product in one launch: A (m x k) -> row-major
// planes (m x kp), B (k x n) -> transposed planes (n x kp), at row pitch
// ldp; kp a multiple of 8, padding zeroed, plane rows 16-byte aligned.
hipError_t launch_split_pair(int np, int64_t m, int64_t n, int64_t k, const float *A, int64_t lda,
                             const float *B, int64_t ldb, uint16_t *const *ap, uint16_t *const *bp,
                             int64_t kp, int64_t ldp, hipStream_t stream);

// Grouped: descriptors and tile-queue items live in device memory.
struct GroupedProblem {          // device-side problem record
  int64_t M, N, K;
  const void *A; const void *B; void *C;
  int64_t lda, ldb, ldc;
  int32_t vec;                   // 16-byte loads allowed
  int32_t pad_;
};
struct WorkItem {                // one output tile
  int32_t prob;                  // problem index
  int32_t cfg;                   // tile config id
  int32_t tm, tn;                // tile coordinates
};
// The work list holds three groups of items, each run by its own persistent
// kernel with its own queue counter (counter[q * kCounterStride], q = 0, 1,
// 2): problems whose own operands allow 16-byte transfers, packed problems
// (their plan-owned copies do), and the rest (register path).
constexpr int kCounterStride = 16, kQueues = 3;
hipError_t launch_grouped(int prec, bool vec, const GroupedProblem *probs, const WorkItem *items,
                          int32_t n_items, uint32_t *counter, int grid, hipStream_t stream);
hipError_t launch_counter_reset(uint32_t *counter, hipStream_t stream);
int grouped_max_grid(int prec);   // persistent workgroups that fit the device

// Copy of one operand into a plan-owned buffer whose rows allow 16-byte
// transfers: dst (drows x dcols, pitch dld, 16-byte aligned, dcols and dld
// whole vectors) receives src (rows x cols, pitch sld, any alignment) with
// zeros in [rows, drows) x [cols, dcols). Blocks [first_block, first_block +
// ceil(drows / kPackRows)) of the copy launch copy it; `grid` workgroups
// (0: one per block) walk the blocks.
struct PackJob {
  const void *src;
  void *dst;
  int64_t sld, dld;
  int64_t rows, cols, drows, dcols;
  int64_t first_block;
};
constexpr int kPackRows = 8;
hipError_t launch_pack(int prec, const PackJob *jobs, int32_t n_jobs, int64_t blocks, int grid,
                       hipStream_t stream);

// Error bookkeeping (thread-local detail string).
int set_error(int code, const std::string &detail);
void clear_error();

}  // namespace g355
