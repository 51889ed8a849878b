// internal.h -- host-side declarations shared by the library's translation
// units (not part of the public ABI).
#pragma once

#include <hip/hip_runtime.h>
#include <stddef.h>
#include <stdint.h>

#include <string>

namespace g355 {

struct GemmArgs;

// Tile configurations the kernels are instantiated for. The id is the
// value the tuner and the grouped planner store.
// Configs below CFG_GROUPED_COUNT use 256 threads and can share the
// persistent grouped kernel; the others run as single-product launches.
enum TileCfg : int {
  CFG_128x128 = 0, CFG_128x64 = 1, CFG_64x64 = 2, CFG_32x32 = 3, CFG_GROUPED_COUNT = 4,
  CFG_128x128_W8 = 4, CFG_128x128_K2 = 5, CFG_128x64_K2 = 6, CFG_COUNT = 7
};
struct CfgInfo { int bm, bn; const char *name; };
const CfgInfo &cfg_info(int id);
bool cfg_supported(int prec, int cfg);

// Operand layout of one launch: TA -> op(A) = A^T stored K x M;
// TB -> op(B) = B^T stored N x K.
enum Layout : int { LAYOUT_NN = 0, LAYOUT_NT = 1, LAYOUT_TN = 2 };

// Launch one single-product kernel (grid = all tiles of C).
// prec: 0 f64, 1 f32, 2 bf16, 3 split. Returns hipSuccess or the launch error.
hipError_t launch_plain(int prec, int layout, int cfg, bool vec, const GemmArgs &a,
                        hipStream_t stream);

// Split kernels: X (rows x cols, ldx) -> hi/lo 16-bit planes. Plane rows
// are written up to `out_pad` >= their length (cols, or rows when
// transposed), the padding with zeros.
hipError_t launch_split(int64_t rows, int64_t cols, const float *X, int64_t ldx, bool transpose,
                        uint16_t *hi, uint16_t *lo, int64_t ldo, int64_t out_pad,
                        hipStream_t stream);

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
hipError_t launch_grouped(int prec, const GroupedProblem *probs, const WorkItem *items,
                          int32_t n_items, uint32_t *counter, int grid, hipStream_t stream);
hipError_t launch_counter_reset(uint32_t *counter, hipStream_t stream);
int grouped_max_grid(int prec);   // persistent workgroups that fit the device

// Error bookkeeping (thread-local detail string).
int set_error(int code, const std::string &detail);
void clear_error();

}  // namespace g355
