/*
 * gemm_mi355x.h -- C ABI of the MI355X (gfx950) dense matrix product library.
 *
 * The operation is the one Hasta and Mutiara (arXiv 1012.2273) benchmark:
 * the product of an (m x k) matrix A and a (k x n) matrix B of contiguous
 * row-major elements into an (m x n) matrix C that is zeroed and then
 * accumulated (Section 3.1, Algorithm 1; Section 3.1.1, Algorithms 2 and 3;
 * Section 3.1.2, Algorithm 4). C is therefore OVERWRITTEN with A*B: there is
 * no alpha/beta scaling.
 *
 * Conventions shared by every call
 *   - Matrices are row-major; a leading dimension (lda, ldb, ...) is the
 *     distance in ELEMENTS between the starts of two consecutive rows.
 *   - Matrix pointers are DEVICE pointers owned by the caller; the library
 *     never frees or retains them. `stream` is a hipStream_t (NULL = the
 *     null stream). Every call is asynchronous on `stream`: no host
 *     synchronisation except where stated (plan creation, autotuning).
 *   - Every call validates its arguments first and launches nothing when
 *     validation fails. Errors reported later by the device surface at the
 *     caller's next synchronisation of `stream`.
 *   - Sizes: m == 0 or n == 0 is a no-op returning GEMM_OK; k == 0 writes
 *     C = 0 (the zero initialisation of Algorithms 3 and 4).
 *   - C must not overlap A or B (not checked).
 *   - Any leading dimension >= the row length is accepted; 16-byte vector
 *     loads are used when the pointer and leading dimension allow it, scalar
 *     loads otherwise.
 *   - Calls are re-entrant; the thread-local text of the last error is
 *     returned by gemm_last_error().
 */
#ifndef GEMM_MI355X_H
#define GEMM_MI355X_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* Return codes. */
enum {
    GEMM_OK = 0,
    GEMM_EINVAL = 1,        /* negative size, count or unknown option            */
    GEMM_ENULL = 2,         /* NULL pointer where data is required               */
    GEMM_ELD = 3,           /* leading dimension smaller than the row length     */
    GEMM_EWORKSPACE = 4,    /* workspace missing or smaller than required        */
    GEMM_EUNSUPPORTED = 5,  /* unknown dtype or dtype not offered by this call   */
    GEMM_EHIP = 6,          /* the HIP runtime reported an error                 */
    GEMM_ENOMEM = 7,        /* device or host allocation failed (plans only)     */
    GEMM_ESTATE = 8         /* plan used in a state that does not allow the call */
};

/* Element types. */
enum {
    GEMM_F64 = 0,   /* A, B, C binary64                                          */
    GEMM_F32 = 1,   /* A, B, C binary32                                          */
    GEMM_BF16 = 2   /* A, B bfloat16 (16-bit patterns), C binary32; products are
                       accumulated in binary32                                   */
};

/*
 * gemm_plain -- C(m x n) = A(m x k) * B(k x n) in one dtype on the matrix
 * cores. Section 3.1, Algorithm 1 (the product) with C zeroed as in
 * Algorithms 3 and 4; the binary64 path is the paper's precision.
 *   dtype   GEMM_F64 / GEMM_F32 / GEMM_BF16 (see the enum for C's type).
 *   A, lda  device, m rows of k elements, lda >= k.
 *   B, ldb  device, k rows of n elements, ldb >= n.
 *   C, ldc  device, m rows of n elements, ldc >= n; overwritten.
 * Row pitches of A and B (ld times the element size) must be below 8 MiB.
 * Errors: EINVAL (m, n or k < 0, or a row pitch of 8 MiB or more), ENULL,
 * ELD, EUNSUPPORTED (dtype), EHIP.
 */
int gemm_plain(int dtype, int64_t m, int64_t n, int64_t k,
               const void *A, int64_t lda, const void *B, int64_t ldb,
               void *C, int64_t ldc, void *stream);

/*
 * gemm_plain_ksplit_workspace_size -- bytes of device workspace
 * gemm_plain_ksplit needs for this product: (chunks - 1) * m * n output
 * elements (C's type), 0 when the product runs unsplit. Depends on the
 * sizes, the device's CU count and this thread's forced settings only.
 * Returns 0 for an unknown dtype or a size <= 0.
 */
size_t gemm_plain_ksplit_workspace_size(int dtype, int64_t m, int64_t n, int64_t k);

/*
 * gemm_plain_ksplit -- the product of gemm_plain (Section 3.1, Algorithm 1;
 * same arguments and result type) for products with too few output tiles
 * to occupy the device (mid-size squares, short and wide or long-K shapes):
 * the sum over K is cut into chunks of whole K-tiles that run as separate
 * workgroups of one launch, chunk 0 writing its partial product to C and
 * chunk j > 0 to plane j - 1 of the workspace; a second launch adds the
 * planes to C in chunk order. The association of the sum over K differs
 * from gemm_plain's (one partial sum per chunk), the result is the same for
 * every call with the same sizes on the same device. Products with enough
 * tiles run as gemm_plain and leave the workspace untouched. (The chunk
 * count and shape can be forced per thread for tests and tuning, see
 * gemm_mi355x_tuning.h.)
 *   workspace, workspace_bytes  device memory owned by the caller, 16-byte
 *     aligned, at least gemm_plain_ksplit_workspace_size(dtype, m, n, k)
 *     bytes (NULL with 0 allowed when that is 0); its contents on entry do
 *     not matter and are overwritten. Calls that share a workspace must be
 *     ordered (one stream, or synchronised).
 * Errors: those of gemm_plain, and EWORKSPACE (NULL, too small or not
 * 16-byte aligned workspace).
 */
int gemm_plain_ksplit(int dtype, int64_t m, int64_t n, int64_t k,
                      const void *A, int64_t lda, const void *B, int64_t ldb,
                      void *C, int64_t ldc, void *workspace, size_t workspace_bytes,
                      void *stream);

/*
 * GEMM_NOALLOC_SCRATCH_BYTES -- size of the per-device scratch array of
 * gemm_plain_ksplit_noalloc (64 MiB; each device the library runs on holds
 * one until the process ends).
 */
#define GEMM_NOALLOC_SCRATCH_BYTES (64u << 20)

/*
 * gemm_plain_ksplit_noalloc -- gemm_plain_ksplit for callers that cannot
 * allocate device memory (code under HIP graph capture, tight serving loops,
 * harnesses that forbid allocation). Same arguments, product, chunking and
 * result bits as gemm_plain_ksplit, without the workspace: the partial
 * products go to a scratch array of GEMM_NOALLOC_SCRATCH_BYTES that the
 * library holds on each device. The call allocates nothing (no hipMalloc,
 * hipFree or allocating library routine); its first call on a device looks
 * the array's address up once.
 *   Concurrency: every call on one device shares that device's array, which
 *   keeps the last call's contents; calls that overlap on one device (other
 *   streams or threads without ordering) race and give undefined results.
 *   Order them on one stream or synchronise between them.
 * Errors: those of gemm_plain, EWORKSPACE when the product's K split needs
 * more than GEMM_NOALLOC_SCRATCH_BYTES (gemm_plain_ksplit_workspace_size
 * gives the need), EHIP when the array's address cannot be looked up.
 */
int gemm_plain_ksplit_noalloc(int dtype, int64_t m, int64_t n, int64_t k,
                              const void *A, int64_t lda, const void *B, int64_t ldb,
                              void *C, int64_t ldc, void *stream);

/*
 * gemm_split_workspace_size -- bytes of device workspace gemm_split needs
 * for this shape (the four bfloat16 operand planes, rows of k rounded up to
 * 8 elements at a pitch rounded up to 64 elements, planes 256-byte aligned).
 * Returns 0 for negative sizes.
 */
size_t gemm_split_workspace_size(int64_t m, int64_t n, int64_t k);

/*
 * gemm_split_convert -- the split step alone: each binary32 element x of
 * the (rows x cols) matrix X becomes hi = bf16(x) and lo = bf16(x - hi),
 * both rounded to nearest, ties to even; x - hi is exact in binary32.
 *   transpose = 0: hi[r][c] at hi + r*ldo + c (ldo >= cols)
 *   transpose = 1: hi[c][r] at hi + c*ldo + r (ldo >= rows), same for lo.
 * hi and lo are device arrays of 16-bit patterns owned by the caller.
 * This is the precision extension of the dense product (the paper fixes
 * binary64 only); see gemm_split for how the planes are used.
 * Errors: EINVAL, ENULL, ELD, EHIP.
 */
int gemm_split_convert(int64_t rows, int64_t cols, const float *X, int64_t ldx,
                       int transpose, uint16_t *hi, uint16_t *lo, int64_t ldo,
                       void *stream);

/*
 * gemm_split -- C(m x n) ~= A(m x k) * B(k x n) for binary32 A, B, C through
 * a two-way bfloat16 split of both operands and three products accumulated
 * in binary32 on the matrix cores: C = A_lo*B_hi + A_hi*B_lo + A_hi*B_hi
 * (A_lo*B_lo is dropped; its size is at most 2^-16 of |A||B|). The same
 * product as gemm_plain (Section 3.1, Algorithm 1), at a precision close to
 * binary32.
 *   workspace  device memory of at least gemm_split_workspace_size(m, n, k)
 *              bytes, owned by the caller, 16-byte aligned; it holds the
 *              planes between the split launch and the product launch, so it
 *              must not be shared by overlapping calls.
 * Workspace layout after a two-step call (16-bit patterns; kp = k rounded up
 * to 8, row pitch ldp = kp rounded up to 64 elements; each plane starts on a
 * 256-byte boundary, in this order): A_hi, A_lo, each m rows of ldp holding
 * A's rows (element (r, c) at r*ldp + c); then B_hi, B_lo, each n rows of ldp
 * holding B's columns (B transposed: element (r, c) of B at c*ldp + r).
 * Columns [k, kp) of every plane row hold zeros, [kp, ldp) are not written.
 * Small products (see gemm_split_one_launch) run as one launch that splits
 * each operand fragment in registers instead; the result is the same bit
 * for bit and the workspace is then left untouched (it is still required).
 * Errors: EINVAL, ENULL, ELD, EWORKSPACE, EHIP.
 */
int gemm_split(int64_t m, int64_t n, int64_t k,
               const float *A, int64_t lda, const float *B, int64_t ldb,
               float *C, int64_t ldc, void *workspace, size_t workspace_bytes,
               void *stream);

/*
 * gemm_split_one_launch -- 1 if gemm_split with these arguments runs as one
 * launch that splits each fragment in registers, 0 if it runs the split step
 * and then the plane product (or if the arguments are empty or null; nothing
 * is validated or launched). The in-register form needs A and B 16-byte
 * aligned with row pitches of a multiple of 16 bytes, k and n multiples of
 * 4, and either k <= 1024 with at most one 128 x 128 output tile per two CUs
 * of the current device (gemm_split3 runs in registers there too), or from
 * one tile per two CUs to one tile per CU (gemm_split only): there the
 * separate split step's pass over A and B costs more than repeating the
 * conversion in every wave that reads a fragment. All forms give the same
 * result bit for bit (Section 3.1, Algorithm 1 with the split operands of
 * gemm_split / gemm_split3).
 */
int gemm_split_one_launch(int64_t m, int64_t n, int64_t k, const float *A, int64_t lda,
                          const float *B, int64_t ldb);

/*
 * gemm_split3_workspace_size -- bytes of device workspace gemm_split3 needs
 * (six bfloat16 planes laid out as for gemm_split). Returns 0 for negative
 * sizes.
 */
size_t gemm_split3_workspace_size(int64_t m, int64_t n, int64_t k);

/*
 * gemm_split3_convert -- the three-way split step alone: each binary32
 * element x becomes hi = bf16(x), mid = bf16(x - hi), lo = bf16(x - hi -
 * mid), each rounded to nearest, ties to even; every difference is exact
 * in binary32, so hi + mid + lo carries all 24 significand bits of a
 * normal x. Layout, ownership and errors as gemm_split_convert, with three
 * output planes (hi, mid, lo).
 */
int gemm_split3_convert(int64_t rows, int64_t cols, const float *X, int64_t ldx,
                        int transpose, uint16_t *hi, uint16_t *mid, uint16_t *lo,
                        int64_t ldo, void *stream);

/*
 * gemm_split3 -- C(m x n) ~= A(m x k) * B(k x n) for binary32 A, B, C through
 * a three-way bfloat16 split of both operands and six products accumulated
 * in binary32 on the matrix cores, smallest first:
 *   C = A_lo*B_hi + A_hi*B_lo + A_mid*B_mid + A_mid*B_hi + A_hi*B_mid + A_hi*B_hi
 * (A_mid*B_lo, A_lo*B_mid and A_lo*B_lo are dropped: together at most about
 * 2^-23 of |A||B|, below the binary32 accumulation error). The same product
 * as gemm_plain (Section 3.1, Algorithm 1) at binary32 accuracy, on the
 * bfloat16 matrix cores; the higher-accuracy variant of gemm_split.
 *   workspace  device memory of at least gemm_split3_workspace_size(m, n, k)
 *              bytes, owned by the caller, 16-byte aligned, not shared by
 *              overlapping calls. Small products run as one launch that
 *              splits in registers (k <= 1024, at most one tile per two CUs);
 *              from one tile per two CUs up, except between three and five
 *              tiles per CU, one launch whose loader waves split each tile
 *              once into LDS (both need 16-byte rows, as gemm_split_one_launch
 *              states); either leaves the workspace untouched. After a
 *              two-step call it holds A_hi, A_mid, A_lo, B_hi, B_mid, B_lo
 *              in the layout gemm_split describes.
 * Errors: EINVAL, ENULL, ELD, EWORKSPACE, EHIP.
 */
int gemm_split3(int64_t m, int64_t n, int64_t k,
                const float *A, int64_t lda, const float *B, int64_t ldb,
                float *C, int64_t ldc, void *workspace, size_t workspace_bytes,
                void *stream);

/*
 * gemm_backward -- gradients of a scalar loss through C = A*B, given
 * dC = dL/dC (m x n):  dA = dC * B^T  (m x k),  dB = A^T * dC  (k x n).
 * The transposed operands are read in place (no transposed copy is made).
 * The differentiated product is the one of Section 3.1, Algorithm 1.
 *   dtype   GEMM_F64 / GEMM_F32 (all six matrices of that type) or GEMM_BF16
 *           (A, B, dC bfloat16; dA, dB binary32).
 *   dA or dB may be NULL to skip that gradient (then its ld is ignored).
 *   lda >= k, ldb >= n, lddc >= n, ldda >= k, lddb >= n.
 * Errors: EINVAL, ENULL, ELD, EUNSUPPORTED, EHIP.
 */
int gemm_backward(int dtype, int64_t m, int64_t n, int64_t k,
                  const void *A, int64_t lda, const void *B, int64_t ldb,
                  const void *dC, int64_t lddc, void *dA, int64_t ldda,
                  void *dB, int64_t lddb, void *stream);

/* One independent product of a group: C = A*B with the conventions above. */
typedef struct gemm_problem {
    int64_t m, n, k;
    const void *A;
    const void *B;
    void *C;
    int64_t lda, ldb, ldc;
} gemm_problem;

typedef struct gemm_plan gemm_plan;

/* Plan flags. */
enum {
    GEMM_PLAN_AUTOTUNE = 1,   /* time candidate tile policies on the device now */
    GEMM_PLAN_NO_GRAPH = 2,   /* launch directly instead of through a hipGraph  */
    GEMM_PLAN_NO_PACK = 4     /* read every operand where it is (no copies)     */
};

/*
 * gemm_grouped_plan_create -- prepare `count` independent products
 * (Section 3.1, Algorithm 1, applied to each) for one persistent launch.
 * The row-block work split of Section 3.1.1 (Algorithm 2) is replaced by a
 * device work queue of output tiles over all problems, largest first.
 *   dtype      GEMM_F64 or GEMM_F32.
 *   probs      host array of `count` descriptors, copied into the plan.
 *   tune_cache path of a JSON file holding tuned tile policies (read, and
 *              written after tuning); NULL for none.
 *   flags      GEMM_PLAN_* bits.
 *   stream     stream used for the upload, tuning and graph capture; the call
 *              synchronises it before returning.
 * The plan owns its device descriptor and queue arrays and its hipGraphExec
 * until gemm_grouped_plan_destroy. Tuning overwrites the C matrices.
 * Packing (unless GEMM_PLAN_NO_PACK): a problem (m, n, k > 0) whose A or B
 * rows are not whole 16-byte vectors (binary64 k or n odd, binary32 not
 * multiples of 4, or a base or leading dimension off 16 bytes) gets
 * plan-owned copies A' (m x k') and B' (k' x n'), k' and n' rounded up to
 * whole vectors and zero padded, (m k' + k' n') * element size bytes of
 * device memory in all; every run first copies A and B into them (one
 * launch for every such problem), then computes C from the copies, which
 * lets the persistent kernel use 16-byte transfers for every problem. C is
 * written in place as always. A packed problem's C equals, bit for bit, a
 * single gemm_plain launch at the same tile shape on A' and B' (its first n
 * columns); with GEMM_PLAN_NO_PACK it equals one on A and B themselves.
 * Errors: EINVAL (count < 0, bad flags, negative sizes), ENULL, ELD,
 * EUNSUPPORTED, ENOMEM, EHIP.
 */
int gemm_grouped_plan_create(gemm_plan **out, int dtype, const gemm_problem *probs,
                             int32_t count, const char *tune_cache, int flags,
                             void *stream);

/* gemm_grouped_run -- one launch of the plan (a hipGraphLaunch of the
 * captured queue reset + persistent kernel, unless GEMM_PLAN_NO_GRAPH).
 * `stream` may differ from the creation stream. Errors: ENULL, EHIP. */
int gemm_grouped_run(gemm_plan *plan, void *stream);

/* gemm_grouped_plan_update -- replace the A, B, C pointers (and nothing else)
 * of every problem; sizes and leading dimensions must equal the plan's.
 * A problem whose own A and B allowed 16-byte transfers at plan creation
 * runs in the kernel that reads them that way: its new A and B must be
 * 16-byte aligned as well (packed problems and, with GEMM_PLAN_NO_PACK, the
 * other problems take any alignment). Takes effect
 * for the next run without re-capture; synchronous copy, so no run of the
 * plan may still be executing (synchronise its stream first). Nothing
 * changes when the call fails.
 * Errors: ENULL, EINVAL (count or a size differs, or a 16-byte planned
 * problem gets operands that are not 16-byte aligned), EHIP. */
int gemm_grouped_plan_update(gemm_plan *plan, const gemm_problem *probs, int32_t count);

/* gemm_grouped_plan_destroy -- free the plan (NULL is a no-op). */
int gemm_grouped_plan_destroy(gemm_plan *plan);

/* gemm_grouped_plan_info -- number of output tiles and the tile policy
 * chosen per size class (writes up to `cap` config ids into `policy`). */
int gemm_grouped_plan_info(const gemm_plan *plan, int64_t *tiles, int32_t *policy,
                           int32_t cap);

/*
 * gemm_grouped -- uncaptured convenience: plan with the default policy (or
 * the last policy tuned for this dtype in this process), run once on
 * `stream`, release the plan after the stream completes (the call
 * synchronises `stream`). Errors: as plan_create and run.
 */
int gemm_grouped(int dtype, const gemm_problem *probs, int32_t count, void *stream);

/* gemm_strerror -- static text for a return code. */
const char *gemm_strerror(int status);

/* gemm_last_error -- thread-local detail of the last failing call on this
 * thread ("" if none). The pointer stays valid until the next call. */
const char *gemm_last_error(void);

/* gemm_tile_config_count / gemm_tile_config_name -- the tile shapes the
 * kernels are built for, named "BMxBN" plus a suffix: w8 (8 waves), k2 / k4
 * (two or four waves per output position, each taking a part of every
 * K-tile); "" for an id out of range. The grouped plan info reports its
 * policy with these ids. */
int gemm_tile_config_count(void);
const char *gemm_tile_config_name(int id);

#ifdef __cplusplus
}
#endif
#endif /* GEMM_MI355X_H */
