/*
 * gemm_mi355x_tuning.h -- tuning knobs of libgemm_mi355x.so for tests and
 * tuning tools. Not part of the product ABI (gemm_mi355x.h): production
 * callers never need them. Each knob holds per calling thread, so forcing a
 * shape on one thread never changes the launches of another.
 */
#ifndef GEMM_MI355X_TUNING_H
#define GEMM_MI355X_TUNING_H

#ifdef __cplusplus
extern "C" {
#endif

/*
 * gemm_tuning_force_tile_config -- make this thread's single-product calls
 * (gemm_plain, gemm_split, gemm_split3, gemm_backward) use tile config `id`
 * (an index of gemm_tile_config_name) wherever the precision and operand
 * layout offer it; -1 restores the size-based choice. gemm_plain_ksplit
 * takes the forced shape when it names 128x128, 128x128w8, 128x64 or 64x64.
 * The product computed is unchanged (Section 3.1, Algorithm 1); only its
 * blocking and summation order follow the shape.
 * Errors: EINVAL (id below -1 or not a config index).
 */
int gemm_tuning_force_tile_config(int id);

/*
 * gemm_tuning_force_ksplit_parts -- make this thread's gemm_plain_ksplit
 * calls (and workspace queries) cut K into `parts` chunks of a multiple of
 * 64 indices (fewer if K is short); -1 restores the automatic count.
 * Errors: EINVAL (parts 0, below -1 or above 65535).
 */
int gemm_tuning_force_ksplit_parts(int parts);

/*
 * gemm_tuning_force_split_form -- make this thread's gemm_split and
 * gemm_split3 calls use one form: 0 the split step into the workspace and
 * then the plane product, 1 one launch that splits each fragment in the
 * registers of the waves that multiply it, 2 one launch whose loader waves
 * split every tile once into LDS planes; -1 restores the size-based choice.
 * Forms 1 and 2 need A and B rows of whole 16-byte vectors (binary32: 16-
 * byte aligned, k and n multiples of 4) and fall back to form 0 otherwise.
 * All forms give the same result bit for bit for the same tile shape.
 * Errors: EINVAL (form below -1 or above 2).
 */
int gemm_tuning_force_split_form(int form);

#ifdef __cplusplus
}
#endif
#endif /* GEMM_MI355X_TUNING_H */
