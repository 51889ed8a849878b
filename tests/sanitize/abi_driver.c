/*
 * Sanitizer driver for the host side of libgemm_mi355x.so (test
 * infrastructure): the library's host code is built with AddressSanitizer and
 * UndefinedBehaviorSanitizer, and this program calls every entry point of the
 * C ABI with arguments the validation must refuse (negative sizes, NULL
 * operands, short leading dimensions, unknown dtypes, missing, short or
 * misaligned workspaces, out-of-range knobs and plan arguments) plus the
 * queries that touch no device. None of these calls reaches a kernel launch,
 * so the driver runs without a GPU. Exit status 0: every call returned the
 * documented status and the sanitizers reported nothing.
 */
#include <stdint.h>
#include <stdio.h>
#include <string.h>

#include "gemm_mi355x.h"
#include "gemm_mi355x_tuning.h"

static int failures = 0;
#define EXPECT(call, status)                                                      \
    do {                                                                          \
        int rc_ = (call);                                                         \
        if (rc_ != (status)) {                                                    \
            fprintf(stderr, "line %d: %s returned %d, expected %d (%s)\n", __LINE__, \
                    #call, rc_, (status), gemm_last_error());                     \
            ++failures;                                                           \
        }                                                                         \
    } while (0)

int main(void)
{
    /* addresses that are never dereferenced: validation fails first */
    void *p = (void *)(uintptr_t)4096, *q = (void *)(uintptr_t)8192;
    void *w = (void *)(uintptr_t)65536, *w8 = (void *)(uintptr_t)65544;

    for (int s = 0; s <= 9; ++s) {
        const char *t = gemm_strerror(s);
        if (!t || !*t) ++failures;
    }
    if (strcmp(gemm_strerror(99), "unknown status") != 0) ++failures;
    for (int i = -1; i <= gemm_tile_config_count(); ++i) (void)strlen(gemm_tile_config_name(i));

    /* gemm_plain */
    EXPECT(gemm_plain(7, 4, 4, 4, p, 4, q, 4, w, 4, NULL), GEMM_EUNSUPPORTED);
    EXPECT(gemm_plain(GEMM_F64, -1, 4, 4, p, 4, q, 4, w, 4, NULL), GEMM_EINVAL);
    EXPECT(gemm_plain(GEMM_F64, 4, 4, 4, NULL, 4, q, 4, w, 4, NULL), GEMM_ENULL);
    EXPECT(gemm_plain(GEMM_F64, 4, 4, 4, p, 3, q, 4, w, 4, NULL), GEMM_ELD);
    EXPECT(gemm_plain(GEMM_F32, 4, 4, 4, p, 4, q, 3, w, 4, NULL), GEMM_ELD);
    EXPECT(gemm_plain(GEMM_BF16, 4, 4, 4, p, 4, q, 4, w, 3, NULL), GEMM_ELD);
    EXPECT(gemm_plain(GEMM_F64, 0, 4, 4, NULL, 4, q, 4, NULL, 4, NULL), GEMM_OK);
    EXPECT(gemm_plain(GEMM_F64, 4, 4, 4, p, (int64_t)1 << 21, q, 4, w, 4, NULL), GEMM_EINVAL);

    /* K split, its workspace query and the allocation-free form */
    const size_t ks = gemm_plain_ksplit_workspace_size(GEMM_F64, 256, 256, 65536);
    if (ks != (size_t)63 * 256 * 256 * 8) ++failures;
    if (gemm_plain_ksplit_workspace_size(9, 256, 256, 65536) != 0) ++failures;
    EXPECT(gemm_plain_ksplit(GEMM_F64, 256, 256, 65536, p, 65536, q, 256, w, 256, NULL, ks, NULL),
           GEMM_EWORKSPACE);
    EXPECT(gemm_plain_ksplit(GEMM_F64, 256, 256, 65536, p, 65536, q, 256, w, 256, w, ks - 1, NULL),
           GEMM_EWORKSPACE);
    EXPECT(gemm_plain_ksplit(GEMM_F64, 256, 256, 65536, p, 65536, q, 256, w, 256, w8, ks, NULL),
           GEMM_EWORKSPACE);
    EXPECT(gemm_plain_ksplit(GEMM_F64, 256, 256, 65536, p, 65535, q, 256, w, 256, w, ks, NULL),
           GEMM_ELD);
    EXPECT(gemm_tuning_force_ksplit_parts(20), GEMM_OK);
    EXPECT(gemm_plain_ksplit_noalloc(GEMM_F64, 1024, 1024, 8192, p, 8192, q, 1024, w, 1024, NULL),
           GEMM_EWORKSPACE);
    EXPECT(gemm_tuning_force_ksplit_parts(-1), GEMM_OK);
    EXPECT(gemm_tuning_force_ksplit_parts(0), GEMM_EINVAL);
    EXPECT(gemm_tuning_force_ksplit_parts(70000), GEMM_EINVAL);
    EXPECT(gemm_plain_ksplit_noalloc(GEMM_F64, 4, 4, -2, p, 4, q, 4, w, 4, NULL), GEMM_EINVAL);

    /* split products */
    const size_t ws2 = gemm_split_workspace_size(100, 60, 70);
    const size_t ws3 = gemm_split3_workspace_size(100, 60, 70);
    if (ws2 == 0 || ws3 <= ws2) ++failures;
    EXPECT(gemm_split(100, 60, 70, p, 70, q, 60, w, 60, NULL, ws2, NULL), GEMM_EWORKSPACE);
    EXPECT(gemm_split(100, 60, 70, p, 70, q, 60, w, 60, w, ws2 - 1, NULL), GEMM_EWORKSPACE);
    EXPECT(gemm_split(100, 60, 70, p, 70, q, 60, w, 60, w8, ws2, NULL), GEMM_EWORKSPACE);
    EXPECT(gemm_split(100, 60, 70, p, 69, q, 60, w, 60, w, ws2, NULL), GEMM_ELD);
    EXPECT(gemm_split(-3, 60, 70, p, 70, q, 60, w, 60, w, ws2, NULL), GEMM_EINVAL);
    EXPECT(gemm_split3(100, 60, 70, p, 70, NULL, 60, w, 60, w, ws3, NULL), GEMM_ENULL);
    EXPECT(gemm_split3(100, 60, 70, p, 70, q, 60, w, 60, w, ws2, NULL), GEMM_EWORKSPACE);
    EXPECT(gemm_split_convert(4, 4, p, 3, 0, q, w, 4, NULL), GEMM_ELD);
    EXPECT(gemm_split_convert(4, 4, p, 4, 1, q, w, 3, NULL), GEMM_ELD);
    EXPECT(gemm_split_convert(-1, 4, p, 4, 0, q, w, 4, NULL), GEMM_EINVAL);
    EXPECT(gemm_split_convert(4, 4, p, 4, 0, NULL, w, 4, NULL), GEMM_ENULL);
    EXPECT(gemm_split3_convert(4, 4, p, 4, 0, q, NULL, w, 4, NULL), GEMM_ENULL);
    EXPECT(gemm_tuning_force_split_form(3), GEMM_EINVAL);
    EXPECT(gemm_tuning_force_split_form(-2), GEMM_EINVAL);
    EXPECT(gemm_tuning_force_split_form(-1), GEMM_OK);
    (void)gemm_split_one_launch(100, 60, 70, p, 70, q, 60);

    /* backward */
    EXPECT(gemm_backward(5, 4, 4, 4, p, 4, q, 4, w, 4, p, 4, q, 4, NULL), GEMM_EUNSUPPORTED);
    EXPECT(gemm_backward(GEMM_F64, 4, 4, 4, p, 4, q, 4, NULL, 4, p, 4, q, 4, NULL), GEMM_ENULL);
    EXPECT(gemm_backward(GEMM_F64, 4, 4, 4, p, 4, q, 3, w, 4, p, 4, NULL, 0, NULL), GEMM_ELD);
    EXPECT(gemm_backward(GEMM_F32, 4, -1, 4, p, 4, q, 4, w, 4, p, 4, q, 4, NULL), GEMM_EINVAL);

    /* grouped plans */
    gemm_problem probs[2] = {{4, 4, 4, p, q, w, 4, 4, 4}, {4, 4, 4, p, q, w, 3, 4, 4}};
    gemm_plan *plan = NULL;
    EXPECT(gemm_grouped_plan_create(&plan, GEMM_F64, probs, 2, NULL, 0, NULL), GEMM_ELD);
    EXPECT(gemm_grouped_plan_create(&plan, GEMM_BF16, probs, 2, NULL, 0, NULL), GEMM_EUNSUPPORTED);
    EXPECT(gemm_grouped_plan_create(&plan, GEMM_F64, probs, -1, NULL, 0, NULL), GEMM_EINVAL);
    EXPECT(gemm_grouped_plan_create(&plan, GEMM_F64, probs, 1, NULL, 8, NULL), GEMM_EINVAL);
    EXPECT(gemm_grouped_plan_create(NULL, GEMM_F64, probs, 1, NULL, 0, NULL), GEMM_ENULL);
    EXPECT(gemm_grouped(GEMM_F32, probs, 2, NULL), GEMM_ELD);
    EXPECT(gemm_grouped(GEMM_F64, NULL, 2, NULL), GEMM_ENULL);
    EXPECT(gemm_grouped_run(NULL, NULL), GEMM_ENULL);
    EXPECT(gemm_grouped_plan_update(NULL, probs, 1), GEMM_ENULL);
    EXPECT(gemm_grouped_plan_info(NULL, NULL, NULL, 0), GEMM_ENULL);
    EXPECT(gemm_grouped_plan_destroy(NULL), GEMM_OK);
    EXPECT(gemm_tuning_force_tile_config(gemm_tile_config_count()), GEMM_EINVAL);
    EXPECT(gemm_tuning_force_tile_config(-1), GEMM_OK);

    if (failures) {
        fprintf(stderr, "%d check(s) failed\n", failures);
        return 1;
    }
    printf("ABI sanitizer driver: all checks held\n");
    return 0;
}
