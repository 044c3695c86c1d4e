/* Host sanitizer driver for the C ABI's argument checks
 * (tests/test_host_sanitizers.py): every call below must be rejected (or
 * answered) on the host, before any GPU work, with the documented code; the
 * library and this driver are built with AddressSanitizer and
 * UndefinedBehaviorSanitizer on their host code.  Needs no GPU. */
#include <stdio.h>
#include <string.h>

#include "gsyeig.h"

static int fails = 0;
#define EXPECT(call, want)                                                                        \
    do {                                                                                          \
        const int got_ = (call);                                                                  \
        if (got_ != (want)) {                                                                     \
            printf("%s: got %d, want %d\n", #call, got_, (int)(want));                            \
            ++fails;                                                                              \
        }                                                                                         \
    } while (0)

int main(void)
{
    double d[4] = {0, 0, 0, 0};
    float f[4] = {0, 0, 0, 0};
    gsyeig_opts o;
    gsyeig_info info;
    size_t bytes = 0;
    memset(&info, 0, sizeof(info));
    if (!gsyeig_version() || !gsyeig_version()[0]) ++fails;
    EXPECT(gsyeig_opts_default(NULL), -1);
    EXPECT(gsyeig_opts_default(&o), 0);
    EXPECT(gsyeig_workspace_size(0, 1, &o, &bytes), -1);
    EXPECT(gsyeig_workspace_size(10, 11, &o, &bytes), -2);
    EXPECT(gsyeig_workspace_size(10, 2, &o, NULL), -4);
    EXPECT(gsyeig_workspace_size(16384, 100, NULL, &bytes), 0);
    if (bytes < (size_t)16384 * 12001 * 8) ++fails;
    o.prec = GSYEIG_MIXED;
    EXPECT(gsyeig_workspace_size(16384, 100, &o, &bytes), 0);
    gsyeig_opts_default(&o);
    EXPECT(gsyeig_create(NULL, NULL), -1);
    EXPECT(gsyeig_destroy(NULL), -1);
    EXPECT(gsyeig_set_trsv_block(NULL, 512), -1);
    EXPECT(gsyeig_set_trsv_sweep(NULL, 0), -1);
    EXPECT(gsyeig_set_spin_limit(NULL, 1), -1);
    EXPECT(gsyeig_sync(NULL), -1);
    EXPECT(gsyeig_autotune(NULL, 100, 0, NULL, NULL), -1);
    EXPECT(gsyeig_potrf(NULL, 10, d, 10, &o, NULL), -1);
    EXPECT(gsyeig_trsv(NULL, 10, d, 10, 0, d, d), -1);
    EXPECT(gsyeig_trsv_lp(NULL, 10, f, 10, 0, d, d), -1);
    EXPECT(gsyeig_trsm_lp(NULL, 10, f, 10, 0, 2, d, 10, d, 10), -1);
    EXPECT(gsyeig_syev_small(NULL, 10, d, 10, 2, 0, d, d, 10), -1);
    EXPECT(gsyeig_solve(NULL, 10, 2, d, 10, d, 10, &o, d, d, 10, &info), -1);
    EXPECT(gsyeig_symv_noalloc(NULL, 0, d, 1, d, d), -2);
    EXPECT(gsyeig_symv_noalloc(NULL, GSYEIG_NOALLOC_MAX_N + 1, d, GSYEIG_NOALLOC_MAX_N + 1, d, d), GSYEIG_ETOOBIG);
    EXPECT(gsyeig_symv_noalloc(NULL, 10, NULL, 10, d, d), -3);
    EXPECT(gsyeig_symv_noalloc(NULL, 10, d, 9, d, d), -4);
    EXPECT(gsyeig_symv_noalloc(NULL, 10, d, 10, NULL, d), -5);
    EXPECT(gsyeig_symv_noalloc(NULL, 10, d, 10, d, NULL), -6);
    if (fails) {
        printf("%d failures\n", fails);
        return 1;
    }
    printf("ok\n");
    return 0;
}
