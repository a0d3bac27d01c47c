/* Host-side checks of libccmi under AddressSanitizer and
 * UndefinedBehaviorSanitizer: every entry point is called with arguments
 * its host code must refuse, or with sizes whose arithmetic it does on the
 * host (workspace bounds up to the ABI's limits), plus the router file
 * parser on good and malformed files.  Nothing here needs a GPU.  Built and
 * run by tests/test_host_sanitizer.py against _build/san/libccmi_san.so;
 * exits non-zero on the first unexpected return code, and the sanitizers
 * abort on any memory error or undefined behaviour. */
#include <stdint.h>
#include <stdio.h>
#include <stdlib.h>
#include <string.h>

#include "cc.h"

static int failures = 0;

#define EXPECT(call, want)                                                                        \
    do {                                                                                          \
        long long got_ = (long long)(call);                                                       \
        if (got_ != (long long)(want)) {                                                          \
            fprintf(stderr, "%s:%d: %s returned %lld, expected %lld (%s)\n", __FILE__, __LINE__, #call, \
                    got_, (long long)(want), cc_last_error());                                    \
            ++failures;                                                                           \
        }                                                                                         \
    } while (0)

#define EXPECT_MSG()                                                                              \
    do {                                                                                          \
        if (!cc_last_error() || !cc_last_error()[0]) {                                            \
            fprintf(stderr, "%s:%d: empty error message\n", __FILE__, __LINE__);                  \
            ++failures;                                                                           \
        }                                                                                         \
    } while (0)

static void write_file(const char* path, const char* text) {
    FILE* f = fopen(path, "w");
    if (!f) {
        perror(path);
        exit(2);
    }
    fputs(text, f);
    fclose(f);
}

int main(int argc, char** argv) {
    const char* dir = argc > 1 ? argv[1] : ".";
    const char* weights = argc > 2 ? argv[2] : NULL;
    int32_t* P = (int32_t*)(uintptr_t)64;   /* never dereferenced: every call below fails first */
    int64_t* P64 = (int64_t*)(uintptr_t)64;
    char path[4096];

    EXPECT(cc_version(), CC_VERSION);
    EXPECT(cc_last_error()[0], 0);

    cc_options o;
    cc_default_options(&o);
    cc_default_options(NULL);
    EXPECT(o.route, CC_ROUTE_AUTO);
    EXPECT(o.check, 0);

    /* cc_label_ex: host validation */
    EXPECT(cc_label_ex(P, P, -1, 5, P, NULL, NULL, NULL), CC_EINVAL);
    EXPECT_MSG();
    EXPECT(cc_label_ex(P, P, 5, -1, P, NULL, NULL, NULL), CC_EINVAL);
    EXPECT(cc_label_ex(P, P, 5, 0, P, NULL, NULL, NULL), CC_EINVAL);
    EXPECT(cc_label_ex(NULL, P, 5, 5, P, NULL, NULL, NULL), CC_EINVAL);
    EXPECT(cc_label_ex(P, P, 5, 5, NULL, NULL, NULL, NULL), CC_EINVAL);
    EXPECT(cc_label_ex(P, P, INT64_MAX, 5, P, NULL, NULL, NULL), CC_EINVAL);
    cc_stats st;
    EXPECT(cc_label_ex(NULL, NULL, 0, 0, NULL, NULL, NULL, &st), CC_OK);
    cc_options bad = o;
    bad.route = 99;
    EXPECT(cc_label_ex(P, P, 5, 5, P, NULL, &bad, NULL), CC_EINVAL);
    bad = o;
    bad.max_passes = -3;
    EXPECT(cc_label_ex(P, P, 5, 5, P, NULL, &bad, NULL), CC_EINVAL);
    bad = o;
    bad.scratch = 7;
    EXPECT(cc_label_ex(P, P, 5, 5, P, NULL, &bad, NULL), CC_EINVAL);
    bad = o;
    bad.workspace = P;
    bad.workspace_bytes = 0;
    EXPECT(cc_label_ex(P, P, 5, 5, P, NULL, &bad, NULL), CC_EINVAL);
    bad.workspace_bytes = 100;   /* far below the bound */
    EXPECT(cc_label_ex(P, P, 5000, 5000, P, NULL, &bad, NULL), CC_EINVAL);
    EXPECT(cc_label(P, P, -7, 3, P, NULL), CC_EINVAL);

    /* workspace bounds: host arithmetic over the ABI's whole range */
    const int64_t ms[] = {0, 1, 255, 1 << 20, (int64_t)1 << 22, (int64_t)1 << 31, (int64_t)3 << 31,
                          (int64_t)2048 * INT32_MAX};
    const int32_t ns[] = {0, 1, 4096, 1 << 20, (1 << 29) + 1, INT32_MAX};
    for (unsigned i = 0; i < sizeof ms / sizeof ms[0]; ++i)
        for (unsigned j = 0; j < sizeof ns / sizeof ns[0]; ++j)
            for (int r = CC_ROUTE_AUTO; r <= CC_ROUTE_SV_THETA; ++r) {
                int64_t b = cc_workspace_size(ms[i], ns[j], r);
                if (b <= 0) {
                    fprintf(stderr, "cc_workspace_size(%lld, %d, %d) = %lld\n", (long long)ms[i], ns[j], r,
                            (long long)b);
                    ++failures;
                }
                if (r == CC_ROUTE_SV && b > cc_workspace_size(ms[i], ns[j], CC_ROUTE_AUTO)) {
                    fprintf(stderr, "SV-only bound above the full bound at (%lld, %d)\n", (long long)ms[i], ns[j]);
                    ++failures;
                }
            }
    EXPECT(cc_workspace_size(-1, 5, 0), CC_EINVAL);
    EXPECT(cc_workspace_size(5, -1, 0), CC_EINVAL);
    EXPECT(cc_workspace_size(5, 5, 42), CC_EINVAL);

    /* batched */
    EXPECT(cc_label_batched(P, P, P64, P64, -1, P, NULL), CC_EINVAL);
    EXPECT(cc_label_batched(P, P, NULL, P64, 3, P, NULL), CC_EINVAL);
    EXPECT(cc_label_batched(P, P, P64, NULL, 3, P, NULL), CC_EINVAL);
    EXPECT(cc_label_batched(NULL, NULL, NULL, NULL, 0, NULL, NULL), CC_OK);
    cc_batch_stats bs;
    EXPECT(cc_label_batched_ex(P, P, P64, P64, 3, P, NULL, -5, 0, &bs), CC_EINVAL);

    /* 64-bit ids, the tuple ablation, the allocation-free entry point */
    int64_t nout = 0;
    EXPECT(cc_label64(P64, P64, -1, 8, P64, P64, &nout, NULL), CC_EINVAL);
    EXPECT(cc_label64(P64, P64, 10, 8, P64, P64, NULL, NULL), CC_EINVAL);
    EXPECT(cc_label64(NULL, NULL, 10, 8, P64, P64, &nout, NULL), CC_EINVAL);
    EXPECT(cc_label64(P64, P64, 10, (int64_t)1 << 31, P64, P64, &nout, NULL), CC_EINVAL);
    cc_tuple_stats ts;
    EXPECT(cc_label_tuples(NULL, NULL, -1, 5, NULL, NULL, 0, &ts), CC_EINVAL);
    EXPECT(cc_label_tuples(P, P, (int64_t)1 << 31, 1 << 30, P, NULL, 1, &ts), CC_EINVAL);
    EXPECT(cc_label_tuples(NULL, NULL, 0, 0, NULL, NULL, 0, NULL), CC_OK);
    EXPECT(cc_label_noalloc(NULL, NULL, -1, 5, NULL, NULL), CC_EINVAL);
    EXPECT(cc_label_noalloc(P, P, (int64_t)1 << 40, 5, P, NULL), CC_EINVAL);

    /* checks and the failure hook */
    int64_t badc[3] = {7, 7, 7};
    EXPECT(cc_check_labels(P, P, 3, 0, NULL, NULL, badc), CC_OK);
    EXPECT(badc[2], 3);
    EXPECT(cc_check_labels(NULL, P, 3, 5, P, NULL, badc), CC_EINVAL);
    EXPECT(cc_check_labels(P, P, 3, 5, P, NULL, NULL), CC_EINVAL);
    EXPECT(cc_debug_fail_alloc(-2), CC_EINVAL);
    EXPECT(cc_debug_fail_alloc(5), CC_OK);
    EXPECT(cc_debug_fail_alloc(0), CC_OK);

    EXPECT(cc_measure_peaks(NULL, NULL), CC_EINVAL);

    /* step entry points */
    EXPECT(cc_degree(P, P, -1, 5, P, NULL), CC_EINVAL);
    EXPECT(cc_degree(NULL, P, 4, 5, P, NULL), CC_EINVAL);
    int64_t cnt = 0;
    int32_t am = 0;
    EXPECT(cc_degree_histograms(P, -1, P64, P64, P, 4, &cnt, &am, NULL), CC_EINVAL);
    EXPECT(cc_degree_histograms(P, 5, NULL, P64, P, 4, &cnt, &am, NULL), CC_EINVAL);
    EXPECT(cc_csr(P, P, -1, 5, P, P64, P, NULL), CC_EINVAL);
    EXPECT(cc_mlp_forward(NULL, NULL, -1, NULL, NULL), CC_EINVAL);
    EXPECT(cc_mlp_forward(NULL, NULL, 0, NULL, NULL), CC_OK);
    EXPECT(cc_mlp_forward(NULL, (float*)P, 4, (float*)P, NULL), CC_EINVAL);

    /* router files */
    EXPECT(cc_router_load(NULL), CC_EINVAL);
    snprintf(path, sizeof path, "%s/no/such/file.txt", dir);
    EXPECT(cc_router_load(path), CC_EINVAL);
    snprintf(path, sizeof path, "%s/short.txt", dir);
    write_file(path, "# comment only\n1 2 3\n");
    EXPECT(cc_router_load(path), CC_EINVAL);
    EXPECT_MSG();
    /* every number on one line of about 45 KB */
    size_t cap = (size_t)CC_ROUTER_NPARAMS * 12 + 64, len = 0;
    char* big = (char*)malloc(cap);
    for (int i = 0; i < CC_ROUTER_NPARAMS; ++i) len += (size_t)snprintf(big + len, cap - len, "%.6g ", 1e-3 * i);
    snprintf(big + len, cap - len, "\n");
    snprintf(path, sizeof path, "%s/one_line.txt", dir);
    write_file(path, big);
    EXPECT(cc_router_load(path), CC_OK);
    EXPECT(cc_router_loaded(), 1);
    /* a token too long for any fixed buffer, then a non-finite value */
    memset(big, '7', cap - 2);
    big[cap - 2] = '\n';
    big[cap - 1] = 0;
    snprintf(path, sizeof path, "%s/long_token.txt", dir);
    write_file(path, big);
    EXPECT(cc_router_load(path), CC_EINVAL);
    snprintf(path, sizeof path, "%s/nan.txt", dir);
    write_file(path, "nan inf -inf\n");
    EXPECT(cc_router_load(path), CC_EINVAL);
    free(big);
    if (weights) EXPECT(cc_router_load(weights), CC_OK);
    EXPECT(cc_router_set(NULL), CC_OK);
    EXPECT(cc_router_loaded(), 0);

    if (failures) {
        fprintf(stderr, "%d unexpected results\n", failures);
        return 1;
    }
    printf("host ABI checks passed\n");
    return 0;
}
