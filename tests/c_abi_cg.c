/* Test program (test infrastructure, not part of the library): the C ABI of
 * include/mfe.h used from plain C, without Python.  A context on the null
 * stream with the library's own allocator, the paper's 20^3 problem (Sec. 1:
 * u = 1 on x = 1, 0 on the other faces), FP64 CG to 1e-8 with each SpMV
 * format, the true residual recomputed on the host from mfe_rhs and
 * mfe_spmv, the sizes against their closed forms (m = 21^3, nnz = 61^3,
 * nb = 21 * 61 * 61), and three refused calls.  Prints one line per solve;
 * exit status 0 when every check holds.
 */
#include <math.h>
#include <stdio.h>
#include <stdlib.h>

#include <hip/hip_runtime_api.h>

#include "../include/mfe.h"

static int fails = 0;

#define CHECK(c)                                                              \
    do {                                                                      \
        if (!(c)) {                                                           \
            fprintf(stderr, "check failed: %s (line %d): %s\n", #c, __LINE__, \
                    mfe_last_error());                                        \
            ++fails;                                                          \
        }                                                                     \
    } while (0)

int main(void)
{
    mfe_ctx *ctx = NULL;
    if (mfe_ctx_create(0, NULL, NULL, NULL, NULL, &ctx) != MFE_OK) {
        fprintf(stderr, "mfe_ctx_create: %s\n", mfe_last_error());
        return 2;
    }
    const int N = 20;
    mfe_problem *P = NULL;
    if (mfe_problem_create(ctx, N, N, N, NULL, NULL, MFE_CSR | MFE_BCRS13, MFE_F64, &P) != MFE_OK) {
        fprintf(stderr, "mfe_problem_create: %s\n", mfe_last_error());
        mfe_ctx_destroy(ctx);
        return 2;
    }
    int64_t m = 0, nnz = 0, nb = 0;
    CHECK(mfe_problem_info(P, &m, &nnz, &nb) == MFE_OK);
    CHECK(m == 21 * 21 * 21 && nnz == 61 * 61 * 61 && nb == 21 * 61 * 61);

    double *x = NULL, *b = NULL, *y = NULL;
    CHECK(hipMalloc((void **)&x, (size_t)m * sizeof(double)) == hipSuccess);
    CHECK(hipMalloc((void **)&b, (size_t)m * sizeof(double)) == hipSuccess);
    CHECK(hipMalloc((void **)&y, (size_t)m * sizeof(double)) == hipSuccess);
    double *hb = (double *)malloc((size_t)m * sizeof(double));
    double *hy = (double *)malloc((size_t)m * sizeof(double));
    if (fails || !hb || !hy) return 2;
    CHECK(mfe_rhs(P, b) == MFE_OK);
    CHECK(hipMemcpy(hb, b, (size_t)m * sizeof(double), hipMemcpyDeviceToHost) == hipSuccess);
    double bb = 0.0;
    for (int64_t i = 0; i < m; ++i) bb += hb[i] * hb[i];

    const int formats[2] = {MFE_CSR, MFE_BCRS13};
    const char *names[2] = {"csr", "bcrs13"};
    for (int f = 0; f < 2; ++f) {
        CHECK(hipMemset(x, 0, (size_t)m * sizeof(double)) == hipSuccess);
        mfe_cg_stats st;
        CHECK(mfe_cg(P, formats[f], x, 1e-8, 1000, NULL, &st) == MFE_OK);
        CHECK(st.status == MFE_OK && st.rel_res_true <= 1e-8 && st.iterations > 10 && st.iterations < 100);
        CHECK(mfe_spmv(P, formats[f], x, y) == MFE_OK);
        CHECK(hipMemcpy(hy, y, (size_t)m * sizeof(double), hipMemcpyDeviceToHost) == hipSuccess);
        double rr = 0.0;
        for (int64_t i = 0; i < m; ++i) rr += (hb[i] - hy[i]) * (hb[i] - hy[i]);
        const double rel = sqrt(rr / bb);
        CHECK(fabs(rel - st.rel_res_true) <= 1e-6 * st.rel_res_true + 1e-15);
        printf("%s: %d iterations, true residual %.3e (host %.3e)\n", names[f], st.iterations, st.rel_res_true, rel);
    }

    /* refused calls: a negative tolerance, a mesh with no elements, a format not built */
    mfe_cg_stats st;
    CHECK(mfe_cg(P, MFE_BCRS13, x, -1.0, 10, NULL, &st) == MFE_EINVAL && mfe_last_error()[0] != '\0');
    mfe_problem *Q = NULL;
    CHECK(mfe_problem_create(ctx, 0, 4, 4, NULL, NULL, MFE_CSR, MFE_F64, &Q) == MFE_EINVAL && Q == NULL);
    CHECK(mfe_problem_create(ctx, 4, 4, 4, NULL, NULL, MFE_CSR, MFE_F64, &Q) == MFE_OK);
    if (Q) {
        CHECK(mfe_cg(Q, MFE_BCRS13, x, 1e-8, 10, NULL, &st) == MFE_EUNSUPPORTED);
        CHECK(mfe_problem_destroy(Q) == MFE_OK);
    }

    CHECK(hipFree(x) == hipSuccess && hipFree(b) == hipSuccess && hipFree(y) == hipSuccess);
    free(hb);
    free(hy);
    CHECK(mfe_problem_destroy(P) == MFE_OK);
    CHECK(mfe_ctx_destroy(ctx) == MFE_OK);
    if (fails) {
        fprintf(stderr, "%d checks failed\n", fails);
        return 1;
    }
    printf("C ABI: all checks passed\n");
    return 0;
}
