/* Test driver (test infrastructure, not part of the library): every routine of
 * the oracle (oracle/oracle.c, compiled into this program) on small meshes,
 * for a build with -fsanitize=address,undefined.  Besides the sanitizers'
 * own checks it asserts a few plain facts (formats agree, solvers converge),
 * so that a run that computes nonsense also fails.  Exit status 0 on success.
 */
#include "../oracle/oracle.c"

#include <stdio.h>

static int fails = 0;

#define CHECK(c)                                                                 \
    do {                                                                         \
        if (!(c)) {                                                              \
            fprintf(stderr, "check failed: %s (line %d)\n", #c, __LINE__);       \
            ++fails;                                                             \
        }                                                                        \
    } while (0)

static double max_abs_diff(int64_t m, const double *a, const double *b)
{
    double d = 0.0;
    for (int64_t i = 0; i < m; ++i) d = fmax(d, fabs(a[i] - b[i]));
    return d;
}

static void one_mesh(int Nx, int Ny, int Nz, const double *faces, int with_node_g)
{
    const int64_t m = orc_num_rows(Nx, Ny, Nz);
    const int64_t nnz = orc_count_nnz(Nx, Ny, Nz);
    double *node_g = NULL;
    if (with_node_g) {
        node_g = (double *)malloc((size_t)m * sizeof(double));
        for (int64_t i = 0; i < m; ++i) node_g[i] = 0.25 + 0.5 * (double)(i % 7) / 7.0;
    }
    uint8_t *dir = (uint8_t *)malloc((size_t)m);
    double *g = (double *)malloc((size_t)m * sizeof(double));
    orc_boundary(Nx, Ny, Nz, faces, node_g, dir, g);

    int64_t *ptr = (int64_t *)malloc((size_t)(m + 1) * sizeof(int64_t));
    int32_t *col = (int32_t *)malloc((size_t)nnz * sizeof(int32_t));
    double *val = (double *)malloc((size_t)nnz * sizeof(double));
    double *b = (double *)malloc((size_t)m * sizeof(double));
    CHECK(orc_assemble(Nx, Ny, Nz, faces, node_g, 1, ptr, col, val, b) == ORC_OK);
    CHECK(ptr[m] == nnz);

    /* selected rows agree with the whole assembly */
    const int64_t nr = m < 5 ? m : 5;
    int64_t rows[5];
    for (int64_t r = 0; r < nr; ++r) rows[r] = (r * 7919) % m;
    int32_t rc[5 * 27], cnt[5];
    double rv[5 * 27], rb[5];
    CHECK(orc_assemble_rows(Nx, Ny, Nz, faces, node_g, nr, rows, rc, rv, cnt, rb) == ORC_OK);
    for (int64_t r = 0; r < nr; ++r) {
        const int64_t i = rows[r];
        CHECK(cnt[r] == ptr[i + 1] - ptr[i]);
        for (int k = 0; k < cnt[r]; ++k) {
            CHECK(rc[27 * r + k] == col[ptr[i] + k]);
            CHECK(rv[27 * r + k] == val[ptr[i] + k]);
        }
        CHECK(rb[r] == b[i]);
    }

    /* every product format gives the CRS product */
    double *x = (double *)malloc((size_t)m * sizeof(double));
    double *y = (double *)malloc((size_t)m * sizeof(double));
    double *y2 = (double *)malloc((size_t)m * sizeof(double));
    for (int64_t i = 0; i < m; ++i) x[i] = sin(0.37 * (double)i);
    orc_csr_spmv(m, ptr, col, val, x, y);
    double scale = 0.0;
    for (int64_t k = 0; k < nnz; ++k) scale = fmax(scale, fabs(val[k]));
    const double eps = 64 * 2.3e-16 * (scale > 0 ? scale : 1.0);

    const int64_t nns = orc_bcrsvar_count(m, ptr, col);
    int32_t *jas = (int32_t *)malloc((size_t)(nns > 0 ? nns : 1) * sizeof(int32_t));
    int64_t *off = (int64_t *)malloc((size_t)(nns + 1) * sizeof(int64_t));
    int64_t *bp = (int64_t *)malloc((size_t)(m + 1) * sizeof(int64_t));
    orc_bcrsvar_build(m, ptr, col, jas, off, bp);
    CHECK(bp[m] == nns && off[nns] == nnz);
    orc_bcrsvar_spmv(m, bp, jas, off, val, x, y2);
    CHECK(max_abs_diff(m, y, y2) <= eps);
    orc_bcrsvar_spmv_switch(m, bp, jas, off, val, x, y2);
    CHECK(max_abs_diff(m, y, y2) <= eps);

    if (m >= 3) {
        const int64_t nb = orc_bcrs13_build(m, ptr, col, NULL, NULL, NULL, NULL);
        int64_t *bptr = (int64_t *)malloc((size_t)(m + 1) * sizeof(int64_t));
        int32_t *bcol = (int32_t *)malloc((size_t)nb * sizeof(int32_t));
        double *bval = (double *)malloc((size_t)(3 * nb) * sizeof(double));
        CHECK(orc_bcrs13_build(m, ptr, col, val, bptr, bcol, bval) == nb);
        orc_bcrs13_spmv(m, bptr, bcol, bval, x, y2);
        CHECK(max_abs_diff(m, y, y2) <= eps);
        free(bptr);
        free(bcol);
        free(bval);
    }

    /* the solvers: from zero, to 1e-9 (the mixed ones to 1e-10) */
    const int cap = 4000;
    double *hist = (double *)malloc((size_t)(cap + 1) * sizeof(double));
    int its = 0, outer = 0, inner = 0, fb = 0;
    double rr = 0.0, rt = 0.0;
    typedef int (*solver)(int64_t, const int64_t *, const int32_t *, const double *, const double *, double *,
                          double, int, int *, double *, double *, double *);
    const solver solvers[3] = {orc_cg, orc_cg_single_reduction, orc_cg_jacobi};
    for (int s = 0; s < 3; ++s) {
        memset(y, 0, (size_t)m * sizeof(double));
        const int st = solvers[s](m, ptr, col, val, b, y, 1e-9, cap, &its, &rr, &rt, hist);
        CHECK(st == ORC_OK && rt <= 1e-8);
    }
    memset(y, 0, (size_t)m * sizeof(double));
    CHECK(orc_cg_mixed(m, ptr, col, val, b, y, 1e-10, 1e-4, 50, cap, &outer, &inner, &rt) == ORC_OK);
    CHECK(rt <= 1e-9);
    for (int keep = 0; keep <= 1; ++keep)
        for (int f32 = 0; f32 <= 1; ++f32)
            for (int adaptive = 0; adaptive <= 1; ++adaptive) {
                memset(y, 0, (size_t)m * sizeof(double));
                const int st = orc_cg_mixed_keep(m, ptr, col, val, b, y, 1e-10, keep ? 1e-2 : 1e-4, 50, cap, keep,
                                                 f32, adaptive, 1, &outer, &inner, &fb, &rt);
                CHECK(st == ORC_OK && rt <= 1e-9);
            }
    /* a capped solve and a fallback: one inner iteration per step */
    memset(y, 0, (size_t)m * sizeof(double));
    (void)orc_cg(m, ptr, col, val, b, y, 1e-12, 2, &its, &rr, &rt, hist);
    CHECK(its <= 2);
    memset(y, 0, (size_t)m * sizeof(double));
    (void)orc_cg_mixed_keep(m, ptr, col, val, b, y, 1e-10, 1e-4, 50, 1, 0, 1, 1, 1, &outer, &inner, &fb, &rt);

    free(hist);
    free(jas);
    free(off);
    free(bp);
    free(x);
    free(y);
    free(y2);
    free(ptr);
    free(col);
    free(val);
    free(b);
    free(dir);
    free(g);
    free(node_g);
}

int main(void)
{
    static const double faces[6] = {0.2, 0.9, 0.1, 0.7, 0.3, 0.5};
    double K[64];
    orc_element_matrix(0.5, 0.25, 1.0 / 3.0, K);
    CHECK(fabs(orc_analytic_u(0.5, 0.5, 0.5, 41) - 1.0 / 6.0) < 1e-3);
    CHECK(orc_num_threads() >= 1);
    CHECK(orc_assemble(0, 1, 1, NULL, NULL, 1, NULL, NULL, NULL, NULL) == ORC_EINVAL);
    const int meshes[6][3] = {{1, 1, 1}, {2, 2, 2}, {2, 3, 4}, {5, 3, 7}, {6, 6, 6}, {9, 4, 5}};
    for (int k = 0; k < 6; ++k) {
        one_mesh(meshes[k][0], meshes[k][1], meshes[k][2], NULL, 0);
        one_mesh(meshes[k][0], meshes[k][1], meshes[k][2], faces, 0);
        one_mesh(meshes[k][0], meshes[k][1], meshes[k][2], NULL, 1);
    }
    if (fails) {
        fprintf(stderr, "%d checks failed\n", fails);
        return 1;
    }
    printf("oracle sanitizer driver: all checks passed\n");
    return 0;
}
