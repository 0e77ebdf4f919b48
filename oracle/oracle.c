/*
 * Plain FP64 CPU oracle for the MiniFE-style finite-element method of
 * "The Research and Optimization of Parallel Finite Element Algorithm based
 * on MiniFE" (Wu, Yang, Xiang, Cheng).
 *
 * TEST INFRASTRUCTURE ONLY.  This file is the slow, obviously-correct
 * statement of what the GPU library computes.  Only the test-suite, the
 * smoke check and the CPU-baseline leg of the benchmark load it.  It shares
 * no code, header, table or constant generator with the HIP library and
 * neither side includes or links the other.
 *
 * Build: gcc -O2 -ffp-contract=off -fPIC -shared oracle.c -lm
 *   (-ffp-contract=off keeps every a*b+c as two roundings, so the CSR and
 *   BCRS loops below produce identical sums.)
 *
 * Contents, each following the passage named at the function:
 *   mesh numbering and boundary values      (Sec. 1 problem statement)
 *   trilinear hexahedron element operator   (Sec. 1, element operator)
 *   CRS structure generation                (Sec. 3.2, Fig 3.6 loop)
 *   element-by-element assembly             (Sec. 1 assembly, Fig 3.7)
 *   Dirichlet elimination                   (Sec. 1 boundary values)
 *   CRS SpMV                                (Sec. 3.1, Fig 3.1)
 *   variable 1xn BCRS build + SpMV          (Sec. 3.1, Fig 3.2, Fig 3.3)
 *   fixed 1x3 zero-padded BCRS build + SpMV (derived from Sec. 3.1)
 *   unpreconditioned CG                     (Sec. 1, CG module)
 *   FP32-inner / FP64-refinement CG         (mixed-precision extension)
 *   single-reduction CG                     (Chronopoulos-Gear form of the CG
 *                                            module; Sec. 3, Fig 3.5 discussion)
 *   Jacobi-preconditioned CG                (comparison variant of the CG module)
 *   separation-of-variables series solution (Sec. 1, result verification)
 *
 * Conventions (readings of passages where the paper is silent):
 *   - Node (ix,iy,iz), 0<=ix<=Nx etc., id = ix + nx*(iy + ny*iz) with
 *     nx=Nx+1, ny=Ny+1: x varies fastest.  This is the order in which the
 *     Fig 3.6 neighbour loop (sz outer, sx inner) produces ascending columns.
 *   - Coordinates ix/Nx, iy/Ny, iz/Nz on the unit cube.
 *   - Zero source term.  Every node on the cube's surface is a Dirichlet
 *     node.  A node on several faces takes the value of the first face in
 *     the order x=1, x=0, y=1, y=0, z=1, z=0.
 *   - Dirichlet rows are eliminated symmetrically: for a free row i and a
 *     Dirichlet column j, b_i -= A_ij g_j and A_ij = 0; a Dirichlet row is
 *     the identity row with b_i = g_i.  Structural entries stay stored.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

/* The benchmark's CPU baseline also times this file built with -fopenmp:
 * the row loops of the CRS and 1x3 BCRS products and the vector loops and
 * dot products of orc_cg then run over the host's cores (the dots' partial sums combined in
 * OpenMP's reduction order).  The plain build, the oracle, ignores these
 * annotations: single-threaded, every sum in the order stated. */
#define ORC_PRAGMA(x) _Pragma(#x)
#ifdef _OPENMP
#include <omp.h>
#define ORC_PARALLEL_FOR ORC_PRAGMA(omp parallel for schedule(static))
#define ORC_PARALLEL_SUM(v) ORC_PRAGMA(omp parallel for schedule(static) reduction(+ : v))
#else
#define ORC_PARALLEL_FOR
#define ORC_PARALLEL_SUM(v)
#endif

/* Threads a parallel loop of this build uses (1 for the plain build). */
int orc_num_threads(void)
{
#ifdef _OPENMP
    return omp_get_max_threads();
#else
    return 1;
#endif
}

#define ORC_OK 0
#define ORC_NOT_CONVERGED 1
#define ORC_EINVAL (-1)
#define ORC_ENOMEM (-2)
#define ORC_BREAKDOWN (-4)

/* ------------------------------------------------------------------ */
/* Mesh (Sec. 1: unit box, Nx x Ny x Nz hexahedral elements)            */
/* ------------------------------------------------------------------ */

int64_t orc_num_rows(int Nx, int Ny, int Nz)
{
    return (int64_t)(Nx + 1) * (Ny + 1) * (Nz + 1);
}

/* Node id of (ix,iy,iz), or -1 when the node lies outside the box (the
 * range test of the Fig 3.6 loop). */
static int64_t node_id(int Nx, int Ny, int Nz, int ix, int iy, int iz)
{
    if (ix < 0 || ix > Nx || iy < 0 || iy > Ny || iz < 0 || iz > Nz)
        return -1;
    return (int64_t)ix + (int64_t)(Nx + 1) * ((int64_t)iy + (int64_t)(Ny + 1) * iz);
}

/* Boundary value of node (ix,iy,iz): returns 1 and sets *g for a boundary
 * node, 0 for an interior node.  face_vals = {x0,x1,y0,y1,z0,z1}; NULL means
 * the paper's problem {0,1,0,0,0,0}.  When node_g is given, the value of a
 * boundary node is node_g[id] instead (face_vals then unused). */
static int boundary_of(int Nx, int Ny, int Nz, const double *face_vals, const double *node_g,
                       int ix, int iy, int iz, double *g)
{
    static const double paper_faces[6] = {0.0, 1.0, 0.0, 0.0, 0.0, 0.0};
    const double *f = face_vals ? face_vals : paper_faces;
    double v;
    /* first face in the order x=1, x=0, y=1, y=0, z=1, z=0 */
    if (ix == Nx) v = f[1];
    else if (ix == 0) v = f[0];
    else if (iy == Ny) v = f[3];
    else if (iy == 0) v = f[2];
    else if (iz == Nz) v = f[5];
    else if (iz == 0) v = f[4];
    else return 0;
    if (node_g) v = node_g[node_id(Nx, Ny, Nz, ix, iy, iz)];
    *g = v;
    return 1;
}

/* Boundary flag and value of every node (g = 0 for interior nodes). */
void orc_boundary(int Nx, int Ny, int Nz, const double *face_vals,
                  const double *node_g, uint8_t *is_dir, double *g)
{
    for (int iz = 0; iz <= Nz; ++iz)
        for (int iy = 0; iy <= Ny; ++iy)
            for (int ix = 0; ix <= Nx; ++ix) {
                int64_t id = node_id(Nx, Ny, Nz, ix, iy, iz);
                double v = 0.0;
                is_dir[id] = (uint8_t)boundary_of(Nx, Ny, Nz, face_vals, node_g, ix, iy, iz, &v);
                g[id] = v;
            }
}

/* ------------------------------------------------------------------ */
/* Element operator (Sec. 1, "element equation system")                */
/* ------------------------------------------------------------------ */

/* 8x8 stiffness of one brick of sides hx,hy,hz for the Laplacian with
 * trilinear shape functions, K_ab = integral of grad N_a . grad N_b, by
 * 2x2x2 Gauss-Legendre quadrature on the reference cube [-1,1]^3 (exact for
 * this integrand on a brick).  Local node a = a0 + 2 a1 + 4 a2 sits at
 * reference corner (2a0-1, 2a1-1, 2a2-1).  The upper triangle is computed
 * and mirrored so that K is exactly symmetric. */
void orc_element_matrix(double hx, double hy, double hz, double *K)
{
    const double gp = 1.0 / sqrt(3.0);
    const double pts[2] = {-gp, gp};
    const double jx = 2.0 / hx, jy = 2.0 / hy, jz = 2.0 / hz; /* d(xi)/dx */
    const double detJ = hx * hy * hz / 8.0;
    for (int i = 0; i < 64; ++i) K[i] = 0.0;
    for (int qz = 0; qz < 2; ++qz)
        for (int qy = 0; qy < 2; ++qy)
            for (int qx = 0; qx < 2; ++qx) {
                double xi = pts[qx], eta = pts[qy], zeta = pts[qz];
                double dN[8][3];
                for (int a = 0; a < 8; ++a) {
                    double sa = (a & 1) ? 1.0 : -1.0;
                    double ta = (a & 2) ? 1.0 : -1.0;
                    double ua = (a & 4) ? 1.0 : -1.0;
                    /* N_a = (1+sa xi)(1+ta eta)(1+ua zeta)/8 */
                    dN[a][0] = sa * (1.0 + ta * eta) * (1.0 + ua * zeta) / 8.0 * jx;
                    dN[a][1] = (1.0 + sa * xi) * ta * (1.0 + ua * zeta) / 8.0 * jy;
                    dN[a][2] = (1.0 + sa * xi) * (1.0 + ta * eta) * ua / 8.0 * jz;
                }
                for (int a = 0; a < 8; ++a)
                    for (int b = a; b < 8; ++b) {
                        double d = dN[a][0] * dN[b][0] + dN[a][1] * dN[b][1] + dN[a][2] * dN[b][2];
                        K[a * 8 + b] += d * detJ; /* Gauss weights are 1 */
                    }
            }
    for (int a = 0; a < 8; ++a)
        for (int b = 0; b < a; ++b) K[a * 8 + b] = K[b * 8 + a];
}

/* ------------------------------------------------------------------ */
/* Matrix generation: CRS structure (Sec. 3.2, Fig 3.6)                */
/* ------------------------------------------------------------------ */

/* Number of stored entries: every in-range node of the 27-neighbourhood of
 * every row, counted by running the neighbour loop. */
int64_t orc_count_nnz(int Nx, int Ny, int Nz)
{
    int64_t nnz = 0;
    for (int iz = 0; iz <= Nz; ++iz)
        for (int iy = 0; iy <= Ny; ++iy)
            for (int ix = 0; ix <= Nx; ++ix)
                for (int sz = -1; sz <= 1; ++sz)
                    for (int sy = -1; sy <= 1; ++sy)
                        for (int sx = -1; sx <= 1; ++sx)
                            if (node_id(Nx, Ny, Nz, ix + sx, iy + sy, iz + sz) >= 0) ++nnz;
    return nnz;
}

/* Fill ptr[m+1] and col[nnz] (ascending columns per row, structural zeros
 * kept).  val is zeroed. */
static void build_structure(int Nx, int Ny, int Nz, int64_t *ptr, int32_t *col, double *val)
{
    int64_t k = 0, row = 0;
    for (int iz = 0; iz <= Nz; ++iz)
        for (int iy = 0; iy <= Ny; ++iy)
            for (int ix = 0; ix <= Nx; ++ix) {
                ptr[row++] = k;
                for (int sz = -1; sz <= 1; ++sz)
                    for (int sy = -1; sy <= 1; ++sy)
                        for (int sx = -1; sx <= 1; ++sx) {
                            int64_t c = node_id(Nx, Ny, Nz, ix + sx, iy + sy, iz + sz);
                            if (c >= 0) { col[k] = (int32_t)c; val[k] = 0.0; ++k; }
                        }
            }
    ptr[row] = k;
}

/* Position of column c in row r (linear search), or -1. */
static int64_t find_entry(const int64_t *ptr, const int32_t *col, int64_t r, int64_t c)
{
    for (int64_t k = ptr[r]; k < ptr[r + 1]; ++k)
        if (col[k] == c) return k;
    return -1;
}

/* ------------------------------------------------------------------ */
/* Assembly (Sec. 1 assembly module, Fig 3.7) + Dirichlet elimination   */
/* ------------------------------------------------------------------ */

/* Assemble A (CRS) and b for the box problem.  Arrays are caller-owned:
 * ptr[m+1], col[nnz], val[nnz], b[m] with nnz = orc_count_nnz().
 * apply_bc = 0 returns the raw stiffness matrix and a zero b.
 * Returns ORC_OK, or ORC_EINVAL for a non-positive size. */
int orc_assemble(int Nx, int Ny, int Nz, const double *face_vals, const double *node_g,
                 int apply_bc, int64_t *ptr, int32_t *col, double *val, double *b)
{
    if (Nx < 1 || Ny < 1 || Nz < 1) return ORC_EINVAL;
    const int64_t m = orc_num_rows(Nx, Ny, Nz);
    build_structure(Nx, Ny, Nz, ptr, col, val);
    for (int64_t i = 0; i < m; ++i) b[i] = 0.0; /* zero source: element loads vanish */

    double K[64];
    orc_element_matrix(1.0 / Nx, 1.0 / Ny, 1.0 / Nz, K); /* every element is the same brick */
    /* element loop in ascending element id ex + Nx*(ey + Ny*ez) */
    for (int ez = 0; ez < Nz; ++ez)
        for (int ey = 0; ey < Ny; ++ey)
            for (int ex = 0; ex < Nx; ++ex) {
                int64_t nodes[8];
                for (int a = 0; a < 8; ++a)
                    nodes[a] = node_id(Nx, Ny, Nz, ex + (a & 1), ey + ((a >> 1) & 1), ez + ((a >> 2) & 1));
                for (int a = 0; a < 8; ++a)
                    for (int bb = 0; bb < 8; ++bb) {
                        int64_t k = find_entry(ptr, col, nodes[a], nodes[bb]);
                        val[k] += K[a * 8 + bb];
                    }
            }
    if (!apply_bc) return ORC_OK;

    uint8_t *dir = (uint8_t *)malloc((size_t)m);
    double *g = (double *)malloc((size_t)m * sizeof(double));
    if (!dir || !g) { free(dir); free(g); return ORC_ENOMEM; }
    orc_boundary(Nx, Ny, Nz, face_vals, node_g, dir, g);
    for (int64_t i = 0; i < m; ++i) {
        if (dir[i]) {
            for (int64_t k = ptr[i]; k < ptr[i + 1]; ++k) val[k] = (col[k] == i) ? 1.0 : 0.0;
            b[i] = g[i];
        } else {
            for (int64_t k = ptr[i]; k < ptr[i + 1]; ++k)
                if (dir[col[k]]) { b[i] -= val[k] * g[col[k]]; val[k] = 0.0; }
        }
    }
    free(dir);
    free(g);
    return ORC_OK;
}

/* Selected rows of the same assembled system, one at a time, for checks on
 * meshes too large to assemble whole.  Row i is built exactly as in
 * orc_assemble: element contributions in ascending element order, then the
 * Dirichlet elimination of that row.  For rows[r], cols/vals[27*r ..] get the
 * row's entries in ascending column order, counts[r] their number, b[r] the
 * right-hand side. */
int orc_assemble_rows(int Nx, int Ny, int Nz, const double *face_vals, const double *node_g,
                      int64_t nrows, const int64_t *rows, int32_t *cols, double *vals,
                      int32_t *counts, double *b)
{
    if (Nx < 1 || Ny < 1 || Nz < 1) return ORC_EINVAL;
    const int64_t m = orc_num_rows(Nx, Ny, Nz);
    double K[64];
    orc_element_matrix(1.0 / Nx, 1.0 / Ny, 1.0 / Nz, K);
    for (int64_t r = 0; r < nrows; ++r) {
        int64_t i = rows[r];
        if (i < 0 || i >= m) return ORC_EINVAL;
        int ix = (int)(i % (Nx + 1)), iy = (int)((i / (Nx + 1)) % (Ny + 1));
        int iz = (int)(i / ((int64_t)(Nx + 1) * (Ny + 1)));
        int32_t *c = cols + 27 * r;
        double *v = vals + 27 * r;
        int n = 0;
        for (int sz = -1; sz <= 1; ++sz)          /* structure: Fig 3.6 loop */
            for (int sy = -1; sy <= 1; ++sy)
                for (int sx = -1; sx <= 1; ++sx) {
                    int64_t j = node_id(Nx, Ny, Nz, ix + sx, iy + sy, iz + sz);
                    if (j >= 0) { c[n] = (int32_t)j; v[n] = 0.0; ++n; }
                }
        counts[r] = n;
        for (int ez = iz - 1; ez <= iz; ++ez)     /* elements holding node i, ascending id */
            for (int ey = iy - 1; ey <= iy; ++ey)
                for (int ex = ix - 1; ex <= ix; ++ex) {
                    if (ex < 0 || ex >= Nx || ey < 0 || ey >= Ny || ez < 0 || ez >= Nz) continue;
                    int a = (ix - ex) + 2 * (iy - ey) + 4 * (iz - ez);
                    for (int bb = 0; bb < 8; ++bb) {
                        int64_t j = node_id(Nx, Ny, Nz, ex + (bb & 1), ey + ((bb >> 1) & 1), ez + ((bb >> 2) & 1));
                        for (int k = 0; k < n; ++k)
                            if (c[k] == j) { v[k] += K[a * 8 + bb]; break; }
                    }
                }
        double gi, bi = 0.0;
        if (boundary_of(Nx, Ny, Nz, face_vals, node_g, ix, iy, iz, &gi)) {
            for (int k = 0; k < n; ++k) v[k] = (c[k] == i) ? 1.0 : 0.0;
            bi = gi;
        } else {
            for (int k = 0; k < n; ++k) {
                int64_t j = c[k];
                int jx = (int)(j % (Nx + 1)), jy = (int)((j / (Nx + 1)) % (Ny + 1));
                int jz = (int)(j / ((int64_t)(Nx + 1) * (Ny + 1)));
                double gj;
                if (boundary_of(Nx, Ny, Nz, face_vals, node_g, jx, jy, jz, &gj)) { bi -= v[k] * gj; v[k] = 0.0; }
            }
        }
        b[r] = bi;
    }
    return ORC_OK;
}

/* ------------------------------------------------------------------ */
/* SpMV, CRS (Sec. 3.1, Fig 3.1)                                       */
/* ------------------------------------------------------------------ */

void orc_csr_spmv(int64_t m, const int64_t *ptr, const int32_t *col, const double *val,
                  const double *x, double *y)
{
    ORC_PARALLEL_FOR
    for (int64_t i = 0; i < m; ++i) {
        double s = 0.0;
        for (int64_t j = ptr[i]; j < ptr[i + 1]; ++j) s += val[j] * x[col[j]];
        y[i] = s;
    }
}

/* ------------------------------------------------------------------ */
/* BCRS with 1xn blocks of variable n (Sec. 3.1, Figs 3.2, 3.3)        */
/* ------------------------------------------------------------------ */

/* Number of non-zero segments: maximal runs of consecutive stored columns. */
int64_t orc_bcrsvar_count(int64_t m, const int64_t *ptr, const int32_t *col)
{
    int64_t nns = 0;
    for (int64_t i = 0; i < m; ++i)
        for (int64_t k = ptr[i]; k < ptr[i + 1]; ++k)
            if (k == ptr[i] || col[k] != col[k - 1] + 1) ++nns;
    return nns;
}

/* val is the CRS val unchanged (segments keep their entries in order);
 * jas[nns] first column of each segment, offsets[nns+1] start of each
 * segment in val, bptr[m+1] first segment of each row. */
void orc_bcrsvar_build(int64_t m, const int64_t *ptr, const int32_t *col,
                       int32_t *jas, int64_t *offsets, int64_t *bptr)
{
    int64_t s = 0;
    for (int64_t i = 0; i < m; ++i) {
        bptr[i] = s;
        for (int64_t k = ptr[i]; k < ptr[i + 1]; ++k)
            if (k == ptr[i] || col[k] != col[k - 1] + 1) {
                jas[s] = col[k];
                offsets[s] = k;
                ++s;
            }
    }
    bptr[m] = s;
    offsets[s] = ptr[m];
}

/* Fig 3.2: a segment is a run of val times consecutive x. */
void orc_bcrsvar_spmv(int64_t m, const int64_t *bptr, const int32_t *jas, const int64_t *offsets,
                      const double *val, const double *x, double *y)
{
    for (int64_t i = 0; i < m; ++i) {
        double s = 0.0;
        for (int64_t j = bptr[i]; j < bptr[i + 1]; ++j) {
            int64_t c = jas[j];
            for (int64_t k = offsets[j]; k < offsets[j + 1]; ++k) s += val[k] * x[c++];
        }
        y[i] = s;
    }
}

/* Fig 3.3: the segment loop unrolled by length, length 3 tested first.  A
 * run longer than 4 (possible only for Nx <= 2, where x-lines merge) falls
 * back to the plain loop. */
void orc_bcrsvar_spmv_switch(int64_t m, const int64_t *bptr, const int32_t *jas,
                             const int64_t *offsets, const double *val, const double *x, double *y)
{
    for (int64_t i = 0; i < m; ++i) {
        double s = 0.0;
        for (int64_t j = bptr[i]; j < bptr[i + 1]; ++j) {
            int64_t c = jas[j], n = offsets[j];
            int64_t len = offsets[j + 1] - n;
            switch (len) {
            case 3:
                s += val[n] * x[c]; s += val[n + 1] * x[c + 1]; s += val[n + 2] * x[c + 2];
                break;
            case 1:
                s += val[n] * x[c];
                break;
            case 2:
                s += val[n] * x[c]; s += val[n + 1] * x[c + 1];
                break;
            case 4:
                s += val[n] * x[c]; s += val[n + 1] * x[c + 1];
                s += val[n + 2] * x[c + 2]; s += val[n + 3] * x[c + 3];
                break;
            default:
                for (int64_t k = 0; k < len; ++k) s += val[n + k] * x[c + k];
            }
        }
        y[i] = s;
    }
}

/* ------------------------------------------------------------------ */
/* Fixed 1x3 BCRS, zero padded (the segment format with n fixed to 3)   */
/* ------------------------------------------------------------------ */

/* Greedy blocks per row: a block starts at the first stored column c not yet
 * covered (moved back to m-3 when c > m-3) and covers c, c+1, c+2.  A slot
 * holds the stored value of its column when that column is stored and not
 * covered by an earlier block of the row, else 0.  Returns the block count;
 * with bptr/bcol/bval non-NULL also fills them (bptr[m+1], bcol[nb],
 * bval[3*nb]). */
int64_t orc_bcrs13_build(int64_t m, const int64_t *ptr, const int32_t *col, const double *val,
                         int64_t *bptr, int32_t *bcol, double *bval)
{
    int64_t nb = 0;
    for (int64_t i = 0; i < m; ++i) {
        if (bptr) bptr[i] = nb;
        int64_t k = ptr[i];
        while (k < ptr[i + 1]) {
            int64_t c = col[k];
            if (c > m - 3) c = m - 3;
            if (bcol) {
                bcol[nb] = (int32_t)c;
                bval[3 * nb] = bval[3 * nb + 1] = bval[3 * nb + 2] = 0.0;
            }
            /* consume stored entries that fall in [c, c+2] */
            while (k < ptr[i + 1] && col[k] <= c + 2) {
                if (bval) bval[3 * nb + (col[k] - c)] = val[k];
                ++k;
            }
            ++nb;
        }
    }
    if (bptr) bptr[m] = nb;
    return nb;
}

void orc_bcrs13_spmv(int64_t m, const int64_t *bptr, const int32_t *bcol, const double *bval,
                     const double *x, double *y)
{
    ORC_PARALLEL_FOR
    for (int64_t i = 0; i < m; ++i) {
        double s = 0.0;
        for (int64_t j = bptr[i]; j < bptr[i + 1]; ++j) {
            int64_t c = bcol[j];
            s += bval[3 * j] * x[c];
            s += bval[3 * j + 1] * x[c + 1];
            s += bval[3 * j + 2] * x[c + 2];
        }
        y[i] = s;
    }
}

/* ------------------------------------------------------------------ */
/* Vector operations (Sec. 1 CG module: DOT and WAXPY)                 */
/* ------------------------------------------------------------------ */

static double dot(int64_t m, const double *a, const double *b)
{
    double s = 0.0;
    ORC_PARALLEL_SUM(s)
    for (int64_t i = 0; i < m; ++i) s += a[i] * b[i];
    return s;
}

/* ------------------------------------------------------------------ */
/* Unpreconditioned conjugate gradient (Sec. 1, CG module)              */
/* ------------------------------------------------------------------ */

/* Hestenes-Stiefel CG on A x = b from the x given on entry.
 * Stop when ||r||_2 / ||b||_2 <= tol with r the recurrence residual; the
 * iteration count is the number of SpMVs inside the loop.
 * hist (optional, max_iter+1 entries) receives ||r_k||/||b|| for k=0..its.
 * res_true receives ||b - A x||/||b|| at exit.
 * Returns ORC_OK, ORC_NOT_CONVERGED (cap reached), ORC_BREAKDOWN (p.Ap <= 0
 * or not finite: x holds the last iterate) or ORC_ENOMEM. */
int orc_cg(int64_t m, const int64_t *ptr, const int32_t *col, const double *val,
           const double *b, double *x, double tol, int max_iter,
           int *iters, double *res_rec, double *res_true, double *hist)
{
    double *r = (double *)malloc((size_t)m * sizeof(double));
    double *p = (double *)malloc((size_t)m * sizeof(double));
    double *q = (double *)malloc((size_t)m * sizeof(double));
    if (!r || !p || !q) { free(r); free(p); free(q); return ORC_ENOMEM; }
    int status = ORC_NOT_CONVERGED, k = 0;

    orc_csr_spmv(m, ptr, col, val, x, q);
    ORC_PARALLEL_FOR
    for (int64_t i = 0; i < m; ++i) { r[i] = b[i] - q[i]; p[i] = r[i]; }
    double rho = dot(m, r, r);
    double bnorm = sqrt(dot(m, b, b));
    if (bnorm == 0.0) {
        for (int64_t i = 0; i < m; ++i) x[i] = 0.0;
        *iters = 0; *res_rec = 0.0; *res_true = 0.0;
        if (hist) hist[0] = 0.0;
        free(r); free(p); free(q);
        return ORC_OK;
    }
    if (hist) hist[0] = sqrt(rho) / bnorm;
    if (sqrt(rho) / bnorm <= tol) status = ORC_OK;
    while (status == ORC_NOT_CONVERGED && k < max_iter) {
        orc_csr_spmv(m, ptr, col, val, p, q);
        double pq = dot(m, p, q);
        if (!(pq > 0.0) || !isfinite(pq)) { status = ORC_BREAKDOWN; break; }
        double alpha = rho / pq;
        ORC_PARALLEL_FOR
        for (int64_t i = 0; i < m; ++i) x[i] += alpha * p[i];
        ORC_PARALLEL_FOR
        for (int64_t i = 0; i < m; ++i) r[i] -= alpha * q[i];
        double rho_new = dot(m, r, r);
        ++k;
        if (hist) hist[k] = sqrt(rho_new) / bnorm;
        if (sqrt(rho_new) / bnorm <= tol) { rho = rho_new; status = ORC_OK; break; }
        double beta = rho_new / rho;
        ORC_PARALLEL_FOR
        for (int64_t i = 0; i < m; ++i) p[i] = r[i] + beta * p[i];
        rho = rho_new;
    }
    *iters = k;
    *res_rec = sqrt(rho) / bnorm;
    orc_csr_spmv(m, ptr, col, val, x, q);
    for (int64_t i = 0; i < m; ++i) r[i] = b[i] - q[i];
    *res_true = sqrt(dot(m, r, r)) / bnorm;
    free(r); free(p); free(q);
    return status;
}

/* ------------------------------------------------------------------ */
/* Mixed precision: FP32 inner CG inside FP64 iterative refinement      */
/* ------------------------------------------------------------------ */

static void csr_spmv_f32(int64_t m, const int64_t *ptr, const int32_t *col, const float *val,
                         const float *x, float *y)
{
    for (int64_t i = 0; i < m; ++i) {
        float s = 0.0f;
        for (int64_t j = ptr[i]; j < ptr[i + 1]; ++j) s += val[j] * x[col[j]];
        y[i] = s;
    }
}

/* FP64 accumulation of a product of two FP32 vectors. */
static double dot_f32(int64_t m, const float *a, const float *b)
{
    double s = 0.0;
    for (int64_t i = 0; i < m; ++i) s += (double)a[i] * (double)b[i];
    return s;
}

/* Outer loop (FP64): r = b - A x; stop when ||r||/||b|| <= tol; s = ||r||;
 * solve A32 d = fl32(r/s) by FP32 CG from d = 0 to relative residual
 * inner_tol (or max_inner steps); x += s * d.
 * Inner CG: FP32 matrix, FP32 SpMV sum, FP32 vector updates with alpha and
 * beta rounded to FP32; the two dot products accumulate in FP64 and alpha,
 * beta are formed in FP64.
 * outer = number of inner solves, inner_total = sum of inner iterations.
 * Returns ORC_OK, ORC_NOT_CONVERGED, ORC_BREAKDOWN or ORC_ENOMEM. */
int orc_cg_mixed(int64_t m, const int64_t *ptr, const int32_t *col, const double *val,
                 const double *b, double *x, double tol, double inner_tol,
                 int max_outer, int max_inner, int *outer, int *inner_total, double *res_true)
{
    int64_t nnz = ptr[m];
    float *v32 = (float *)malloc((size_t)nnz * sizeof(float));
    double *r = (double *)malloc((size_t)m * sizeof(double));
    double *ax = (double *)malloc((size_t)m * sizeof(double));
    float *r32 = (float *)malloc((size_t)m * sizeof(float));
    float *d = (float *)malloc((size_t)m * sizeof(float));
    float *p = (float *)malloc((size_t)m * sizeof(float));
    float *q = (float *)malloc((size_t)m * sizeof(float));
    int status = ORC_NOT_CONVERGED;
    if (!v32 || !r || !ax || !r32 || !d || !p || !q) { status = ORC_ENOMEM; goto out; }
    for (int64_t k = 0; k < nnz; ++k) v32[k] = (float)val[k];
    double bnorm = sqrt(dot(m, b, b));
    *outer = 0; *inner_total = 0;
    if (bnorm == 0.0) {
        for (int64_t i = 0; i < m; ++i) x[i] = 0.0;
        *res_true = 0.0; status = ORC_OK; goto out;
    }
    for (;;) {
        orc_csr_spmv(m, ptr, col, val, x, ax);
        for (int64_t i = 0; i < m; ++i) r[i] = b[i] - ax[i];
        double s = sqrt(dot(m, r, r));
        *res_true = s / bnorm;
        if (s / bnorm <= tol) { status = ORC_OK; break; }
        if (*outer >= max_outer) { status = ORC_NOT_CONVERGED; break; }
        for (int64_t i = 0; i < m; ++i) { r32[i] = (float)(r[i] / s); d[i] = 0.0f; p[i] = r32[i]; }
        double rho = dot_f32(m, r32, r32), rho0 = rho;
        int k = 0;
        while (k < max_inner) {
            csr_spmv_f32(m, ptr, col, v32, p, q);
            double pq = dot_f32(m, p, q);
            if (!(pq > 0.0) || !isfinite(pq)) { status = ORC_BREAKDOWN; break; }
            float a = (float)(rho / pq);
            for (int64_t i = 0; i < m; ++i) d[i] += a * p[i];
            for (int64_t i = 0; i < m; ++i) r32[i] -= a * q[i];
            double rho_new = dot_f32(m, r32, r32);
            ++k;
            if (sqrt(rho_new / rho0) <= inner_tol) break;
            float be = (float)(rho_new / rho);
            for (int64_t i = 0; i < m; ++i) p[i] = r32[i] + be * p[i];
            rho = rho_new;
        }
        *inner_total += k;
        *outer += 1;
        if (status == ORC_BREAKDOWN) break;
        for (int64_t i = 0; i < m; ++i) x[i] += s * (double)d[i];
    }
out:
    free(v32); free(r); free(ax); free(r32); free(d); free(p); free(q);
    return status;
}

/* Rounding of the inner solve of orc_cg_mixed_keep: to FP32 when f32 != 0,
 * none otherwise.  Each FP32 operation there is the FP64 operation on FP32
 * operands followed by this rounding; for +, - and x that double rounding is
 * innocuous (FP64 carries more than 2 x 24 + 2 significand bits), so the
 * result is the FP32 operation's own. */
static double rnd(int f32, double v) { return f32 ? (double)(float)v : v; }

/* Refinement that keeps the inner CG's search direction from one step to
 * the next instead of restarting it: the inner residual is replaced by the
 * FP64 residual of the refinement step (a reliable update of the residual,
 * after Sleijpen and van der Vorst, 1996), and the inner recurrence goes on.
 * As orc_cg_mixed, except after an inner solve that met its tolerance: with
 * s_old and s the norms of the previous and the new FP64 residual r, beta
 * and P the last inner step's beta = rho_new / rho and direction,
 *     r_inner = fl(r / s),   p = r_inner + fl(beta s_old / s) P,
 * i.e. the CG step P_next = R + beta P in the new scale, with the FP64
 * residual for R.  After a capped inner solve, or with keep = 0, the inner
 * CG restarts from p = r_inner.
 * f32 = 1: the inner solve in FP32 as in orc_cg_mixed (with keep = 0 this
 * computes what orc_cg_mixed computes); f32 = 0: the same steps in FP64 with
 * the FP64 matrix.  In exact arithmetic the FP64 residual equals the
 * recursive one, so keep = 1 then takes the iterates of plain CG.
 *
 * Two safeguards of the refinement (a reading: the method fixes neither):
 *   adaptive = 1: an inner solve need not reduce its residual further than
 *     the outer target asks.  With s the norm of the residual it starts
 *     from, its relative tolerance is max(inner_tol, min(0.5, tol ||b|| /
 *     (2 s))): on the last refinement step usually much looser than
 *     inner_tol.
 *   fallback = 1: a refinement step whose new FP64 residual is not at most
 *     half the previous one (while the outer tolerance is not met), or an
 *     inner breakdown, ends the refinement; plain FP64 CG (orc_cg) then
 *     continues from the current x to tol, capped at max_inner * max_outer
 *     iterations, and its status is the result.  *fallback_its receives its
 *     iteration count (0 when it did not run); *res_true its true residual.
 * Returns as orc_cg_mixed. */
int orc_cg_mixed_keep(int64_t m, const int64_t *ptr, const int32_t *col, const double *val,
                      const double *b, double *x, double tol, double inner_tol, int max_outer,
                      int max_inner, int keep, int f32, int adaptive, int fallback,
                      int *outer, int *inner_total, int *fallback_its, double *res_true)
{
    int64_t nnz = ptr[m];
    double *vi = (double *)malloc((size_t)nnz * sizeof(double));
    double *r = (double *)malloc((size_t)m * sizeof(double));
    double *ax = (double *)malloc((size_t)m * sizeof(double));
    double *ri = (double *)malloc((size_t)m * sizeof(double));
    double *d = (double *)malloc((size_t)m * sizeof(double));
    double *p = (double *)malloc((size_t)m * sizeof(double));
    double *q = (double *)malloc((size_t)m * sizeof(double));
    int status = ORC_NOT_CONVERGED;
    if (!vi || !r || !ax || !ri || !d || !p || !q) { status = ORC_ENOMEM; goto out; }
    for (int64_t k = 0; k < nnz; ++k) vi[k] = rnd(f32, val[k]);
    double bnorm = sqrt(dot(m, b, b));
    *outer = 0; *inner_total = 0;
    if (bnorm == 0.0) {
        for (int64_t i = 0; i < m; ++i) x[i] = 0.0;
        *res_true = 0.0; status = ORC_OK; goto out;
    }
    int have_dir = 0, go_fp64 = 0;
    double beta = 0.0, s_old = 0.0, s_prev = -1.0;
    *fallback_its = 0;
    for (;;) {
        orc_csr_spmv(m, ptr, col, val, x, ax);
        for (int64_t i = 0; i < m; ++i) r[i] = b[i] - ax[i];
        double s = sqrt(dot(m, r, r));
        *res_true = s / bnorm;
        if (s / bnorm <= tol) { status = ORC_OK; break; }
        if (fallback && s_prev >= 0.0 && !(s <= 0.5 * s_prev)) { go_fp64 = 1; break; }
        if (*outer >= max_outer) { status = ORC_NOT_CONVERGED; break; }
        s_prev = s;
        double itol = inner_tol;
        if (adaptive) {
            double need = tol * bnorm / (2.0 * s);
            if (need > itol) itol = need < 0.5 ? need : 0.5;
        }
        const double c = rnd(f32, beta * (s_old / s));
        for (int64_t i = 0; i < m; ++i) {
            ri[i] = rnd(f32, r[i] / s);
            d[i] = 0.0;
            p[i] = (keep && have_dir) ? rnd(f32, ri[i] + rnd(f32, c * p[i])) : ri[i];
        }
        double rho = dot(m, ri, ri), rho0 = rho;
        int k = 0;
        have_dir = 0;
        while (k < max_inner) {
            for (int64_t i = 0; i < m; ++i) {
                double acc = 0.0;
                for (int64_t j = ptr[i]; j < ptr[i + 1]; ++j) acc = rnd(f32, acc + rnd(f32, vi[j] * p[col[j]]));
                q[i] = acc;
            }
            double pq = dot(m, p, q);
            if (!(pq > 0.0) || !isfinite(pq)) { status = ORC_BREAKDOWN; break; }
            double a = rnd(f32, rho / pq);
            for (int64_t i = 0; i < m; ++i) d[i] = rnd(f32, d[i] + rnd(f32, a * p[i]));
            for (int64_t i = 0; i < m; ++i) ri[i] = rnd(f32, ri[i] - rnd(f32, a * q[i]));
            double rho_new = dot(m, ri, ri);
            ++k;
            double be = rho_new / rho;
            if (sqrt(rho_new / rho0) <= itol) { beta = be; have_dir = 1; break; }
            double bf = rnd(f32, be);
            for (int64_t i = 0; i < m; ++i) p[i] = rnd(f32, ri[i] + rnd(f32, bf * p[i]));
            rho = rho_new;
        }
        *inner_total += k;
        *outer += 1;
        if (status == ORC_BREAKDOWN) {
            if (fallback) go_fp64 = 1;
            break;
        }
        for (int64_t i = 0; i < m; ++i) x[i] += s * d[i];
        s_old = s;
    }
    if (go_fp64) {
        int its = 0;
        double rec = 0.0;
        int cap = max_inner * (max_outer > 1 ? max_outer : 1);
        status = orc_cg(m, ptr, col, val, b, x, tol, cap, &its, &rec, res_true, NULL);
        *fallback_its = its;
    }
out:
    free(vi); free(r); free(ax); free(ri); free(d); free(p); free(q);
    return status;
}

/* ------------------------------------------------------------------ */
/* Single-reduction CG (Chronopoulos and Gear, 1989)                    */
/* ------------------------------------------------------------------ */

/* The CG recurrence rearranged so that both inner products of an iteration
 * are taken together, right after the product with the matrix: the global
 * synchronisation after SpMV that the paper measures in its CG module
 * (Sec. 3, discussion of Fig 3.5) then happens once per iteration instead
 * of twice.  In exact arithmetic the iterates are those of orc_cg.
 *
 * With r = b - A x0, bnorm = ||b||:
 *   w = A r;  gamma = r.r;  delta = w.r          (one SpMV, two dots)
 *   stop when sqrt(gamma)/bnorm <= tol (the current r), or after max_iter
 *   updates;  otherwise
 *     first update:  beta = 0,  alpha = gamma/delta,  p = r,  s = w
 *     later:         beta = gamma/gamma_prev,
 *                    alpha = gamma/(delta - beta gamma/alpha_prev),
 *                    p = r + beta p,  s = w + beta s        (s = A p)
 *     x += alpha p;  r -= alpha s
 * The denominator equals p.Ap in exact arithmetic: a non-positive or
 * non-finite one is a breakdown.  iterations = updates of x; hist[k] =
 * ||r_k||/||b||.  At exit the true residual is recomputed. */
int orc_cg_single_reduction(int64_t m, const int64_t *ptr, const int32_t *col, const double *val,
                            const double *b, double *x, double tol, int max_iter,
                            int *iters, double *res_rec, double *res_true, double *hist)
{
    double *r = (double *)malloc((size_t)m * sizeof(double));
    double *w = (double *)malloc((size_t)m * sizeof(double));
    double *p = (double *)malloc((size_t)m * sizeof(double));
    double *sv = (double *)malloc((size_t)m * sizeof(double));
    if (!r || !w || !p || !sv) { free(r); free(w); free(p); free(sv); return ORC_ENOMEM; }
    int status = ORC_NOT_CONVERGED, k = 0;
    orc_csr_spmv(m, ptr, col, val, x, w);
    for (int64_t i = 0; i < m; ++i) r[i] = b[i] - w[i];
    double bnorm = sqrt(dot(m, b, b));
    double gamma = dot(m, r, r), gamma_prev = 0.0, alpha_prev = 0.0;
    if (bnorm == 0.0) {
        for (int64_t i = 0; i < m; ++i) x[i] = 0.0;
        *iters = 0; *res_rec = 0.0; *res_true = 0.0;
        if (hist) hist[0] = 0.0;
        free(r); free(w); free(p); free(sv);
        return ORC_OK;
    }
    if (hist) hist[0] = sqrt(gamma) / bnorm;
    if (sqrt(gamma) / bnorm <= tol) status = ORC_OK;
    while (status == ORC_NOT_CONVERGED && k < max_iter) {
        orc_csr_spmv(m, ptr, col, val, r, w);
        double delta = dot(m, w, r);
        double alpha, beta, denom;
        if (k == 0) {
            beta = 0.0;
            denom = delta;
        } else {
            beta = gamma / gamma_prev;
            denom = delta - beta * gamma / alpha_prev;
        }
        if (!(denom > 0.0) || !isfinite(denom)) { status = ORC_BREAKDOWN; break; }
        alpha = gamma / denom;
        for (int64_t i = 0; i < m; ++i) {
            p[i] = k == 0 ? r[i] : r[i] + beta * p[i];
            sv[i] = k == 0 ? w[i] : w[i] + beta * sv[i];
        }
        for (int64_t i = 0; i < m; ++i) x[i] += alpha * p[i];
        for (int64_t i = 0; i < m; ++i) r[i] -= alpha * sv[i];
        ++k;
        gamma_prev = gamma;
        alpha_prev = alpha;
        gamma = dot(m, r, r);
        if (hist) hist[k] = sqrt(gamma) / bnorm;
        if (sqrt(gamma) / bnorm <= tol) status = ORC_OK;
    }
    *iters = k;
    *res_rec = sqrt(gamma) / bnorm;
    orc_csr_spmv(m, ptr, col, val, x, w);
    for (int64_t i = 0; i < m; ++i) r[i] = b[i] - w[i];
    *res_true = sqrt(dot(m, r, r)) / bnorm;
    free(r); free(w); free(p); free(sv);
    return status;
}

/* ------------------------------------------------------------------ */
/* Jacobi-preconditioned CG                                             */
/* ------------------------------------------------------------------ */

/* CG on A x = b preconditioned by the diagonal D of A (the paper's solver is
 * unpreconditioned; this is the textbook preconditioned recurrence with
 * M = D).  With r = b - A x0, z = D^-1 r, p = z, rho = r.z:
 *   q = A p;  alpha = rho / p.q;  x += alpha p;  r -= alpha q;
 *   z = D^-1 r;  rho' = r.z;  stop when ||r||_2/||b||_2 <= tol;
 *   p = z + (rho'/rho) p.
 * The stopping test uses the unpreconditioned residual, as plain CG does, so
 * the iteration counts compare directly.  A zero or non-finite diagonal entry
 * returns ORC_EINVAL; p.q <= 0 or non-finite, ORC_BREAKDOWN.  hist[k] =
 * ||r_k||/||b||. */
int orc_cg_jacobi(int64_t m, const int64_t *ptr, const int32_t *col, const double *val,
                  const double *b, double *x, double tol, int max_iter,
                  int *iters, double *res_rec, double *res_true, double *hist)
{
    double *r = (double *)malloc((size_t)m * sizeof(double));
    double *z = (double *)malloc((size_t)m * sizeof(double));
    double *p = (double *)malloc((size_t)m * sizeof(double));
    double *q = (double *)malloc((size_t)m * sizeof(double));
    double *dinv = (double *)malloc((size_t)m * sizeof(double));
    int status = ORC_NOT_CONVERGED, k = 0;
    if (!r || !z || !p || !q || !dinv) { status = ORC_ENOMEM; goto out; }
    for (int64_t i = 0; i < m; ++i) {
        double d = 0.0;
        for (int64_t j = ptr[i]; j < ptr[i + 1]; ++j)
            if (col[j] == i) d = val[j];
        if (d == 0.0 || !isfinite(d)) { status = ORC_EINVAL; goto out; }
        dinv[i] = 1.0 / d;
    }
    orc_csr_spmv(m, ptr, col, val, x, q);
    for (int64_t i = 0; i < m; ++i) { r[i] = b[i] - q[i]; z[i] = dinv[i] * r[i]; p[i] = z[i]; }
    double rho = dot(m, r, z);
    double rr = dot(m, r, r);
    double bnorm = sqrt(dot(m, b, b));
    if (bnorm == 0.0) {
        for (int64_t i = 0; i < m; ++i) x[i] = 0.0;
        *iters = 0; *res_rec = 0.0; *res_true = 0.0;
        if (hist) hist[0] = 0.0;
        status = ORC_OK;
        goto out;
    }
    if (hist) hist[0] = sqrt(rr) / bnorm;
    if (sqrt(rr) / bnorm <= tol) status = ORC_OK;
    while (status == ORC_NOT_CONVERGED && k < max_iter) {
        orc_csr_spmv(m, ptr, col, val, p, q);
        double pq = dot(m, p, q);
        if (!(pq > 0.0) || !isfinite(pq)) { status = ORC_BREAKDOWN; break; }
        double alpha = rho / pq;
        for (int64_t i = 0; i < m; ++i) x[i] += alpha * p[i];
        for (int64_t i = 0; i < m; ++i) r[i] -= alpha * q[i];
        for (int64_t i = 0; i < m; ++i) z[i] = dinv[i] * r[i];
        double rho_new = dot(m, r, z);
        rr = dot(m, r, r);
        ++k;
        if (hist) hist[k] = sqrt(rr) / bnorm;
        if (sqrt(rr) / bnorm <= tol) { status = ORC_OK; break; }
        double beta = rho_new / rho;
        for (int64_t i = 0; i < m; ++i) p[i] = z[i] + beta * p[i];
        rho = rho_new;
    }
    *iters = k;
    *res_rec = sqrt(rr) / bnorm;
    orc_csr_spmv(m, ptr, col, val, x, q);
    for (int64_t i = 0; i < m; ++i) r[i] = b[i] - q[i];
    *res_true = sqrt(dot(m, r, r)) / bnorm;
out:
    free(r); free(z); free(p); free(q); free(dinv);
    return status;
}

/* ------------------------------------------------------------------ */
/* Analytic solution (Sec. 1, result verification)                      */
/* ------------------------------------------------------------------ */

/* Separation of variables for u=1 on x=1 and u=0 on the other faces of the
 * unit cube:
 *   u = sum over odd p,q of 16/(pi^2 p q) sin(p pi y) sin(q pi z)
 *         sinh(g x)/sinh(g),   g = pi sqrt(p^2+q^2).
 * The sinh ratio is evaluated as e^{g(x-1)} (1-e^{-2gx})/(1-e^{-2g}).
 * Terms are summed while their bound 16/(pi^2 p q) e^{g(x-1)} exceeds
 * 1e-18, up to p,q <= max_pq. */
double orc_analytic_u(double x, double y, double z, int max_pq)
{
    const double pi = 3.14159265358979323846;
    double u = 0.0;
    for (int p = 1; p <= max_pq; p += 2) {
        double gp = pi * p;
        if (16.0 / (pi * pi * p) * exp(gp * (x - 1.0)) < 1e-18) break;
        for (int q = 1; q <= max_pq; q += 2) {
            double g = pi * sqrt((double)p * p + (double)q * q);
            double bound = 16.0 / (pi * pi * p * q) * exp(g * (x - 1.0));
            if (bound < 1e-18) break;
            double ratio = exp(g * (x - 1.0)) * (1.0 - exp(-2.0 * g * x)) / (1.0 - exp(-2.0 * g));
            u += 16.0 / (pi * pi * p * q) * sin(p * pi * y) * sin(q * pi * z) * ratio;
        }
    }
    return u;
}
