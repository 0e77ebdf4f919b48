/*
 * mfe.h -- C ABI of the MI355X (gfx950) library for the MiniFE-style
 * finite-element method of Wu, Yang, Xiang and Cheng, "The Research and
 * Optimization of Parallel Finite Element Algorithm based on MiniFE".
 *
 * The library generates the Nx x Ny x Nz hexahedral box mesh of the unit
 * cube, assembles the trilinear element equations of steady heat conduction
 * with Dirichlet faces (Sec. 1: u = 1 on x = 1, u = 0 on the other faces by
 * default), stores the matrix in CRS (Sec. 3.1, Fig 3.1) and in fixed 1x3
 * BCRS (the segment format of Sec. 3.1, Figs 3.2/3.3, with the segment
 * length fixed to 3 and zero padding), and solves it with unpreconditioned
 * conjugate gradient (Sec. 1, CG module: MATVEC, DOT, WAXPY).
 *
 * Conventions for every entry point
 *   - Return value: MFE_OK (0), MFE_NOT_CONVERGED (1, results valid, the
 *     iteration cap was reached) or a negative error code.  No function
 *     throws or aborts.  mfe_last_error() gives a message for the calling
 *     thread's last failure.
 *   - Pointers named *_dev are device pointers (HIP global memory of the
 *     context's device); all other pointers are host pointers.  Vectors are
 *     dense, contiguous, of length m (rows) unless stated otherwise.
 *   - Caller-owned: every pointer argument.  Library-owned: the context and
 *     problem objects and the matrix/format/workspace storage behind them,
 *     released by the matching *_destroy call.
 *   - Work is enqueued on the context's stream.  Calls that return results
 *     on the host (stats, info, dot values) synchronise that stream first;
 *     the others return without synchronising.
 *   - A context and everything attached to it are used by one host thread at
 *     a time: calls on one context must not overlap (they share the stream,
 *     pinned host slots and reduction scratch).  Different contexts are
 *     independent.
 *   - Mesh numbering: node (ix, iy, iz), 0 <= ix <= Nx, ..., has id
 *     ix + (Nx+1)*(iy + (Ny+1)*iz) (x fastest) and coordinates
 *     (ix/Nx, iy/Ny, iz/Nz).  Matrix rows are nodes, all of them: Dirichlet
 *     rows are identity rows and Dirichlet columns of free rows are zeroed
 *     (symmetric elimination); structural zeros stay stored, so every row
 *     holds its full in-range 27-point neighbourhood in ascending column
 *     order, nnz = (3Nx+1)(3Ny+1)(3Nz+1).
 */
#ifndef MFE_H
#define MFE_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* status codes */
#define MFE_OK 0
#define MFE_NOT_CONVERGED 1
#define MFE_EINVAL (-1)        /* bad argument (null pointer, size, flag) */
#define MFE_ENOMEM (-2)        /* device allocation failed */
#define MFE_EHIP (-3)          /* a HIP runtime call failed */
#define MFE_EBREAKDOWN (-4)    /* CG met p.Ap <= 0 or a non-finite value */
#define MFE_EUNSUPPORTED (-5)  /* size beyond 32-bit indexing, or format/precision not built */

/* matrix formats (bit flags) */
#define MFE_CSR 1      /* compressed row storage, Sec. 3.1 */
#define MFE_BCRS13 2   /* fixed 1x3 blocks, zero padded, 64-row slice-major layout
                          (see mfe_problem_bcrs13_layout) */

/* precisions (bit flags) */
#define MFE_F64 1
#define MFE_F32 2

typedef struct mfe_ctx mfe_ctx;
typedef struct mfe_problem mfe_problem;

/* Optional device allocator.  alloc returns a device pointer aligned to at
 * least 256 bytes, or NULL; free releases it.  With NULL callbacks the
 * library uses hipMalloc / hipFree. */
typedef void *(*mfe_alloc_fn)(size_t bytes, void *user);
typedef void (*mfe_free_fn)(void *ptr, void *user);

typedef struct mfe_cg_stats {
    int32_t status;            /* MFE_OK, MFE_NOT_CONVERGED or MFE_EBREAKDOWN */
    int32_t iterations;        /* SpMVs inside the CG loop (mixed: summed over inner solves) */
    int32_t outer;             /* mixed precision: refinement steps; else 0 */
    int32_t spmv_count;        /* all SpMVs issued, including residual evaluations */
    double rel_res_recurrence; /* sqrt(r.r)/||b|| of the recurrence residual at exit */
    double rel_res_true;       /* ||b - A x||_2 / ||b||_2 recomputed in FP64 at exit */
    double seconds;            /* host wall time of the call */
    int32_t guess_rejected;    /* mfe_cg_warm: 1 if the solve started from x = 0 instead of the guess */
    int32_t reserved_;
} mfe_cg_stats;

/* Message for the calling thread's last error ("" if none). */
const char *mfe_last_error(void);

/* ABI version, bumped on any change of these declarations. */
int mfe_version(void);

/* Create a context on HIP device `device`.  `stream` is a hipStream_t (NULL =
 * the null stream) on which all work of this context is enqueued.  The
 * allocator pair may be NULL.  *out receives the context. */
int mfe_ctx_create(int device, void *stream, mfe_alloc_fn alloc, mfe_free_fn free_fn,
                   void *alloc_user, mfe_ctx **out);
/* Synchronises the stream and destroys the context together with every
 * problem, batch and network still attached to it (their handles become
 * invalid). */
int mfe_ctx_destroy(mfe_ctx *ctx);

/* Problem statement and assembly (Sec. 1; Fig 3.6 structure, Fig 3.7
 * element assembly).  Nx, Ny, Nz >= 1 elements per axis.  Boundary values:
 * node_g_dev (device, length m, only boundary entries read) if non-NULL,
 * else face_vals[6] = {x=0, x=1, y=0, y=1, z=0, z=1} if non-NULL, else the
 * paper's {0, 1, 0, 0, 0, 0}.  A node on several faces takes the first face
 * in the order x=1, x=0, y=1, y=0, z=1, z=0.  Zero source.
 * `formats` (MFE_CSR | MFE_BCRS13) and `precisions` (MFE_F64 | MFE_F32)
 * select which stored forms are built (CSR FP64 is always built: it is the
 * assembly format).  Fails with MFE_EUNSUPPORTED when nnz >= 2^31. */
int mfe_problem_create(mfe_ctx *ctx, int Nx, int Ny, int Nz, const double *face_vals,
                       const double *node_g_dev, int formats, int precisions, mfe_problem **out);

/* Generic CRS problem (Sec. 3.1): copies ptr_dev[m+1], col_dev[nnz] (ascending,
 * distinct, in [0,m) per row), val_dev[nnz], b_dev[m] (b_dev may be NULL: b = 0).
 * Rows may be empty.  Intended for symmetric positive definite A. */
int mfe_problem_from_csr(mfe_ctx *ctx, int64_t m, const int32_t *ptr_dev, const int32_t *col_dev,
                         const double *val_dev, const double *b_dev, int formats, int precisions,
                         mfe_problem **out);

/* mfe_problem_from_csr from host arrays (the CRS arrays of Sec. 3.1 as a
 * caller holds them in host memory): ptr[m+1] (ptr[0] = 0), col[ptr[m]],
 * val[ptr[m]], b[m] (may be NULL: b = 0) are copied to the device before
 * the call returns; the caller may reuse them at once.  Same checks, results
 * and errors as mfe_problem_from_csr. */
int mfe_problem_from_csr_host(mfe_ctx *ctx, int64_t m, const int32_t *ptr, const int32_t *col, const double *val,
                              const double *b, int formats, int precisions, mfe_problem **out);

/* Re-impose new Dirichlet data on a mesh problem without re-assembling:
 * recomputes b (same rules as mfe_problem_create).  MFE_EINVAL for a problem
 * made by mfe_problem_from_csr. */
int mfe_problem_set_bc(mfe_problem *p, const double *face_vals, const double *node_g_dev);

/* Sizes: rows, stored entries, 1x3 blocks (0 when BCRS13 was not built).
 * Any output pointer may be NULL. */
int mfe_problem_info(const mfe_problem *p, int64_t *m, int64_t *nnz, int64_t *nblocks);

/* Storage of the CRS as the CRS product walks it: wavefront tiles of
 * *tile_rows consecutive rows (*tiles of them), and the tiles whose column
 * indices the product forms from a 112-byte per-tile descriptor instead of
 * reading them (full tiles whose rows all hold 27 entries with column
 * i + off_k for entry k of row i: the interior of a box mesh).  The indices
 * stay stored.  Any output pointer may be NULL. */
int mfe_problem_csr_layout(const mfe_problem *p, int64_t *tile_rows, int64_t *tiles, int64_t *compressed_tiles);

/* The CRS product's walk of a mesh problem (all zero when it walks the
 * wavefront tiles of mfe_problem_csr_layout instead): *items work items in
 * row order, *groups of them runs of up to 64 consecutive rows that hold 27
 * entries each with the mesh's 27 neighbour columns (*group_rows rows in
 * all, their values staged with 16-byte loads and their columns formed from
 * the 27 offsets, whose indices stay stored), the other *other_rows rows
 * taken 16 per item from a row list with their column indices read.  Any
 * output pointer may be NULL. */
int mfe_problem_csr_groups(const mfe_problem *p, int64_t *items, int64_t *groups, int64_t *group_rows,
                           int64_t *other_rows);

/* Storage of the 1x3 BCRS (all zero when it was not built): 64-row slices;
 * slot rows (slice s stores 64 x its slot count blocks, padding included);
 * slices whose column indices the SpMV forms from a 48-byte per-slice
 * descriptor instead of reading them (slices of 64 rows x 9 blocks in which
 * the first column of block k of row i is i + e_i + d_k, e_i in {0, 1}: the
 * interior of a box mesh), and the real blocks of those slices.  The
 * indices of every slice stay stored.  Any output pointer may be NULL. */
int mfe_problem_bcrs13_layout(const mfe_problem *p, int64_t *slices, int64_t *slots, int64_t *compressed_slices,
                              int64_t *compressed_blocks);

/* Copy the FP64 CRS matrix and b into caller device buffers
 * (ptr_dev[m+1], col_dev[nnz], val_dev[nnz], b_dev[m]; any may be NULL). */
int mfe_problem_export_csr(const mfe_problem *p, int32_t *ptr_dev, int32_t *col_dev,
                           double *val_dev, double *b_dev);

/* mfe_problem_export_csr into host arrays (ptr[m+1], col[nnz], val[nnz],
 * b[m]; any may be NULL).  Synchronises the stream. */
int mfe_problem_export_csr_host(const mfe_problem *p, int32_t *ptr, int32_t *col, double *val, double *b);

/* The right-hand side b of A x = b (Sec. 1: the assembled load vector after
 * the Dirichlet values are imposed; for a CRS problem the b it was given)
 * into b_dev[m].  Does not synchronise. */
int mfe_rhs(const mfe_problem *p, double *b_dev);

/* Copy the 1x3 BCRS as per-row block lists: bptr_dev[m+1] (first block of
 * each row, bptr[m] = nblocks), bcol_dev[nblocks] (first column of each
 * block), bval_dev[3*nblocks] (FP64).  Padding slots of the slice layout
 * are dropped; blocks keep their per-row order. */
int mfe_problem_export_bcrs13(const mfe_problem *p, int32_t *bptr_dev, int32_t *bcol_dev,
                              double *bval_dev);

int mfe_problem_destroy(mfe_problem *p);

/* y = A x (Sec. 3.1 MATVEC; Fig 3.1 for MFE_CSR, the 1x3 segment loop of
 * Figs 3.2/3.3 for MFE_BCRS13).  FP64 values and vectors, FP64 sums.
 * x_dev and y_dev must not overlap. */
int mfe_spmv(const mfe_problem *p, int format, const double *x_dev, double *y_dev);

/* FP32 values and vectors, FP32 sums (needs MFE_F32 at create). */
int mfe_spmv_f32(const mfe_problem *p, int format, const float *x_dev, float *y_dev);

/* q = A p fused with the DOT that follows MATVEC in CG (Sec. 1 CG module;
 * Sec. 3.1 on the dot product after SpMV): writes q_dev and the FP64 value
 * p.q to *pq_dev (a device scalar), reduced in a fixed order.  FP64.  The
 * kernel is the one each CG iteration runs; this entry point exists to use
 * and time it on its own.  ev_before / ev_after (hipEvent_t, may be NULL)
 * are recorded on the context's stream immediately before and after that
 * kernel's launch.  Does not synchronise. */
int mfe_spmv_dot(const mfe_problem *p, int format, const double *p_dev, double *q_dev, double *pq_dev,
                 void *ev_before, void *ev_after);

/* The same fused product in FP32 (the kernel of the inner solves of
 * mfe_cg_mixed): FP32 matrix values, p and q, FP32 row sums, p.q accumulated
 * in FP64 into *pq_dev.  Needs MFE_F32 at create.  Does not synchronise. */
int mfe_spmv_dot_f32(const mfe_problem *p, int format, const float *p_dev, float *q_dev, double *pq_dev,
                     void *ev_before, void *ev_after);

/* mfe_spmv_dot for callers that cannot allocate device memory (code under
 * HIP graph capture, allocation-free serving loops, harnesses that forbid
 * hipMalloc): the same kernels and results (q and p.q bitwise those of
 * mfe_spmv_dot), but the reduction partials and the solver state live in a
 * static device array of the library, 33,024 bytes per GPU (partials of up
 * to 4096 workgroups, which no launch of the product exceeds; one that would
 * is refused with MFE_EUNSUPPORTED before any work is enqueued), held from
 * the first mfe_ctx_create on that GPU until the process ends.  The call
 * allocates nothing and does not synchronise; it enqueues three kernels on
 * the context's stream.  Every call on one GPU shares that array, whatever
 * its context or stream: calls that overlap on one GPU race (the caller
 * orders them, for instance on one stream).  Each call sets all of the
 * array's contents it reads.  FP64, formats as mfe_spmv_dot. */
int mfe_spmv_dot_noalloc(const mfe_problem *p, int format, const double *p_dev, double *q_dev, double *pq_dev);

/* Dot product (Sec. 1, DOT) of two FP64 device vectors of length n >= 0
 * (x_dev, y_dev may be NULL when n = 0),
 * reduced in a fixed order (bitwise reproducible run to run).  The result is
 * written to *out_host (the stream is synchronised). */
int mfe_dot(mfe_ctx *ctx, int64_t n, const double *x_dev, const double *y_dev, double *out_host);

/* Streaming bandwidth probe, a measurement reference for the kernels above
 * (not part of the method): kind 0 copies n doubles from src_dev to dst_dev,
 * kind 1 reads n doubles from src_dev and writes one partial sum per
 * workgroup to dst_dev (room for 4096 doubles), both with grid-stride
 * 16-byte non-temporal accesses on a resident grid.  src_dev and dst_dev
 * must not overlap.  ev_before / ev_after as in mfe_spmv_dot.  Does not
 * synchronise. */
int mfe_stream_probe(mfe_ctx *ctx, int kind, int64_t n, const double *src_dev, double *dst_dev, void *ev_before,
                     void *ev_after);

/* Unpreconditioned CG (Sec. 1 CG module) on A x = b in FP64, with the
 * SpMV of `format` (MFE_CSR or MFE_BCRS13, which must have been built).
 * x_dev holds x0 on entry and the solution on exit.  r0 = b - A x0; the loop
 * stops when the recurrence residual satisfies ||r_k||_2 / ||b||_2 <= tol
 * (k = number of SpMVs in the loop) or after max_iter iterations; b = 0
 * gives x = 0.  tol >= 0, max_iter >= 0.  hist_dev (may be NULL) receives
 * ||r_k||/||b|| for k = 0..iterations (room for max_iter+1 doubles).  stats
 * may be NULL.  Returns MFE_OK, MFE_NOT_CONVERGED or MFE_EBREAKDOWN (x then
 * holds the last iterate).  Calls on one problem must not overlap. */
int mfe_cg(const mfe_problem *p, int format, double *x_dev, double tol, int max_iter,
           double *hist_dev, mfe_cg_stats *stats);

/* mfe_cg from an initial guess that may be poor (for instance a learned
 * prediction): with r0 = b - A x0, if ||r0||_2 >= ||b||_2 (the zero start is
 * at least as close) the solve starts from x0 = 0 instead, so it is never
 * worse than plain CG from zero.  The choice is made on the device in the
 * same kernels that start mfe_cg (no extra host round trip);
 * stats->guess_rejected reports it.  Arguments and return values as mfe_cg. */
int mfe_cg_warm(const mfe_problem *p, int format, double *x_dev, double tol, int max_iter,
                double *hist_dev, mfe_cg_stats *stats);

/* Single-reduction CG (the Chronopoulos-Gear form of the CG module of
 * Sec. 1): the same Krylov iterates as mfe_cg in exact arithmetic, but both
 * inner products of an iteration (r.r and r.Ar) are taken together in the
 * kernel that forms w = A r, so an iteration has one reduction point where
 * mfe_cg has two (Sec. 3, discussion of Fig 3.5: the global synchronisation
 * after SpMV).  Recurrences: beta = gamma/gamma_prev, alpha = gamma /
 * (delta - beta gamma/alpha_prev), p = r + beta p, s = w + beta s, x +=
 * alpha p, r -= alpha s with gamma = r.r, delta = r.w.  FP64 only.  The
 * stopping rule, hist_dev, stats and return values are those of mfe_cg
 * (iterations = updates of x); the loop issues iterations + 1 SpMVs since
 * the residual norm of an iterate is known only after its product.  A
 * non-positive or non-finite alpha denominator returns MFE_EBREAKDOWN. */
int mfe_cg_single_reduction(const mfe_problem *p, int format, double *x_dev, double tol, int max_iter,
                            double *hist_dev, mfe_cg_stats *stats);

/* Jacobi-preconditioned CG (a comparison variant of the unpreconditioned CG
 * module of Sec. 1): preconditioner M = diag(A), built once per problem from
 * the FP64 CRS values (MFE_EINVAL if a diagonal entry is zero, missing or
 * not finite).  z = D^-1 r, alpha = r.z / p.Ap, p = z + beta p.  The
 * stopping test, hist_dev (||r_k||/||b||), stats and return values are
 * those of mfe_cg, so iteration counts compare directly.  FP64 only. */
int mfe_cg_jacobi(const mfe_problem *p, int format, double *x_dev, double tol, int max_iter,
                  double *hist_dev, mfe_cg_stats *stats);

/* Result verification (Sec. 1) for the paper's boundary data (u = 1 on
 * x = 1, u = 0 on the other faces; the problem must come from
 * mfe_problem_create, else MFE_EUNSUPPORTED).  On the device, evaluates the
 * separation-of-variables solution
 *   u = sum_{p,q odd} 16/(pi^2 p q) sin(p pi y) sin(q pi z) sinh(g x)/sinh(g),
 *   g = pi sqrt(p^2 + q^2)   (terms summed while their bound exceeds 1e-18)
 * at every node with x-coordinate <= x_max (0 < x_max < 1; the series
 * converges slowly next to x = 1) and reduces, over those nodes, max |x - u|
 * into *max_err, sqrt(mean (x - u)^2) into *rms_err and their number into
 * *count (host scalars).  u_dev (length m, may be NULL) receives u at those
 * nodes and NaN elsewhere.  Synchronises the stream. */
int mfe_verify_series(const mfe_problem *p, const double *x_dev, double x_max, double *u_dev, double *max_err,
                      double *rms_err, int64_t *count);

/* Mixed precision CG (FP32-inner / FP64-refinement extension of the CG
 * module of Sec. 1).  Outer loop in FP64: r = b - A x with the FP64 matrix,
 * stop when ||r||_2/||b||_2 <= tol, s = ||r||; inner unpreconditioned CG in
 * FP32 on A32 d = fl32(r/s) from d = 0 (FP32 matrix values, SpMV sums and
 * vector updates; FP64 dot-product accumulation and alpha/beta) until its
 * relative residual is <= max(inner_tol, tol ||b|| / (2 s)) or max_inner
 * iterations; then x += s d in FP64.  A refinement step that does not halve ||r||, or an inner
 * breakdown, continues with FP64 CG (mfe_cg) from the current x.  Needs
 * MFE_F32 at create.  stats->iterations sums all CG iterations (inner and
 * fallback), stats->outer counts refinement steps, rel_res_true is the
 * final FP64 ||b - A x||/||b||.  0 <= tol, 0 < inner_tol < 1, max_outer >= 1,
 * max_inner >= 1.  Returns MFE_OK or MFE_NOT_CONVERGED (max_outer reached). */
int mfe_cg_mixed(const mfe_problem *p, int format, double *x_dev, double tol, double inner_tol,
                 int max_outer, int max_inner, mfe_cg_stats *stats);

/* mfe_cg_mixed from an initial guess that may be poor (the learned
 * prediction with mixed precision): if the first FP64 residual has
 * ||b - A x0||_2 >= ||b||_2 the solve starts from x0 = 0 instead, decided on
 * the device as in mfe_cg_warm; stats->guess_rejected reports it.
 * Arguments and return values as mfe_cg_mixed. */
int mfe_cg_mixed_warm(const mfe_problem *p, int format, double *x_dev, double tol, double inner_tol,
                      int max_outer, int max_inner, mfe_cg_stats *stats);

/* Flags of mfe_cg_mixed_ex. */
#define MFE_MIXED_WARM 1           /* start from x_dev as mfe_cg_mixed_warm does */
#define MFE_MIXED_KEEP_DIRECTION 2 /* keep the inner CG's direction across refinement steps */
/* mfe_cg_mixed (flags 0) and mfe_cg_mixed_warm (MFE_MIXED_WARM) with
 * options.  MFE_MIXED_KEEP_DIRECTION: after an inner solve that met its
 * tolerance the next one is not restarted from d = 0, p = r; its recursive
 * residual is replaced by the new FP64 residual (a reliable update of the
 * residual, after Sleijpen and van der Vorst) and its recurrence goes on:
 * with s_old and s the previous and the new ||r||, r32 = fl32(r / s) and
 * p32 = r32 + (s_old / s)(p32 - r32_old), the CG step P_next = R + beta P in
 * the new scale with the FP64 residual for R (in exact arithmetic the inner
 * iterations are then those of one uninterrupted CG).  After a capped inner
 * solve the next one restarts.  Other flag bits: MFE_EINVAL.  Arguments,
 * stats and return values as mfe_cg_mixed. */
int mfe_cg_mixed_ex(const mfe_problem *p, int format, double *x_dev, double tol, double inner_tol, int max_outer,
                    int max_inner, int flags, mfe_cg_stats *stats);

/* Trilinear prolongation (an initial guess on a refined mesh): xc_dev holds
 * nodal values of the Nx x Ny x Nz element box mesh (node numbering as
 * above), xf_dev receives the interpolant of the coarse trilinear elements
 * (Sec. 1 element space) at the nodes of the (factor Nx) x (factor Ny) x
 * (factor Nz) mesh; with bnd_dev (length of the fine mesh, may be NULL) the
 * fine boundary nodes take bnd_dev's values instead, for instance the fine
 * problem's b (its Dirichlet values: its boundary rows are identity rows).
 * factor >= 1.  Does not synchronise. */
int mfe_prolong_trilinear(mfe_ctx *ctx, int Nx, int Ny, int Nz, const double *xc_dev, int factor,
                          const double *bnd_dev, double *xf_dev);

/* ---------------------------------------------------------------------
 * Batched solves: many box meshes of uneven size solved together (the
 * batched extension of the Sec. 1 CG module).  Each system follows exactly
 * the single-system recurrence (own alpha, beta, ||b||, stopping test) and
 * is frozen once converged.  The systems are stored as one block-diagonal
 * matrix; vectors are the concatenation of the systems' vectors (system j
 * occupies rows row_offsets[j] .. row_offsets[j+1]-1, node numbering inside
 * a system as for a single mesh).
 * ------------------------------------------------------------------- */
typedef struct mfe_batch mfe_batch;

/* sizes: host int32[3*nsys] (Nx, Ny, Nz per system, each >= 1); face_vals:
 * host double[6*nsys] (per system, order as in mfe_problem_create) or NULL
 * for the paper's values.  MFE_EUNSUPPORTED when the total nnz >= 2^31.
 * Destroy a batch before its context. */
int mfe_batch_create(mfe_ctx *ctx, int nsys, const int32_t *sizes, const double *face_vals, int formats,
                     int precisions, mfe_batch **out);
/* A batch of existing problems (mesh or CRS, all of context ctx, copied: the
 * problems stay usable and may be destroyed afterwards): the block-diagonal
 * matrix of their FP64 CRS and b, system j at rows row_offsets[j].. in the
 * order given, with `formats` and `precisions` built for it as at
 * mfe_problem_create.  mfe_batch_set_bc applies only when every system is a
 * mesh problem (else MFE_EINVAL).  MFE_EUNSUPPORTED when the total nnz >=
 * 2^31. */
int mfe_batch_from_problems(mfe_ctx *ctx, int nsys, mfe_problem *const *sys, int formats, int precisions,
                            mfe_batch **out);
int mfe_batch_destroy(mfe_batch *b);
/* Total rows, total stored entries, row_offsets (host int64[nsys+1]); any may be NULL. */
int mfe_batch_info(const mfe_batch *b, int64_t *m_total, int64_t *nnz_total, int64_t *row_offsets);
/* New Dirichlet data for every system without re-assembly (as
 * mfe_problem_set_bc): node_g_dev (device, length m_total, concatenated per
 * system, boundary entries used) if non-NULL, else face_vals (host
 * double[6*nsys]) if non-NULL, else the paper's values. */
int mfe_batch_set_bc(mfe_batch *b, const double *face_vals, const double *node_g_dev);
/* 1x3 BCRS storage of the block-diagonal matrix (as mfe_problem_bcrs13_layout;
 * slices are those of the concatenated rows, so a slice may span two systems). */
int mfe_batch_bcrs13_layout(const mfe_batch *b, int64_t *slices, int64_t *slots, int64_t *compressed_slices,
                            int64_t *compressed_blocks);
/* FP64 CRS of the block-diagonal matrix and b (device buffers, as mfe_problem_export_csr). */
int mfe_batch_export_csr(const mfe_batch *b, int32_t *ptr_dev, int32_t *col_dev, double *val_dev, double *b_dev);
/* Times the batched SpMV for each candidate launch shape (CRS: lanes per row
 * 8/16/32, i.e. rows per wavefront 8/4/2; 1x3 BCRS: one lane per row and
 * 1 or 2 64-row slices per wavefront and pass, i.e. rows per wavefront
 * 64/128; both with grid = 1, 2 or 4 times the resident workgroups) on this
 * batch and keeps the fastest for later solves in `format`.  *lanes_out
 * (CRS lanes per row, or 1x3 BCRS slices per wavefront) and *factor_out (may
 * be NULL) receive the choice. */
int mfe_batch_autotune(mfe_batch *b, int format, int *lanes_out, int *factor_out);
/* FP64 CG on every system from x_dev (length m_total): per system stop at
 * ||r||/||b|| <= tol or max_iter iterations.  stats: host array of nsys.
 * Returns MFE_OK when every system converged, MFE_NOT_CONVERGED if one hit
 * the cap, MFE_EBREAKDOWN if one broke down. */
int mfe_batch_cg(mfe_batch *b, int format, double *x_dev, double tol, int max_iter, mfe_cg_stats *stats);
/* FP32-inner / FP64-refinement CG (as mfe_cg_mixed) on every system
 * together; needs MFE_F32 at create. */
int mfe_batch_cg_mixed(mfe_batch *b, int format, double *x_dev, double tol, double inner_tol, int max_outer,
                       int max_inner, mfe_cg_stats *stats);
/* mfe_batch_cg_mixed with flags: MFE_MIXED_KEEP_DIRECTION keeps each
 * system's inner direction across refinement steps as mfe_cg_mixed_ex does
 * (per system: after an inner solve that met its tolerance); other bits
 * (MFE_MIXED_WARM included): MFE_EINVAL. */
int mfe_batch_cg_mixed_ex(mfe_batch *b, int format, double *x_dev, double tol, double inner_tol, int max_outer,
                          int max_inner, int flags, mfe_cg_stats *stats);

/* One batched solve of existing problems in a single call: builds the batch
 * of mfe_batch_from_problems in `format`, copies each x_dev[j] (length m_j:
 * x0 in, the solution out) in, runs mfe_batch_cg (mixed = 0) or
 * mfe_batch_cg_mixed with inner tolerance 1e-4, 50 refinement steps and
 * max_iter inner iterations (mixed = 1; FP32 values are built), copies the
 * results (the last iterates after a breakdown) back and releases the batch.
 * Every system follows the single-system recurrence with its own stopping
 * test.  stats: host array of nsys (may be NULL).  Returns as mfe_batch_cg.
 * The batch is rebuilt on every call; repeated solves of the same systems
 * should keep a batch of mfe_batch_from_problems instead. */
int mfe_cg_batched(mfe_ctx *ctx, int nsys, mfe_problem *const *sys, int format, double *const *x_dev, double tol,
                   int max_iter, int mixed, mfe_cg_stats *stats);

/* ---------------------------------------------------------------------
 * Learned initial guess (extension of the CG module): a 3-D convolutional
 * encoder-decoder on the node grid of a G x G x G node box mesh (G - 1
 * divisible by 8), BF16 weights and activations, FP32 accumulation on the
 * matrix cores, FP32 master weights and Adam.  Architecture (channels):
 * input 8 (boundary value, boundary mask, 6 zero) -> 16 -> 16 -> [stride 2]
 * 32 -> 32 -> [stride 2] 64 -> 64 -> [stride 2] 128 -> 128 -> [transposed
 * stride 2] 64 (+ skip) -> 64 -> 32 (+ skip) -> 32 -> 16 (+ skip) -> 8, all
 * 3x3x3 convolutions with bias, ReLU after every layer but the last;
 * channel 0 of the last layer is the prediction.  Node values are indexed
 * as the mesh's nodes (x fastest); batches are concatenated.
 * ------------------------------------------------------------------- */
typedef struct mfe_net mfe_net;

int mfe_net_create(mfe_ctx *ctx, int G, int batch_max, mfe_net **out);
int mfe_net_destroy(mfe_net *net);
/* Parameter count in the natural layout: for each layer W[o][27][c] (tap
 * d = dx + 3 dy + 9 dz) followed by b[o]. */
int mfe_net_num_params(const mfe_net *net, int64_t *n);
/* Host FP32 arrays in the natural layout.  set also resets the Adam state. */
int mfe_net_set_params(mfe_net *net, const float *params_host);
int mfe_net_get_params(const mfe_net *net, float *params_host);
/* Forward pass on batch boundary fields g_dev (FP64 [batch][G^3]; interior
 * entries ignored); pred_dev (FP32 [batch][G^3], may be NULL) gets channel 0. */
int mfe_net_forward(mfe_net *net, int batch, const double *g_dev, float *pred_dev);
/* Forward, mean squared error over interior nodes against target_dev (FP64
 * [batch][G^3], e.g. CG solutions), and backward into the parameter gradient
 * (kept for mfe_net_adam_step).  loss_host and grad_host (natural layout) may
 * be NULL. */
int mfe_net_loss_grad(mfe_net *net, int batch, const double *g_dev, const double *target_dev, double *loss_host,
                      float *grad_host);
/* As mfe_net_loss_grad with the energy norm of the error in place of its
 * square: e = prediction - target on interior nodes (0 on boundary nodes),
 * loss = e^T A e / (batch (G-2)^3), output gradient 2 A e / (batch (G-2)^3),
 * A the stiffness matrix of `problem` (the (G-1)^3 element box mesh of the
 * network's grid, built with `format`; its product runs on the GPU).  CG
 * minimises this norm of the error over its Krylov space (the CG module of
 * Sec. 1; the property is the textbook one), so it measures how far a guess is
 * from the solution in the solver's own terms.  Allocates two FP64 work
 * vectors of batch_max G^3 entries on first use (freed with the net). */
int mfe_net_loss_grad_energy(mfe_net *net, const mfe_problem *problem, int format, int batch, const double *g_dev,
                             const double *target_dev, double *loss_host, float *grad_host);
/* Replace the gradient that the next mfe_net_adam_step applies (host FP32,
 * natural layout), for instance one averaged over devices or computed
 * elsewhere.  The next mfe_net_loss_grad(_energy) overwrites it. */
int mfe_net_set_grad(mfe_net *net, const float *grad_host);
/* One Adam update (Kingma and Ba) with the gradient of the last
 * mfe_net_loss_grad(_energy) or mfe_net_set_grad, in FP32 on the master
 * weights, t counting the steps since mfe_net_set_params:
 *   m = beta1 m + (1 - beta1) g,  v = beta2 v + (1 - beta2) g^2,
 *   p -= lr (m / (1 - beta1^t)) / (sqrt(v / (1 - beta2^t)) + eps);
 * then the bf16 copies of the weights are rebuilt.  lr >= 0,
 * 0 <= beta1, beta2 < 1, eps > 0. */
int mfe_net_adam_step(mfe_net *net, float lr, float beta1, float beta2, float eps);
/* x0_dev (FP64 [G^3]) = g on boundary nodes, the network's prediction inside. */
int mfe_net_predict_x0(mfe_net *net, const double *g_dev, double *x0_dev);

/* Single 3x3x3 convolution on the matrix cores (the network's building
 * block, exposed for testing): in/out bf16 channels-last [batch][G^3][c],
 * mode 0 stride 1, 1 stride 2, 2 transposed stride 2; w_host FP32
 * [cout][27][cin] (rounded to bf16), bias_host FP32 [cout] or NULL, relu 0/1;
 * out32_dev (FP32, may be NULL) gets the unrounded result.  Channels must be
 * 8, 16, 32, 64 or 128.  Synchronises. */
int mfe_conv3d_bf16(mfe_ctx *ctx, int mode, int batch, int Gi, int cin, const void *in_dev, int cout,
                    const float *w_host, const float *bias_host, int relu, void *out_dev, float *out32_dev);
/* Input gradient of that convolution (the backward pass's building block):
 * gx[q][c] = sum over output voxels v and taps d with src(v, d) = q of
 * w[o][d][c] gy[v][o], gy bf16 [batch][Go^3][cout] on the output grid
 * Go of `mode` applied to Gi, gx bf16 [batch][Gi^3][cin].  It runs as the
 * network's backward pass does: the adjoint convolution (s1 with mirrored
 * taps for s1, the transposed stride-2 form for s2, stride 2 for t2) with
 * the (o, c)-transposed weights, rounded to bf16 from w_host (FP32
 * [cout][27][cin]), on the matrix cores with FP32 accumulation.
 * accumulate = 1: gx += that (the sum rounded once to bf16), as the network
 * accumulates gradients from several layers; 0: gx = that.  gx32_dev (FP32,
 * may be NULL) gets the unrounded sum.  Gi must be odd for mode 1 (the
 * adjoint maps back onto Gi).  Synchronises. */
int mfe_conv3d_dgrad_bf16(mfe_ctx *ctx, int mode, int batch, int Gi, int cin, const void *gy_dev, int cout,
                          const float *w_host, int accumulate, void *gx_dev, float *gx32_dev);
/* Weight gradient of that convolution: dw_host[o][27][c] = sum over samples
 * and output voxels of gy[v][o] x[src(v, d)][c].  Synchronises. */
int mfe_conv3d_wgrad_bf16(mfe_ctx *ctx, int mode, int batch, int Gi, int cin, const void *x_dev, int cout,
                          const void *gy_dev, float *dw_host);

#ifdef __cplusplus
}
#endif

#endif /* MFE_H */
