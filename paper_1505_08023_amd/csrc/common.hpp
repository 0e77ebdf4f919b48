// Internal declarations shared by the library's translation units.
#pragma once

#include <hip/hip_runtime.h>

#include <cstddef>
#include <cstdint>
#include <string>
#include <vector>

#include "../../include/mfe.h"

namespace mfe {

// ------------------------------------------------------------------ errors

void set_error(const std::string &msg);
void clear_error();

#define MFE_HIP_TRY(expr)                                                         \
    do {                                                                          \
        hipError_t e_ = (expr);                                                   \
        if (e_ != hipSuccess) {                                                   \
            ::mfe::set_error(std::string(#expr " failed: ") + hipGetErrorString(e_)); \
            return MFE_EHIP;                                                      \
        }                                                                         \
    } while (0)

#define MFE_TRY(...)                 \
    do {                             \
        int s_ = (__VA_ARGS__);      \
        if (s_ != MFE_OK) return s_; \
    } while (0)

// ------------------------------------------------------------------ launch geometry

constexpr int kBlock = 256;     // threads per workgroup for every streaming kernel
constexpr int kSlice = 64;      // rows per slice of the 1x3 BCRS layout (one wavefront)
constexpr int kNumXcd = 8;      // accelerator complex dies of an MI355X
constexpr int kMaxPartials = 4096;  // per-workgroup partial sums one reduction may hold
constexpr int kPinnedSlots = 4;     // pinned CgState slots per context
constexpr int64_t kMallBytes = 256ll << 20;  // memory-side (Infinity) cache of an MI355X

// Stream CG vectors non-temporally when the five FP64 vectors an iteration
// touches exceed the memory-side cache.
#ifndef MFE_VECTORS_NT
#define MFE_VECTORS_NT 1  // 0: never stream the CG vectors non-temporally
#endif
inline bool vectors_stream_nt(int64_t m) { return MFE_VECTORS_NT != 0 && 40 * m > kMallBytes; }

// Load a stored matrix (values and indices, `bytes` in all) non-temporally
// when it is larger than MFE_MATRIX_NT_MIN_BYTES; a smaller one is loaded
// normally and largely stays in the memory-side cache between products.
// The default is the measured crossover on MI355X: cached loads were faster
// up to a 296 MB matrix (up to 20 % per CG iteration), non-temporal ones
// from 364 MB on.
#ifndef MFE_MATRIX_NT
#define MFE_MATRIX_NT 1  // non-temporal loads for matrices above MFE_MATRIX_NT_MIN_BYTES (0: never)
#endif
#ifndef MFE_MATRIX_NT_MIN_BYTES
#define MFE_MATRIX_NT_MIN_BYTES (320ll << 20)
#endif
inline bool matrix_stream_nt(int64_t bytes) {
    return MFE_MATRIX_NT != 0 && bytes > (int64_t)(MFE_MATRIX_NT_MIN_BYTES);
}

// ------------------------------------------------------------------ device solver state

enum CgStatus : int { kRunning = 0, kConverged = 1, kCapped = 2, kBreakdown = -4 };

// One per solve (one per system in a batched solve).  Lives in device memory;
// every scalar the CG recurrences need stays on the device.
//
// Within one kernel, workgroup 0 writes only fields that no workgroup of that
// kernel reads; the next kernel sees them (kernel boundaries order memory).
struct CgState {
    double rho;       // r.r of the current residual       (written by update_xp)
    double rho_old;   // rho at the start of the iteration (written by update_r)
    double alpha;     // rho / p.q of the current iteration (written by update_r)
    double bnorm;     // ||b||_2
    double tol;       // relative tolerance on ||r||/||b||
    double pq;        // last p.q
    double rr_true;   // ||b - A x||^2 evaluated at exit
    double scale;     // mixed precision: ||r|| of the outer residual
    double *hist;     // optional: hist[k] = ||r_k||/||b||, k = 0..max_iter
    double *dot_out;  // optional: a finalized p.q is also written here
    int status;       // CgStatus                          (written by update_xp / update_r)
    int iters;        // completed iterations               (written by update_xp)
    int max_iter;
    int active;       // 1 once update_r has run in the current iteration (cleared by the SpMV)
    int zero_x;       // 1: b = 0, the solution is x = 0; 2: the guess was rejected, restart from x = 0
    int warm;         // set by the host: reject x0 when ||b - A x0|| >= ||b||
    // single-reduction CG: the iteration count and status as the SpMV saw
    // them (read by the update kernel, which writes iters and status), and
    // gamma = r.r and alpha of the last two updates, indexed by the parity of
    // the update
    int iters_snap;
    int status_snap;
    double ring_g[2], ring_a[2];
    double rr;        // Jacobi-preconditioned CG: r.r of the current residual (rho holds r.z)
};

// (the 1x3 BCRS slice layout is described in b13_layout.hpp)

// CRS wavefront tiles: the CRS product gives each wavefront kCsrsRows
// consecutive rows.  A tile whose rows all hold 27 entries with
// column(row i, entry k) = i + off[k] (the interior of a box mesh) has
// uniform = 1 in its descriptor, and the product forms its columns from the
// 27 offsets instead of loading its 27 kCsrsRows column indices (which stay
// stored); uniform = 2 when, besides, the offsets come in 9 runs of three
// consecutive columns, which the product then takes a run at a time (three
// adjacent x entries per gather pair, as a 1x3 block).
#ifndef MFE_CSRS_ROWS
#define MFE_CSRS_ROWS 16  // rows per wavefront tile (64 / rows lanes per row); 8, 16 and 32 measured
#endif
constexpr int kCsrsRows = MFE_CSRS_ROWS;
struct CsrDesc {
    int32_t off[27];
    int32_t uniform;
};
static_assert(sizeof(CsrDesc) == 112, "CsrDesc is 112 bytes");

// CRS row groups of a mesh problem (MFE_CSR_GROUPS): a row is "full" when it
// holds 27 entries with column row + o_k, o_k the 27 neighbour offsets of the
// mesh numbering (ascending, in 9 runs of three consecutive columns).  Full
// rows come in runs (the interior of each x-line); the CRS product takes up
// to 64 consecutive full rows per wavefront (one lane per row, the group's
// contiguous values staged in LDS with 16-byte loads) and the other rows 16
// at a time from a row list.  Work items in row order:
//   {r0, n},       n in 1..64:  full rows r0 .. r0 + n - 1
//   {start, -n},   n in 1..16:  rows list[start .. start + n - 1]
#ifndef MFE_CSR_GROUPS
#define MFE_CSR_GROUPS 1  // group walk of the CRS product for mesh problems (0: 16-row tiles everywhere)
#endif
struct CsrRuns {
    int32_t r[9];  // first column offset of each run of three
};

// ------------------------------------------------------------------ context / problem

struct Buffer {
    void *ptr = nullptr;
    size_t bytes = 0;
};

}  // namespace mfe

struct mfe_ctx {
    int device = 0;
    hipStream_t stream = nullptr;      // caller's stream: all work goes here
    hipStream_t cap_stream = nullptr;  // private stream used only to capture graphs
    mfe_alloc_fn alloc = nullptr;
    mfe_free_fn free_fn = nullptr;
    void *alloc_user = nullptr;
    int num_cu = 256;
    void *pinned = nullptr;  // pinned host slots (kPinnedSlots x CgState) for solver state
    hipEvent_t ev[2] = {nullptr, nullptr};
    mfe::Buffer scratch;     // reduction partials for mfe_dot
    mfe::Buffer dot_state;   // CgState used by mfe_dot
    mfe::Buffer spmv_dot_state;  // CgState used by mfe_spmv_dot
    std::vector<mfe_problem *> problems;  // live problems, destroyed with the context
    std::vector<mfe_batch *> batches;     // live batches, likewise
    std::vector<mfe_net *> nets;          // live networks, likewise
};

namespace mfe {
// remove `item` from a context's registry (no-op if absent)
template <typename T>
void unregister(std::vector<T *> &v, T *item) {
    for (size_t i = 0; i < v.size(); ++i)
        if (v[i] == item) {
            v.erase(v.begin() + (long)i);
            return;
        }
}
}  // namespace mfe

namespace mfe {

int dev_alloc(mfe_ctx *ctx, Buffer *b, size_t bytes);
void dev_free(mfe_ctx *ctx, Buffer *b);

// Scratch device memory owned by one host function and released when it
// returns, on every path.  The context's stream is synchronised before the
// release, so work enqueued on it that still uses the memory has finished.
struct TempBuffer {
    mfe_ctx *ctx;
    Buffer b;
    explicit TempBuffer(mfe_ctx *c) : ctx(c) {}
    TempBuffer(const TempBuffer &) = delete;
    TempBuffer &operator=(const TempBuffer &) = delete;
    ~TempBuffer();
    int alloc(size_t bytes) { return dev_alloc(ctx, &b, bytes); }
    void *ptr() const { return b.ptr; }
};

}  // namespace mfe

struct mfe_graph_cache;

struct mfe_problem {
    mfe_ctx *ctx = nullptr;
    bool is_mesh = false;
    int Nx = 0, Ny = 0, Nz = 0;
    int64_t m = 0, nnz = 0, nblocks = 0, nslots = 0;
    int64_t b13_cslices = 0, b13_cblocks = 0;  // slices with compressed column indices, their real blocks
    int64_t csr_ctiles = 0;                     // CRS wavefront tiles with a uniform descriptor
    int formats = 0, precisions = 0;
    // CRS (always FP64; FP32 values when MFE_F32)
    mfe::Buffer ptr, col, val64, val32, b;
    mfe::Buffer cdesc;  // CsrDesc per CRS wavefront tile
    mfe::Buffer citems, crows;  // CRS group walk: work items (int2) and the list of the other rows
    int64_t ncitems = 0, ncrows = 0, ncgroups = 0, ncgroup_rows = 0;
    mfe::CsrRuns cruns{};
    // 1x3 BCRS
    mfe::Buffer slot_base, jas, bval64, bval32, rowblocks;
    mfe::Buffer bdesc;  // B13Desc per slice
    // CG workspace (allocated on first solve)
    mfe::Buffer r, p, q, state, partials;
    mfe::Buffer r32, p32, q32, d32, ax;  // mixed precision workspace
    mfe::Buffer s;                       // single-reduction CG: s = A p
    mfe::Buffer dinv;                    // Jacobi-preconditioned CG: 1 / diag(A)
    mfe_graph_cache *graphs = nullptr;
    // mean d log(residual) / d iteration of the last solve of each kind (CG,
    // single-reduction CG, Jacobi CG, FP32 inner CG): the prior of the next
    // solve's forecast (0: none yet)
    double rate[4] = {0.0, 0.0, 0.0, 0.0};
};

namespace mfe {

// ------------------------------------------------------------------ kernel launchers (host)

// assembly (assemble.hip)
int launch_assemble(mfe_problem *P, const double *face_vals, const double *node_g, bool values_and_rhs,
                    bool rhs_only);
int launch_assemble_into(hipStream_t s, int Nx, int Ny, int Nz, const double *face_vals, const double *node_g,
                         int64_t row_off, int64_t nnz_off, int32_t *ptr, int32_t *col, double *val, double *b,
                         bool rhs_only);

// formats (formats.hip)
int build_csr_tiles(mfe_problem *P);
int build_csr_groups(mfe_problem *P);
int build_bcrs13(mfe_problem *P);
int validate_csr(mfe_ctx *ctx, int64_t m, int64_t nnz, const int32_t *ptr, const int32_t *col);
int cast_values_f32(mfe_problem *P);
int export_bcrs13(const mfe_problem *P, int32_t *bptr, int32_t *bcol, double *bval);

// SpMV modes
// Fused epilogues of the SpMV kernels; reductions leave per-workgroup
// partials (second one at offset kMaxPartials) for the next kernel to sum.
enum SpmvMode : int {
    kSpmvPlain = 0,   // y = A x
    kSpmvDot = 1,     // y = A x, partials of x.y
    kSpmvResid = 2,   // r = b - A x, p = r, partials of r.r and b.b
    kSpmvTrue = 3,    // partials of ||b - A x||^2
    kSpmvDot2 = 4,    // w = A r, partials of r.w and r.r (single-reduction CG)
};

struct SpmvArgs {
    const void *x;
    void *y;         // y (plain/dot) or r (resid)
    void *p_out;     // resid: p = r (may be null)
    const double *b; // resid/true
    CgState *st;
    double *partials;
    int max_partials = 0;  // > 0: refuse a launch whose grid would write more partials
};

// *grid (optional) receives the number of workgroups, i.e. of partials written.
int launch_spmv(const mfe_problem *P, int format, bool f32, SpmvMode mode, const SpmvArgs &a,
                hipStream_t s, int *grid = nullptr);

// static scratch of the allocation-free entry point (noalloc.hip): looks up
// this device's address of it; called by mfe_ctx_create with the device current
int noalloc_init(int device);

// problem storage (api.hip)
void free_problem_storage(mfe_problem *P);
int finish_problem(mfe_problem *P);

// CG driver (cg.hip)
constexpr int kGraphIters = 16;  // CG iterations per captured graph
constexpr int kTailIters = 4;    // iterations per graph once the end of a solve is forecast
int ensure_workspace(mfe_problem *P);
int graph_for(mfe_problem *P, int format, bool f32, void *x, void *r, void *p, void *q, CgState *st, int k,
              hipGraphExec_t *out, int kind = 0);

// Host-side forecast of the iterations a solve still needs: a geometric fit
// of its stop-test residual between two polls of the device state, seeded
// with a prior rate (the last solve of the same kind on the same problem).
// Only the length of the graphs the host launches depends on it.
struct Forecast {
    double slope = 0.0;  // d log(residual) / d iteration; < 0 once known
    int it = -1;         // iterations at the last observation
    double lr = 0.0;     // log(residual) there
    // observation: residual res after i iterations; returns the iterations
    // forecast to reach tol (1e30 while no decreasing rate is known)
    double observe(int i, double res, double tol);
};

// The iteration graphs of one solve: k iterations, and kt < k for the end of
// the solve (tail = nullptr when k <= kTailIters).
struct IterGraphs {
    hipGraphExec_t exec = nullptr, tail = nullptr;
    int k = 0, kt = 0;
};
int iteration_graphs(mfe_problem *P, int format, bool f32, void *x, void *r, void *p, void *q, CgState *st,
                     int max_iter, int kind, IterGraphs *G);
// the stop-test residual ||r|| / ||b|| of a polled state (kind 2: the
// unpreconditioned r.r of the Jacobi CG)
double stop_residual(const CgState &s, int kind);
int run_iterations(mfe_problem *P, const IterGraphs &G, const CgState *st, int max_iter, int kind, Forecast &fc,
                   double rem, CgState *fin);
// records the mean rate of a finished solve as the prior of the next one
void record_rate(mfe_problem *P, int slot, double res0, const CgState &fin, int kind);
int cg_solve(mfe_problem *P, int format, double *x, double tol, int max_iter, double *hist, mfe_cg_stats *st,
             bool warm = false);
// Jacobi-preconditioned CG (FP64)
int cg_jacobi_solve(mfe_problem *P, int format, double *x, double tol, int max_iter, double *hist,
                    mfe_cg_stats *st);
int build_dinv(mfe_problem *P);
int launch_pcg_start(const mfe_problem *P, const double *r, double *p, const double *dinv, CgState *st,
                     double *partials, hipStream_t s);
int launch_pupdate_r(const mfe_problem *P, double *r, const double *q, const double *dinv, CgState *st,
                     const double *pq_part, int n_pq, double *part, int *grid, hipStream_t s);
int launch_pupdate_xp(const mfe_problem *P, double *x, double *p, const double *r, const double *dinv, CgState *st,
                      const double *part, int n, hipStream_t s);
// single-reduction CG (FP64)
int cg_sr_solve(mfe_problem *P, int format, double *x, double tol, int max_iter, double *hist, mfe_cg_stats *st);
int launch_sr_update(const mfe_problem *P, double *x, double *r, double *p, double *s, const double *w, CgState *st,
                     const double *partials, int n, hipStream_t stream);
void release_graphs(mfe_problem *P);

// mixed precision (mixed.hip)
int cg_mixed_solve(mfe_problem *P, int format, double *x, double tol, double inner_tol, int max_outer,
                   int max_inner, mfe_cg_stats *st, bool warm = false, bool keep_direction = false);

// vector kernels (vector.hip).  update_r consumes the n_pq partials of p.q
// at pq_partials and writes its r.r partials to rr_partials (*grid of them);
// update_xp consumes those.
int launch_update_r(const mfe_problem *P, bool f32, void *r, const void *q, CgState *st,
                    const double *pq_partials, int n_pq, double *rr_partials, hipStream_t s, int *grid);
int launch_update_xp(const mfe_problem *P, bool f32, void *x, void *p, const void *r, CgState *st,
                     const double *rr_partials, int n_rr, hipStream_t s);
// one-workgroup reductions of partials into the state
enum FinalizeKind : int { kFinStart = 0, kFinTrue = 1, kFinDot = 2 };
int launch_finalize(FinalizeKind kind, const double *partials, int n, CgState *st, hipStream_t s);
int launch_state_reset(CgState *st, double *dot_out, hipStream_t s);
// x = 0 when the state asks for it; on a rejected guess also r = p = b (r, p, b may be NULL otherwise)
int launch_zero_if(int64_t m, double *x, double *r, double *p, const double *b, const CgState *st, int num_cu,
                   hipStream_t s);
int launch_dot(mfe_ctx *ctx, int64_t n, const double *x, const double *y, double *partials, hipStream_t s,
               int *grid);
// bandwidth probes: kind 0 copies src to dst, kind 1 reads src into per-workgroup partials at dst
int launch_stream_probe(mfe_ctx *ctx, int kind, int64_t n, const double *src, double *dst);

// Grid sizing shared by the launchers.  resident_per_cu: workgroups of
// kBlock threads of `kernel` that fit on one CU (cached per kernel).
// resident_grid: min(max_groups, kMaxPartials, ntiles rounded up to a multiple
// of kNumXcd), itself a multiple of kNumXcd and at least kNumXcd.
int resident_per_cu(const void *kernel);
int resident_grid(long max_groups, long ntiles);

}  // namespace mfe
