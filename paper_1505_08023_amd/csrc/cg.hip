// Unpreconditioned CG driver (Sec. 1 CG module).
//
// The paper's CG loop is MATVEC, DOT with a global reduction, and WAXPY, each
// iteration ending in a synchronisation of all processes for the dot
// products.  Here one iteration is three kernels, all scalars stay in device
// memory, and the host never waits per iteration:
//   spmv_dot  : q = A p, partials of p.q
//   update_r  : alpha = rho / p.q; r -= alpha q, partials of r.r
//   update_xp : beta = r.r / rho; x += alpha p, p = r + beta p; stop test
// K iterations are captured once into a HIP graph and replayed.  The host
// keeps one graph ahead and polls a pinned copy of the solver state after
// each; once the state leaves "running" every kernel returns at entry, so
// the speculative graph changes nothing.
#include <chrono>
#include <cmath>
#include <vector>

#include "common.hpp"

// Iteration graphs kept per problem, keyed by solver kind, format, precision,
// solution buffer, graph length and state slot.
constexpr int kMaxGraphs = 16;

struct mfe_graph_cache {
    struct Entry {
        int kind;  // 0: CG, 1: single-reduction CG, 2: Jacobi-preconditioned CG
        int format;
        bool f32;
        const void *x;
        int k;
        const void *st;
        hipGraphExec_t exec;
    };
    std::vector<Entry> entries;
};

namespace mfe {

int ensure_workspace(mfe_problem *P) {
    mfe_ctx *ctx = P->ctx;
    const size_t vb = (size_t)P->m * sizeof(double);
    if (!P->r.ptr) MFE_TRY(dev_alloc(ctx, &P->r, vb));
    if (!P->p.ptr) MFE_TRY(dev_alloc(ctx, &P->p, vb));
    if (!P->q.ptr) MFE_TRY(dev_alloc(ctx, &P->q, vb));
    if (!P->state.ptr) {
        // [0]: the FP64 solve (or the outer refinement), [1]: the inner FP32 solve
        MFE_TRY(dev_alloc(ctx, &P->state, 2 * sizeof(CgState)));
        MFE_HIP_TRY(hipMemsetAsync(P->state.ptr, 0, 2 * sizeof(CgState), ctx->stream));
    }
    if (!P->partials.ptr) MFE_TRY(dev_alloc(ctx, &P->partials, 3 * kMaxPartials * sizeof(double)));
    if (!P->graphs) P->graphs = new mfe_graph_cache();
    return MFE_OK;
}

namespace {

// Capture k CG iterations on the context's private capture stream.  kind 0:
// SpMV + p.q, r update + r.r, x/p update; kind 1 (single reduction, FP64):
// w = A r with r.w and r.r, then the update of p, s, x, r.
int capture(mfe_problem *P, int kind, int format, bool f32, void *x, void *r, void *p, void *q, CgState *st,
            int k, hipGraphExec_t *out) {
    hipStream_t cs = P->ctx->cap_stream;
    double *partials = (double *)P->partials.ptr;
    MFE_HIP_TRY(hipStreamBeginCapture(cs, hipStreamCaptureModeThreadLocal));
    int rc = MFE_OK;
    double *pq_part = partials, *rr_part = partials + 2 * kMaxPartials;
    for (int i = 0; i < k && rc == MFE_OK; ++i) {
        if (kind == 2) {
            SpmvArgs a{p, q, nullptr, nullptr, st, pq_part};
            int n_pq = 0, n = 0;
            const double *dinv = (const double *)P->dinv.ptr;
            double *part = partials + kMaxPartials;  // r.z, and r.r one block further
            rc = launch_spmv(P, format, false, kSpmvDot, a, cs, &n_pq);
            if (rc == MFE_OK)
                rc = launch_pupdate_r(P, (double *)r, (const double *)q, dinv, st, pq_part, n_pq, part, &n, cs);
            if (rc == MFE_OK) rc = launch_pupdate_xp(P, (double *)x, (double *)p, (const double *)r, dinv, st, part, n, cs);
            continue;
        }
        if (kind == 1) {
            SpmvArgs a{r, q, nullptr, nullptr, st, partials};
            int n = 0;
            rc = launch_spmv(P, format, false, kSpmvDot2, a, cs, &n);
            if (rc == MFE_OK)
                rc = launch_sr_update(P, (double *)x, (double *)r, (double *)p, (double *)P->s.ptr,
                                      (const double *)q, st, partials, n, cs);
            continue;
        }
        SpmvArgs a{p, q, nullptr, nullptr, st, pq_part};
        int n_pq = 0, n_rr = 0;
        rc = launch_spmv(P, format, f32, kSpmvDot, a, cs, &n_pq);
        if (rc == MFE_OK) rc = launch_update_r(P, f32, r, q, st, pq_part, n_pq, rr_part, cs, &n_rr);
        if (rc == MFE_OK) rc = launch_update_xp(P, f32, x, p, r, st, rr_part, n_rr, cs);
    }
    hipGraph_t g = nullptr;
    const hipError_t e = hipStreamEndCapture(cs, &g);
    if (rc != MFE_OK) {
        if (g) (void)hipGraphDestroy(g);
        return rc;
    }
    if (e != hipSuccess) {
        set_error(std::string("hipStreamEndCapture failed: ") + hipGetErrorString(e));
        return MFE_EHIP;
    }
    const hipError_t e2 = hipGraphInstantiate(out, g, nullptr, nullptr, 0);
    (void)hipGraphDestroy(g);
    if (e2 != hipSuccess) {
        set_error(std::string("hipGraphInstantiate failed: ") + hipGetErrorString(e2));
        return MFE_EHIP;
    }
    return MFE_OK;
}

}  // namespace

int graph_for(mfe_problem *P, int format, bool f32, void *x, void *r, void *p, void *q, CgState *st, int k,
              hipGraphExec_t *out, int kind) {
    for (auto &e : P->graphs->entries)
        if (e.kind == kind && e.format == format && e.f32 == f32 && e.x == x && e.k == k && e.st == st) {
            *out = e.exec;
            return MFE_OK;
        }
    hipGraphExec_t ex = nullptr;
    MFE_TRY(capture(P, kind, format, f32, x, r, p, q, st, k, &ex));
    // bounded cache (callers that pass a new x buffer per solve would grow it
    // without end): drop the oldest graph once no work of the context uses it
    auto &v = P->graphs->entries;
    if (v.size() >= (size_t)kMaxGraphs) {
        const hipError_t e = hipStreamSynchronize(P->ctx->stream);
        if (e != hipSuccess) {
            (void)hipGraphExecDestroy(ex);
            set_error(std::string("hipStreamSynchronize failed: ") + hipGetErrorString(e));
            return MFE_EHIP;
        }
        (void)hipGraphExecDestroy(v.front().exec);
        v.erase(v.begin());
    }
    v.push_back({kind, format, f32, x, k, st, ex});
    *out = ex;
    return MFE_OK;
}

void release_graphs(mfe_problem *P) {
    if (!P->graphs) return;
    for (auto &e : P->graphs->entries) (void)hipGraphExecDestroy(e.exec);
    delete P->graphs;
    P->graphs = nullptr;
}

// Replay the iteration graph until the device state stops running.  On
// return *fin holds the final state.
int run_iterations(mfe_problem *P, hipGraphExec_t exec, const CgState *st, int k, int max_iter, CgState *fin) {
    mfe_ctx *ctx = P->ctx;
    hipStream_t s = ctx->stream;
    CgState *pin = (CgState *)ctx->pinned;
    const long limit = (long)max_iter / k + 3;  // the device cap ends the loop well before this
    long launched = 0;
    int slot = 0;
    MFE_HIP_TRY(hipGraphLaunch(exec, s));
    MFE_HIP_TRY(hipMemcpyAsync(&pin[0], st, sizeof(CgState), hipMemcpyDeviceToHost, s));
    MFE_HIP_TRY(hipEventRecord(ctx->ev[0], s));
    launched = 1;
    for (;;) {
        const int nxt = slot ^ 1;
        const bool more = launched < limit;
        if (more) {
            MFE_HIP_TRY(hipGraphLaunch(exec, s));
            MFE_HIP_TRY(hipMemcpyAsync(&pin[nxt], st, sizeof(CgState), hipMemcpyDeviceToHost, s));
            MFE_HIP_TRY(hipEventRecord(ctx->ev[nxt], s));
            ++launched;
        }
        MFE_HIP_TRY(hipEventSynchronize(ctx->ev[slot]));
        if (pin[slot].status != kRunning) {
            if (more) MFE_HIP_TRY(hipEventSynchronize(ctx->ev[nxt]));
            *fin = pin[slot];
            return MFE_OK;
        }
        if (!more) {
            set_error("CG state still running after the iteration cap");
            return MFE_EHIP;
        }
        slot = nxt;
    }
}

int cg_solve(mfe_problem *P, int format, double *x, double tol, int max_iter, double *hist,
             mfe_cg_stats *stats, bool warm) {
    const auto t0 = std::chrono::steady_clock::now();
    mfe_ctx *ctx = P->ctx;
    hipStream_t s = ctx->stream;
    MFE_TRY(ensure_workspace(P));
    CgState *st = (CgState *)P->state.ptr;
    double *partials = (double *)P->partials.ptr;
    CgState *pin = (CgState *)ctx->pinned;

    // initial state
    CgState h{};
    h.tol = tol;
    h.max_iter = max_iter;
    h.hist = hist;
    h.status = kRunning;
    h.warm = warm ? 1 : 0;
    pin[2] = h;
    MFE_HIP_TRY(hipMemcpyAsync(st, &pin[2], sizeof(CgState), hipMemcpyHostToDevice, s));
    // r = b - A x0, p = r, rho, ||b||, start test
    SpmvArgs a0{x, P->r.ptr, P->p.ptr, (const double *)P->b.ptr, st, partials};
    int n0 = 0;
    MFE_TRY(launch_spmv(P, format, false, kSpmvResid, a0, s, &n0));
    MFE_TRY(launch_finalize(kFinStart, partials, n0, st, s));
    MFE_TRY(launch_zero_if(P->m, x, (double *)P->r.ptr, (double *)P->p.ptr, (const double *)P->b.ptr, st,
                           ctx->num_cu, s));
    MFE_HIP_TRY(hipMemcpyAsync(&pin[0], st, sizeof(CgState), hipMemcpyDeviceToHost, s));
    MFE_HIP_TRY(hipStreamSynchronize(s));
    CgState fin = pin[0];
    int spmvs = 1;
    if (fin.status == kRunning) {
        const int k = kGraphIters < max_iter ? kGraphIters : max_iter;
        hipGraphExec_t exec = nullptr;
        MFE_TRY(graph_for(P, format, false, x, P->r.ptr, P->p.ptr, P->q.ptr, st, k, &exec));
        MFE_TRY(run_iterations(P, exec, st, k, max_iter, &fin));
        spmvs += fin.iters + (fin.status == kBreakdown ? 1 : 0);
    }
    // true residual ||b - A x|| in FP64
    SpmvArgs a1{x, nullptr, nullptr, (const double *)P->b.ptr, st, partials};
    int n1 = 0;
    MFE_TRY(launch_spmv(P, format, false, kSpmvTrue, a1, s, &n1));
    MFE_TRY(launch_finalize(kFinTrue, partials, n1, st, s));
    MFE_HIP_TRY(hipMemcpyAsync(&pin[0], st, sizeof(CgState), hipMemcpyDeviceToHost, s));
    MFE_HIP_TRY(hipStreamSynchronize(s));
    ++spmvs;
    const double rr_true = pin[0].rr_true;
    const double bn = fin.bnorm;
    int rc = MFE_OK;
    if (fin.status == kCapped) rc = MFE_NOT_CONVERGED;
    else if (fin.status == kBreakdown) rc = MFE_EBREAKDOWN;
    if (stats) {
        stats->status = rc;
        stats->iterations = fin.iters;
        stats->outer = 0;
        stats->spmv_count = spmvs;
        stats->rel_res_recurrence = bn > 0.0 ? std::sqrt(fin.rho) / bn : 0.0;
        stats->rel_res_true = bn > 0.0 ? std::sqrt(rr_true) / bn : 0.0;
        stats->seconds = std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
        stats->guess_rejected = fin.zero_x == 2 ? 1 : 0;
        stats->reserved_ = 0;
    }
    if (rc == MFE_EBREAKDOWN) set_error("CG breakdown: p.Ap <= 0 or not finite");
    return rc;
}

// Single-reduction CG: as cg_solve, with two kernels per iteration.  The
// loop's last SpMV evaluates the final r.r (the stopping test), so it
// issues iterations + 1 products.
int cg_sr_solve(mfe_problem *P, int format, double *x, double tol, int max_iter, double *hist,
                mfe_cg_stats *stats) {
    const auto t0 = std::chrono::steady_clock::now();
    mfe_ctx *ctx = P->ctx;
    hipStream_t s = ctx->stream;
    MFE_TRY(ensure_workspace(P));
    if (!P->s.ptr) MFE_TRY(dev_alloc(ctx, &P->s, (size_t)P->m * sizeof(double)));
    CgState *st = (CgState *)P->state.ptr;
    double *partials = (double *)P->partials.ptr;
    CgState *pin = (CgState *)ctx->pinned;
    CgState h{};
    h.tol = tol;
    h.max_iter = max_iter;
    h.hist = hist;
    h.status = kRunning;
    pin[2] = h;
    MFE_HIP_TRY(hipMemcpyAsync(st, &pin[2], sizeof(CgState), hipMemcpyHostToDevice, s));
    SpmvArgs a0{x, P->r.ptr, nullptr, (const double *)P->b.ptr, st, partials};
    int n0 = 0;
    MFE_TRY(launch_spmv(P, format, false, kSpmvResid, a0, s, &n0));
    MFE_TRY(launch_finalize(kFinStart, partials, n0, st, s));
    MFE_TRY(launch_zero_if(P->m, x, nullptr, nullptr, nullptr, st, ctx->num_cu, s));
    MFE_HIP_TRY(hipMemcpyAsync(&pin[0], st, sizeof(CgState), hipMemcpyDeviceToHost, s));
    MFE_HIP_TRY(hipStreamSynchronize(s));
    CgState fin = pin[0];
    int spmvs = 1;
    if (fin.status == kRunning) {
        const int k = kGraphIters < max_iter + 1 ? kGraphIters : max_iter + 1;
        hipGraphExec_t exec = nullptr;
        MFE_TRY(graph_for(P, format, false, x, P->r.ptr, P->p.ptr, P->q.ptr, st, k, &exec, 1));
        MFE_TRY(run_iterations(P, exec, st, k, max_iter + 1, &fin));
        spmvs += fin.iters + 1;
    }
    SpmvArgs a1{x, nullptr, nullptr, (const double *)P->b.ptr, st, partials};
    int n1 = 0;
    MFE_TRY(launch_spmv(P, format, false, kSpmvTrue, a1, s, &n1));
    MFE_TRY(launch_finalize(kFinTrue, partials, n1, st, s));
    MFE_HIP_TRY(hipMemcpyAsync(&pin[0], st, sizeof(CgState), hipMemcpyDeviceToHost, s));
    MFE_HIP_TRY(hipStreamSynchronize(s));
    ++spmvs;
    const double rr_true = pin[0].rr_true;
    const double bn = fin.bnorm;
    int rc = MFE_OK;
    if (fin.status == kCapped) rc = MFE_NOT_CONVERGED;
    else if (fin.status == kBreakdown) rc = MFE_EBREAKDOWN;
    if (stats) {
        stats->status = rc;
        stats->iterations = fin.iters;
        stats->outer = 0;
        stats->spmv_count = spmvs;
        stats->rel_res_recurrence = bn > 0.0 ? std::sqrt(fin.rho) / bn : 0.0;
        stats->rel_res_true = bn > 0.0 ? std::sqrt(rr_true) / bn : 0.0;
        stats->seconds = std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
        stats->guess_rejected = 0;
        stats->reserved_ = 0;
    }
    if (rc == MFE_EBREAKDOWN) set_error("single-reduction CG breakdown: r.Ar - beta r.r / alpha <= 0 or not finite");
    return rc;
}

// Jacobi-preconditioned CG: the CG driver with z = D^-1 r; the stopping test
// stays on the unpreconditioned ||r||/||b||.
int cg_jacobi_solve(mfe_problem *P, int format, double *x, double tol, int max_iter, double *hist,
                    mfe_cg_stats *stats) {
    const auto t0 = std::chrono::steady_clock::now();
    mfe_ctx *ctx = P->ctx;
    hipStream_t s = ctx->stream;
    MFE_TRY(ensure_workspace(P));
    MFE_TRY(build_dinv(P));
    CgState *st = (CgState *)P->state.ptr;
    double *partials = (double *)P->partials.ptr;
    CgState *pin = (CgState *)ctx->pinned;
    CgState h{};
    h.tol = tol;
    h.max_iter = max_iter;
    h.hist = hist;
    h.status = kRunning;
    pin[2] = h;
    MFE_HIP_TRY(hipMemcpyAsync(st, &pin[2], sizeof(CgState), hipMemcpyHostToDevice, s));
    // r = b - A x0, start test on r.r; then p = z = D^-1 r, rho = r.z
    SpmvArgs a0{x, P->r.ptr, nullptr, (const double *)P->b.ptr, st, partials};
    int n0 = 0;
    MFE_TRY(launch_spmv(P, format, false, kSpmvResid, a0, s, &n0));
    MFE_TRY(launch_finalize(kFinStart, partials, n0, st, s));
    MFE_TRY(launch_zero_if(P->m, x, nullptr, nullptr, nullptr, st, ctx->num_cu, s));
    MFE_TRY(launch_pcg_start(P, (const double *)P->r.ptr, (double *)P->p.ptr, (const double *)P->dinv.ptr, st,
                             partials + kMaxPartials, s));
    MFE_HIP_TRY(hipMemcpyAsync(&pin[0], st, sizeof(CgState), hipMemcpyDeviceToHost, s));
    MFE_HIP_TRY(hipStreamSynchronize(s));
    CgState fin = pin[0];
    int spmvs = 1;
    if (fin.status == kRunning) {
        const int k = kGraphIters < max_iter ? kGraphIters : max_iter;
        hipGraphExec_t exec = nullptr;
        MFE_TRY(graph_for(P, format, false, x, P->r.ptr, P->p.ptr, P->q.ptr, st, k, &exec, 2));
        MFE_TRY(run_iterations(P, exec, st, k, max_iter, &fin));
        spmvs += fin.iters + (fin.status == kBreakdown ? 1 : 0);
    }
    SpmvArgs a1{x, nullptr, nullptr, (const double *)P->b.ptr, st, partials};
    int n1 = 0;
    MFE_TRY(launch_spmv(P, format, false, kSpmvTrue, a1, s, &n1));
    MFE_TRY(launch_finalize(kFinTrue, partials, n1, st, s));
    MFE_HIP_TRY(hipMemcpyAsync(&pin[0], st, sizeof(CgState), hipMemcpyDeviceToHost, s));
    MFE_HIP_TRY(hipStreamSynchronize(s));
    ++spmvs;
    const double rr_true = pin[0].rr_true;
    const double bn = fin.bnorm;
    int rc = MFE_OK;
    if (fin.status == kCapped) rc = MFE_NOT_CONVERGED;
    else if (fin.status == kBreakdown) rc = MFE_EBREAKDOWN;
    if (stats) {
        stats->status = rc;
        stats->iterations = fin.iters;
        stats->outer = 0;
        stats->spmv_count = spmvs;
        // with b = 0 the start test ends the solve before rr is set
        stats->rel_res_recurrence = bn > 0.0 ? std::sqrt(fin.rr) / bn : 0.0;
        stats->rel_res_true = bn > 0.0 ? std::sqrt(rr_true) / bn : 0.0;
        stats->seconds = std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
        stats->guess_rejected = 0;
        stats->reserved_ = 0;
    }
    if (rc == MFE_EBREAKDOWN) set_error("Jacobi-preconditioned CG breakdown: p.Ap or r.z <= 0 or not finite");
    return rc;
}

}  // namespace mfe
