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
// a speculative graph changes nothing.  It still costs its launches (a
// kernel that returns at entry takes several microseconds to dispatch), so
// once the residual history forecasts the end of the solve the host switches
// to graphs of kTailIters iterations, and launches none ahead when the end is
// forecast within the graphs already in flight.
#include <algorithm>
#include <chrono>
#include <cmath>
#include <vector>

#include "common.hpp"

#ifndef MFE_CG_TAIL
#define MFE_CG_TAIL 1  // short graphs at the forecast end of a solve, none launched ahead past it (0: fixed length)
#endif

// Iteration graphs kept per problem, keyed by solver kind, format, precision,
// solution buffer, graph length and state slot.
constexpr int kMaxGraphs = 32;

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

double Forecast::observe(int i, double res, double tol) {
    if (!(res > 0.0) || !std::isfinite(res)) return 0.0;
    const double l = std::log(res);
    if (it >= 0 && i > it) {
        const double d = (l - lr) / (i - it);
        if (d < 0.0 && std::isfinite(d)) slope = d;  // a stall keeps the previous rate
    }
    it = i;
    lr = l;
    if (res <= tol) return 0.0;
    if (!(slope < 0.0)) return 1e30;
    return (std::log(tol) - l) / slope;
}

double stop_residual(const CgState &s, int kind) {
    const double v = kind == 2 ? s.rr : s.rho;
    return s.bnorm > 0.0 && v >= 0.0 ? std::sqrt(v) / s.bnorm : 0.0;
}

void record_rate(mfe_problem *P, int slot, double res0, const CgState &fin, int kind) {
    const double res = stop_residual(fin, kind);
    if (fin.iters > 0 && res0 > 0.0 && res > 0.0 && std::isfinite(res0) && std::isfinite(res)) {
        const double r = (std::log(res) - std::log(res0)) / fin.iters;
        if (r < 0.0) P->rate[slot] = r;
    }
}

int iteration_graphs(mfe_problem *P, int format, bool f32, void *x, void *r, void *p, void *q, CgState *st,
                     int max_iter, int kind, IterGraphs *G) {
    G->k = kGraphIters < max_iter ? kGraphIters : max_iter;
    MFE_TRY(graph_for(P, format, f32, x, r, p, q, st, G->k, &G->exec, kind));
    G->tail = nullptr;
    G->kt = 0;
    if (MFE_CG_TAIL && G->k > kTailIters) {
        G->kt = kTailIters;
        MFE_TRY(graph_for(P, format, f32, x, r, p, q, st, G->kt, &G->tail, kind));
    }
    return MFE_OK;
}

// Replay the iteration graphs until the device state stops running.  Up to
// two graphs are in flight, each followed by a copy of the state to its
// pinned slot (0 or 1) and an event.  Before waiting for the older one the
// host launches the next, unless the forecast puts the end of the solve
// within the iterations already launched; it launches the tail graph when
// the end is forecast within one more long graph.  rem: the forecast at the
// start (1e30 if unknown).  On return *fin holds the final state.
int run_iterations(mfe_problem *P, const IterGraphs &G, const CgState *st, int max_iter, int kind, Forecast &fc,
                   double rem, CgState *fin) {
    mfe_ctx *ctx = P->ctx;
    hipStream_t s = ctx->stream;
    CgState *pin = (CgState *)ctx->pinned;
    const long limit = (long)max_iter + 2L * G.k;  // iterations launched at most; the device cap ends the loop first
    long launched = 0, polled = 0;                 // iterations launched, and done at the last poll
    int head = 0, count = 0;                       // in-flight graphs occupy slots head, head ^ 1
    for (;;) {
        while (count < 2 && launched < limit) {
            const long ahead = launched - polled;
            // the device stops at max_iter in any case
            const double r = std::min(rem, (double)(max_iter - polled));
            if (MFE_CG_TAIL && count > 0 && r <= (double)ahead) break;  // the end is forecast within the graphs in flight
            const bool tail = G.tail && r <= (double)(ahead + G.k);
            const int slot = (head + count) & 1;
            MFE_HIP_TRY(hipGraphLaunch(tail ? G.tail : G.exec, s));
            MFE_HIP_TRY(hipMemcpyAsync(&pin[slot], st, sizeof(CgState), hipMemcpyDeviceToHost, s));
            MFE_HIP_TRY(hipEventRecord(ctx->ev[slot], s));
            launched += tail ? G.kt : G.k;
            ++count;
        }
        if (count == 0) {
            set_error("CG state still running after the iteration cap");
            return MFE_EHIP;
        }
        const int slot = head;
        MFE_HIP_TRY(hipEventSynchronize(ctx->ev[slot]));
        head ^= 1;
        --count;
        const CgState cur = pin[slot];
        if (cur.status != kRunning) {
            if (count > 0) MFE_HIP_TRY(hipEventSynchronize(ctx->ev[head]));
            *fin = cur;
            return MFE_OK;
        }
        polled = cur.iters;
        rem = fc.observe(cur.iters, stop_residual(cur, kind), cur.tol);
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
        IterGraphs G;
        MFE_TRY(iteration_graphs(P, format, false, x, P->r.ptr, P->p.ptr, P->q.ptr, st, max_iter, 0, &G));
        Forecast fc;
        fc.slope = P->rate[0];
        const double res0 = stop_residual(fin, 0);
        MFE_TRY(run_iterations(P, G, st, max_iter, 0, fc, fc.observe(0, res0, tol), &fin));
        record_rate(P, 0, res0, fin, 0);
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
        IterGraphs G;
        MFE_TRY(iteration_graphs(P, format, false, x, P->r.ptr, P->p.ptr, P->q.ptr, st, max_iter + 1, 1, &G));
        Forecast fc;
        fc.slope = P->rate[1];
        const double res0 = stop_residual(fin, 1);
        MFE_TRY(run_iterations(P, G, st, max_iter + 1, 1, fc, fc.observe(0, res0, tol), &fin));
        record_rate(P, 1, res0, fin, 1);
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
        IterGraphs G;
        MFE_TRY(iteration_graphs(P, format, false, x, P->r.ptr, P->p.ptr, P->q.ptr, st, max_iter, 2, &G));
        Forecast fc;
        fc.slope = P->rate[2];
        const double res0 = stop_residual(fin, 2);
        MFE_TRY(run_iterations(P, G, st, max_iter, 2, fc, fc.observe(0, res0, tol), &fin));
        record_rate(P, 2, res0, fin, 2);
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
