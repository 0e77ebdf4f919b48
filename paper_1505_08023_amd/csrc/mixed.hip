// Mixed precision: FP32 inner CG inside FP64 iterative refinement.
//
// Outer step (FP64):  r = b - A x with the FP64 matrix; stop when
//                     ||r|| / ||b|| <= tol; s = ||r||.
// Inner solve (FP32): A32 d = fl32(r / s) by the same CG kernels as the
//                     FP64 solve, instantiated for float (FP32 matrix
//                     values, FP32 SpMV sums and vector updates; both dot
//                     products accumulate in FP64 and alpha, beta are
//                     formed in FP64), from d = 0 to ||r_inner|| <=
//                     max(inner_tol, tol ||b|| / (2 s)): no tighter than
//                     the outer target needs.
// Update (FP64):      x += s d.
// The inner solve streams half the matrix bytes of an FP64 iteration; the
// FP64 residual keeps the final accuracy independent of FP32 rounding.  A
// refinement step that does not halve the residual switches to FP64 CG.
//
// With keep_direction, an inner solve that met its tolerance is not
// restarted at the next step: its recursive residual is replaced by the new
// FP64 residual (a reliable update of the residual, after Sleijpen and van
// der Vorst) and its recurrence goes on from the last direction, carried to
// the new scale.  At exit the inner CG has already formed p = r + beta P
// (P the last direction, r its recursive residual), so with s_old, s the
// previous and the new residual norms
//     r32 = fl32(r / s),   p32 = r32 + (s_old / s) (p32 - r32_old),
// the CG step P_next = R + beta P in the new scale with the FP64 residual
// for R.  In exact arithmetic the two residuals agree and the inner
// iterations are those of one uninterrupted CG.
#include <chrono>
#include <cmath>

#include "common.hpp"
#include "device_util.hpp"

namespace mfe {
namespace {

// r32 = fl32(r * inv_s), p32 = r32, d32 = 0; partials of r32.r32 (FP64) in
// both slots the start finalizer reads (the inner system's b is r32).
__global__ __launch_bounds__(kBlock) void k_mixed_start(int64_t m, const double *__restrict__ r,
                                                        const CgState *outer, float *__restrict__ r32,
                                                        float *__restrict__ p32, float *__restrict__ d32,
                                                        double *__restrict__ part) {
    const double s = sqrt(outer->rho);
    double acc = 0.0;
    const int64_t stride = (int64_t)gridDim.x * kBlock;
    for (int64_t i = (int64_t)blockIdx.x * kBlock + threadIdx.x; i < m; i += stride) {
        const float v = (float)(r[i] / s);
        r32[i] = v;
        p32[i] = v;
        d32[i] = 0.0f;
        acc += (double)v * (double)v;
    }
    acc = block_sum(acc);
    if (threadIdx.x == 0) {
        part[blockIdx.x] = acc;
        part[kMaxPartials + blockIdx.x] = acc;
    }
}

// Continued inner solve: r32 = fl32(r / s), p32 = r32 + fl32(s_old / s) (p32 - r32_old), d32 = 0;
// partials of r32.r32 in both slots, as k_mixed_start.
__global__ __launch_bounds__(kBlock) void k_mixed_continue(int64_t m, const double *__restrict__ r,
                                                           const CgState *outer, double s_old,
                                                           float *__restrict__ r32, float *__restrict__ p32,
                                                           float *__restrict__ d32, double *__restrict__ part) {
    const double s = sqrt(outer->rho);
    const float c = (float)(s_old / s);
    double acc = 0.0;
    const int64_t stride = (int64_t)gridDim.x * kBlock;
    for (int64_t i = (int64_t)blockIdx.x * kBlock + threadIdx.x; i < m; i += stride) {
        const float v = (float)(r[i] / s);
        p32[i] = v + c * (p32[i] - r32[i]);
        r32[i] = v;
        d32[i] = 0.0f;
        acc += (double)v * (double)v;
    }
    acc = block_sum(acc);
    if (threadIdx.x == 0) {
        part[blockIdx.x] = acc;
        part[kMaxPartials + blockIdx.x] = acc;
    }
}

// x += s d (FP64), s = ||r|| of the outer residual.
__global__ __launch_bounds__(kBlock) void k_mixed_update(int64_t m, double *__restrict__ x,
                                                         const float *__restrict__ d32, const CgState *outer) {
    const double s = sqrt(outer->rho);
    const int64_t stride = (int64_t)gridDim.x * kBlock;
    for (int64_t i = (int64_t)blockIdx.x * kBlock + threadIdx.x; i < m; i += stride) x[i] += s * (double)d32[i];
}

int vgrid(const void *kern, int64_t m, int num_cu) {
    return resident_grid((long)num_cu * resident_per_cu(kern), (long)((m + kBlock - 1) / kBlock));
}

int ensure_mixed(mfe_problem *P) {
    mfe_ctx *ctx = P->ctx;
    const size_t fb = (size_t)P->m * sizeof(float);
    if (!P->r32.ptr) MFE_TRY(dev_alloc(ctx, &P->r32, fb));
    if (!P->p32.ptr) MFE_TRY(dev_alloc(ctx, &P->p32, fb));
    if (!P->q32.ptr) MFE_TRY(dev_alloc(ctx, &P->q32, fb));
    if (!P->d32.ptr) MFE_TRY(dev_alloc(ctx, &P->d32, fb));
    return MFE_OK;
}

// Outer residual r = b - A x (FP64) into P->r and the outer state.
int outer_residual(mfe_problem *P, int format, double *x, CgState *outer, CgState *host) {
    mfe_ctx *ctx = P->ctx;
    hipStream_t s = ctx->stream;
    double *partials = (double *)P->partials.ptr;
    SpmvArgs a{x, P->r.ptr, nullptr, (const double *)P->b.ptr, outer, partials};
    int n = 0;
    MFE_TRY(launch_spmv(P, format, false, kSpmvResid, a, s, &n));
    MFE_TRY(launch_finalize(kFinStart, partials, n, outer, s));
    CgState *pin = (CgState *)ctx->pinned;
    MFE_HIP_TRY(hipMemcpyAsync(&pin[0], outer, sizeof(CgState), hipMemcpyDeviceToHost, s));
    MFE_HIP_TRY(hipStreamSynchronize(s));
    *host = pin[0];
    return MFE_OK;
}

// A fresh solver state (tolerance, cap, running), written on the device so
// that no host round trip separates the refinement steps.
__global__ void k_state_init(CgState *st, double tol, int max_iter, int warm) {
    CgState h{};
    h.tol = tol;
    h.max_iter = max_iter;
    h.status = kRunning;
    h.warm = warm;
    *st = h;
}

int set_state(mfe_ctx *ctx, CgState *dev, double tol, int max_iter, bool warm = false) {
    hipLaunchKernelGGL(k_state_init, dim3(1), dim3(1), 0, ctx->stream, dev, tol, max_iter, warm ? 1 : 0);
    MFE_HIP_TRY(hipGetLastError());
    return MFE_OK;
}

}  // namespace

int cg_mixed_solve(mfe_problem *P, int format, double *x, double tol, double inner_tol, int max_outer,
                   int max_inner, mfe_cg_stats *stats, bool warm, bool keep_direction) {
    const auto t0 = std::chrono::steady_clock::now();
    mfe_ctx *ctx = P->ctx;
    hipStream_t s = ctx->stream;
    MFE_TRY(ensure_workspace(P));
    MFE_TRY(ensure_mixed(P));
    CgState *outer = (CgState *)P->state.ptr;
    CgState *inner = outer + 1;
    double *partials = (double *)P->partials.ptr;
    float *r32 = (float *)P->r32.ptr, *p32 = (float *)P->p32.ptr, *q32 = (float *)P->q32.ptr,
          *d32 = (float *)P->d32.ptr;

    // outer tolerance test uses the start finalizer: max_iter 1 keeps it
    // "running"; with warm, a guess with ||b - A x0|| >= ||b|| is replaced by
    // x0 = 0 (r = b) on the device, as in the FP64 warm start
    MFE_TRY(set_state(ctx, outer, tol, 1, warm));
    CgState o;
    MFE_TRY(outer_residual(P, format, x, outer, &o));
    const double bnorm = o.bnorm;
    int nouter = 0, inner_its = 0, spmvs = 1, rc = MFE_OK;
    bool fallback = false;
    const bool rejected = o.zero_x == 2;
    double prev = o.bnorm > 0 ? std::sqrt(o.rho) : 0.0;
    bool have_dir = false;  // the last inner solve met its tolerance: its direction can go on
    double s_old = 0.0;
    if (o.zero_x)
        MFE_TRY(launch_zero_if(P->m, x, (double *)P->r.ptr, (double *)P->p.ptr, (const double *)P->b.ptr, outer,
                               ctx->num_cu, s));
    while (o.status == kRunning) {
        if (nouter >= max_outer) {
            rc = MFE_NOT_CONVERGED;
            break;
        }
        // inner FP32 solve of A32 d = fl32(r / s).  It need not go further than
        // the outer target (with a factor 2 margin): on the last step that is
        // usually a much looser tolerance than inner_tol.
        double eff = inner_tol;
        const double need = 0.5 * tol * bnorm / prev;
        if (need > eff) eff = need < 0.5 ? need : 0.5;
        MFE_TRY(set_state(ctx, inner, eff, max_inner));
        const int g = vgrid((const void *)k_mixed_start, P->m, ctx->num_cu);
        if (keep_direction && have_dir)
            hipLaunchKernelGGL(k_mixed_continue, dim3(g), dim3(kBlock), 0, s, P->m, (const double *)P->r.ptr,
                               outer, s_old, r32, p32, d32, partials);
        else
            hipLaunchKernelGGL(k_mixed_start, dim3(g), dim3(kBlock), 0, s, P->m, (const double *)P->r.ptr, outer,
                               r32, p32, d32, partials);
        MFE_HIP_TRY(hipGetLastError());
        MFE_TRY(launch_finalize(kFinStart, partials, g, inner, s));
        CgState in{};
        IterGraphs G;
        MFE_TRY(iteration_graphs(P, format, true, d32, r32, p32, q32, inner, max_inner, 0, &G));
        // the inner solve starts at relative residual 1 (its right-hand side is
        // its starting residual)
        Forecast fc;
        fc.slope = P->rate[3];
        MFE_TRY(run_iterations(P, G, inner, max_inner, 0, fc, fc.observe(0, 1.0, eff), &in));
        record_rate(P, 3, 1.0, in, 0);
        inner_its += in.iters;
        spmvs += in.iters;
        ++nouter;
        if (in.status == kBreakdown) {
            fallback = true;
            break;
        }
        have_dir = in.status == kConverged;
        s_old = prev;
        const int gu = vgrid((const void *)k_mixed_update, P->m, ctx->num_cu);
        hipLaunchKernelGGL(k_mixed_update, dim3(gu), dim3(kBlock), 0, s, P->m, x, (const float *)d32, outer);
        MFE_HIP_TRY(hipGetLastError());
        MFE_TRY(set_state(ctx, outer, tol, 1));
        MFE_TRY(outer_residual(P, format, x, outer, &o));
        ++spmvs;
        const double cur = std::sqrt(o.rho);
        if (o.status == kRunning && !(cur <= 0.5 * prev)) {
            fallback = true;  // refinement stagnates at FP32 accuracy
            break;
        }
        prev = cur;
    }
    double rel_true = bnorm > 0 ? std::sqrt(o.rho) / bnorm : 0.0;
    int total_its = inner_its;
    if (fallback) {
        mfe_cg_stats fs{};
        rc = cg_solve(P, format, x, tol, max_inner * (max_outer > 1 ? max_outer : 1), nullptr, &fs);
        total_its += fs.iterations;
        spmvs += fs.spmv_count;
        rel_true = fs.rel_res_true;
    }
    if (stats) {
        stats->status = rc;
        stats->iterations = total_its;
        stats->outer = nouter;
        stats->spmv_count = spmvs;
        stats->rel_res_recurrence = rel_true;
        stats->rel_res_true = rel_true;
        stats->seconds = std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
        stats->guess_rejected = rejected ? 1 : 0;
        stats->reserved_ = 0;
    }
    return rc;
}

}  // namespace mfe
