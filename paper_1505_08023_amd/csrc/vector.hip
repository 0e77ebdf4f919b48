// CG vector operations (Sec. 1 CG module: WAXPY and DOT) with the scalar
// recurrences kept on the device.
//
// Per iteration, after the fused SpMV + p.q kernel has set alpha:
//   update_r : r -= alpha q, partial r.r; the last workgroup forms rho_new,
//              the stopping test, beta = rho_new / rho.     (reads r,q; writes r)
//   update_xp: x += alpha p; p = r + beta p.                 (reads x,p,r; writes x,p)
// 64 bytes per row per iteration in FP64, the fewest for the two-reduction
// recurrence since q must be stored between the p.q and r.r reductions.
#include "common.hpp"
#include "device_util.hpp"

namespace mfe {
namespace {

template <typename T>
__global__ __launch_bounds__(kBlock) void k_update_r(int64_t m, T *__restrict__ r, const T *__restrict__ q,
                                                     CgState *st, double *partials) {
    if (st->status != kRunning) return;
    const T a = (T)st->alpha;
    double d = 0.0;
    const int64_t stride = (int64_t)gridDim.x * kBlock;
    for (int64_t i = (int64_t)blockIdx.x * kBlock + threadIdx.x; i < m; i += stride) {
        const T ri = r[i] - a * q[i];
        r[i] = ri;
        d += (double)ri * (double)ri;
    }
    d = block_sum(d);
    if (threadIdx.x == 0) put_partial(partials, blockIdx.x, d);
    if (!arrive_last(&st->counter[0])) return;
    const double rho_new = sum_partials(partials, gridDim.x);
    if (threadIdx.x != 0) return;
    const int it = st->iters + 1;
    st->iters = it;
    const double res = sqrt(rho_new) / st->bnorm;
    if (st->hist) st->hist[it] = res;
    st->beta = rho_new / st->rho;
    st->rho = rho_new;
    st->xpending = 1;
    if (!isfinite(res)) st->status = kBreakdown;
    else if (res <= st->tol) st->status = kConverged;
    else if (it >= st->max_iter) st->status = kCapped;
}

template <typename T>
__global__ __launch_bounds__(kBlock) void k_update_xp(int64_t m, T *__restrict__ x, T *__restrict__ p,
                                                      const T *__restrict__ r, const CgState *st) {
    if (!st->xpending) return;
    const T a = (T)st->alpha, be = (T)st->beta;
    const bool next = st->status == kRunning;  // p is needed only if another iteration follows
    const int64_t stride = (int64_t)gridDim.x * kBlock;
    if (next) {
        for (int64_t i = (int64_t)blockIdx.x * kBlock + threadIdx.x; i < m; i += stride) {
            const T pi = p[i];
            x[i] += a * pi;
            p[i] = r[i] + be * pi;
        }
    } else {
        for (int64_t i = (int64_t)blockIdx.x * kBlock + threadIdx.x; i < m; i += stride) x[i] += a * p[i];
    }
}

__global__ __launch_bounds__(kBlock) void k_zero_if(int64_t m, double *__restrict__ x, const CgState *st) {
    if (!st->zero_x) return;
    const int64_t stride = (int64_t)gridDim.x * kBlock;
    for (int64_t i = (int64_t)blockIdx.x * kBlock + threadIdx.x; i < m; i += stride) x[i] = 0.0;
}

__global__ __launch_bounds__(kBlock) void k_dot(int64_t n, const double *__restrict__ x,
                                                const double *__restrict__ y, CgState *st, double *partials) {
    double d = 0.0;
    const int64_t stride = (int64_t)gridDim.x * kBlock;
    for (int64_t i = (int64_t)blockIdx.x * kBlock + threadIdx.x; i < n; i += stride) d += x[i] * y[i];
    d = block_sum(d);
    if (threadIdx.x == 0) put_partial(partials, blockIdx.x, d);
    if (!arrive_last(&st->counter[0])) return;
    const double s = sum_partials(partials, gridDim.x);
    if (threadIdx.x == 0) st->pq = s;
}

__global__ void k_state_reset(CgState *st, double *dot_out) {
    st->rho = 1.0;
    st->status = kRunning;
    st->dot_out = dot_out;
}

int vec_grid(const void *kern, int64_t m, int num_cu) {
    return resident_grid((long)num_cu * resident_per_cu(kern), (long)((m + kBlock - 1) / kBlock));
}

}  // namespace

int launch_update_r(const mfe_problem *P, bool f32, void *r, const void *q, CgState *st, double *partials,
                    hipStream_t s) {
    if (f32) {
        const int g = vec_grid((const void *)k_update_r<float>, P->m, P->ctx->num_cu);
        hipLaunchKernelGGL(k_update_r<float>, dim3(g), dim3(kBlock), 0, s, P->m, (float *)r, (const float *)q,
                           st, partials);
    } else {
        const int g = vec_grid((const void *)k_update_r<double>, P->m, P->ctx->num_cu);
        hipLaunchKernelGGL(k_update_r<double>, dim3(g), dim3(kBlock), 0, s, P->m, (double *)r,
                           (const double *)q, st, partials);
    }
    MFE_HIP_TRY(hipGetLastError());
    return MFE_OK;
}

int launch_update_xp(const mfe_problem *P, bool f32, void *x, void *p, const void *r, CgState *st,
                     hipStream_t s) {
    if (f32) {
        const int g = vec_grid((const void *)k_update_xp<float>, P->m, P->ctx->num_cu);
        hipLaunchKernelGGL(k_update_xp<float>, dim3(g), dim3(kBlock), 0, s, P->m, (float *)x, (float *)p,
                           (const float *)r, st);
    } else {
        const int g = vec_grid((const void *)k_update_xp<double>, P->m, P->ctx->num_cu);
        hipLaunchKernelGGL(k_update_xp<double>, dim3(g), dim3(kBlock), 0, s, P->m, (double *)x, (double *)p,
                           (const double *)r, st);
    }
    MFE_HIP_TRY(hipGetLastError());
    return MFE_OK;
}

int launch_zero_if(int64_t m, double *x, const CgState *st, int num_cu, hipStream_t s) {
    const int g = vec_grid((const void *)k_zero_if, m, num_cu);
    hipLaunchKernelGGL(k_zero_if, dim3(g), dim3(kBlock), 0, s, m, x, st);
    MFE_HIP_TRY(hipGetLastError());
    return MFE_OK;
}

int launch_state_reset(CgState *st, double *dot_out, hipStream_t s) {
    hipLaunchKernelGGL(k_state_reset, dim3(1), dim3(1), 0, s, st, dot_out);
    MFE_HIP_TRY(hipGetLastError());
    return MFE_OK;
}

int launch_dot(mfe_ctx *ctx, int64_t n, const double *x, const double *y, double *partials, CgState *st,
               hipStream_t s) {
    const int g = vec_grid((const void *)k_dot, n, ctx->num_cu);
    hipLaunchKernelGGL(k_dot, dim3(g), dim3(kBlock), 0, s, n, x, y, st, partials);
    MFE_HIP_TRY(hipGetLastError());
    return MFE_OK;
}

}  // namespace mfe
