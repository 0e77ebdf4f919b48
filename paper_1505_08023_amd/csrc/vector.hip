// CG vector operations (Sec. 1 CG module: WAXPY and DOT) with the scalar
// recurrences kept on the device.
//
// One iteration is three kernels; each reduction is written as per-workgroup
// partials and summed, in a fixed order, at the start of every workgroup of
// the kernel that needs it (no atomics, no fences, no extra launch):
//   spmv_dot  : q = A p, partials of p.q                         (spmv.hip)
//   update_r  : pi = sum(p.q), alpha = rho / pi (breakdown test);
//               r -= alpha q, partials of r.r                  (reads r,q; writes r)
//   update_xp : rho' = sum(r.r), beta = rho' / rho;
//               x += alpha p, p = r + beta p; stopping test       (reads x,p,r; writes x,p)
// 64 bytes per row per iteration in FP64: the fewest for the two-reduction
// recurrence, since q must be stored between the p.q and r.r reductions.
#include "common.hpp"
#include "device_util.hpp"


namespace mfe {
namespace {

// 16-byte vector of T with only T's alignment (caller vectors need not be
// 16-byte aligned; gfx950 serves such accesses with one load or store).
template <typename T>
struct Vec16 {
    static constexpr int W = 16 / (int)sizeof(T);
    typedef T t __attribute__((ext_vector_type(16 / sizeof(T)), aligned(sizeof(T))));
};

template <typename T, bool NT>
__global__ __launch_bounds__(kBlock) void k_update_r(int64_t m, T *__restrict__ r, const T *__restrict__ q,
                                                     CgState *st, const double *__restrict__ pq_part, int n_pq,
                                                     double *__restrict__ rr_part) {
    if (st->status != kRunning) return;
    const double pq = sum_partials(pq_part, n_pq);
    const double rho = st->rho;
    if (!(pq > 0.0) || !isfinite(pq)) {
        if (blockIdx.x == 0 && threadIdx.x == 0) {
            st->pq = pq;
            st->status = kBreakdown;
        }
        return;
    }
    const double alpha = rho / pq;
    if (blockIdx.x == 0 && threadIdx.x == 0) {
        st->pq = pq;
        st->alpha = alpha;
        st->rho_old = rho;
        st->active = 1;
    }
    const T a = (T)alpha;
    double d = 0.0;
    const int64_t stride = (int64_t)gridDim.x * kBlock;
    const int64_t gid = (int64_t)blockIdx.x * kBlock + threadIdx.x;
    // 16 bytes per vector access (the pointers need only element alignment),
    // then the < W trailing elements (69.1 -> 64.9 us at 256^3)
    using V = Vec16<T>;
    constexpr int W = V::W;
    const int64_t mv = m / W;
    for (int64_t i = gid; i < mv; i += stride) {
        typename V::t rv = ((const typename V::t *)r)[i];
        const typename V::t qv = stream_load((const typename V::t *)q + i, NT);
#pragma unroll
        for (int j = 0; j < W; ++j) {
            const T ri = rv[j] - a * qv[j];
            rv[j] = ri;
            d += (double)ri * (double)ri;
        }
        ((typename V::t *)r)[i] = rv;
    }
    for (int64_t i = mv * W + gid; i < m; i += stride) {
        const T ri = r[i] - a * stream_load(q + i, NT);
        r[i] = ri;
        d += (double)ri * (double)ri;
    }
    d = block_sum(d);
    if (threadIdx.x == 0) rr_part[blockIdx.x] = d;
}

template <typename T, bool NT>
__global__ __launch_bounds__(kBlock) void k_update_xp(int64_t m, T *__restrict__ x, T *__restrict__ p,
                                                      const T *__restrict__ r, CgState *st,
                                                      const double *__restrict__ rr_part, int n_rr) {
    if (!st->active) return;
    const double rho_new = sum_partials(rr_part, n_rr);
    const double alpha = st->alpha, rho_old = st->rho_old;
    const double beta = rho_new / rho_old;
    if (blockIdx.x == 0 && threadIdx.x == 0) {
        const int it = st->iters + 1;
        const double res = sqrt(rho_new) / st->bnorm;
        st->iters = it;
        st->rho = rho_new;
        if (st->hist) st->hist[it] = res;
        if (!isfinite(res)) st->status = kBreakdown;
        else if (res <= st->tol) st->status = kConverged;
        else if (it >= st->max_iter) st->status = kCapped;
    }
    // p is updated even on the last iteration: the update is not needed then,
    // but deciding it would need the stopping test in every workgroup.
    // 16-byte accesses, then the < W trailing elements (at 256^3 on par with
    // 8-byte ones, which need twice the workgroups; 128^3 CG +2 %, 48^3 +5 %)
    const T a = (T)alpha, be = (T)beta;
    const int64_t stride = (int64_t)gridDim.x * kBlock;
    const int64_t gid = (int64_t)blockIdx.x * kBlock + threadIdx.x;
    using V = Vec16<T>;
    constexpr int W = V::W;
    const int64_t mv = m / W;
    for (int64_t i = gid; i < mv; i += stride) {
        const typename V::t pv = ((const typename V::t *)p)[i];
        typename V::t xv = stream_load((const typename V::t *)x + i, NT);
        typename V::t rv = stream_load((const typename V::t *)r + i, NT);
#pragma unroll
        for (int j = 0; j < W; ++j) {
            xv[j] = xv[j] + a * pv[j];
            rv[j] = rv[j] + be * pv[j];
        }
        stream_store(xv, (typename V::t *)x + i, NT);
        ((typename V::t *)p)[i] = rv;
    }
    for (int64_t i = mv * W + gid; i < m; i += stride) {
        const T pi = p[i];
        stream_store(stream_load(x + i, NT) + a * pi, x + i, NT);
        p[i] = stream_load(r + i, NT) + be * pi;
    }
}

// Single-reduction CG update (Chronopoulos-Gear).  The SpMV before it wrote
// w = A r with the partials of delta = r.w and gamma = r.r of the current r.
// Every workgroup sums them, applies the stopping test to gamma and, while
// running, forms
//   beta = gamma / gamma_prev,  alpha = gamma / (delta - beta gamma / alpha_prev)
// (beta = 0, alpha = gamma / delta on the first update), then
//   p = r + beta p,  s = w + beta s,  x += alpha p,  r -= alpha s.
// The previous gamma and alpha come from the ring slot of the other parity,
// and the entry test from the status the SpMV recorded: this kernel writes
// neither, so every wavefront of every workgroup takes the same branch.
// 72 bytes per row (FP64).
__global__ __launch_bounds__(kBlock) void k_sr_update(int64_t m, double *__restrict__ x, double *__restrict__ r,
                                                      double *__restrict__ p, double *__restrict__ s,
                                                      const double *__restrict__ w, CgState *st,
                                                      const double *__restrict__ part, int n) {
    if (st->status_snap != kRunning) return;
    const double delta = sum_partials(part, n);
    const double gamma = sum_partials(part + kMaxPartials, n);
    const int it = st->iters_snap;
    const double res = sqrt(gamma) / st->bnorm;
    const bool stop = !isfinite(res) || res <= st->tol || it >= st->max_iter;
    double beta = 0.0, denom = delta;
    if (it > 0) {
        beta = gamma / st->ring_g[(it + 1) & 1];
        denom = delta - beta * gamma / st->ring_a[(it + 1) & 1];
    }
    const bool brk = !stop && (!(denom > 0.0) || !isfinite(denom));
    const double alpha = gamma / denom;
    if (blockIdx.x == 0 && threadIdx.x == 0) {
        st->rho = gamma;
        if (it > 0 && st->hist) st->hist[it] = res;
        if (!isfinite(res)) st->status = kBreakdown;
        else if (res <= st->tol) st->status = kConverged;
        else if (it >= st->max_iter) st->status = kCapped;
        else if (brk) st->status = kBreakdown;
        st->pq = denom;
        if (!stop && !brk) {
            st->ring_g[it & 1] = gamma;
            st->ring_a[it & 1] = alpha;
            st->alpha = alpha;
            st->iters = it + 1;
        }
    }
    if (stop || brk) return;
    const int64_t stride = (int64_t)gridDim.x * kBlock;
    if (it == 0) {
        for (int64_t i = (int64_t)blockIdx.x * kBlock + threadIdx.x; i < m; i += stride) {
            const double ri = r[i], wi = w[i];
            p[i] = ri;
            s[i] = wi;
            x[i] += alpha * ri;
            r[i] = ri - alpha * wi;
        }
    } else {
        for (int64_t i = (int64_t)blockIdx.x * kBlock + threadIdx.x; i < m; i += stride) {
            const double ri = r[i];
            const double pi = ri + beta * p[i];
            const double si = w[i] + beta * s[i];
            p[i] = pi;
            s[i] = si;
            x[i] += alpha * pi;
            r[i] = ri - alpha * si;
        }
    }
}

// ------------------------------------------------------------ Jacobi-preconditioned CG
// Same three-kernel iteration as CG with z = D^-1 r formed on the fly:
//   update_r  : alpha = (r.z) / p.q; r -= alpha q; partials of r.z and r.r
//   update_xp : rho' = r.z, stop on sqrt(r.r)/||b||; x += alpha p, p = D^-1 r + beta p
// 80 bytes per row per iteration (the D^-1 vector is read twice).

__global__ __launch_bounds__(kBlock) void k_pcg_start(int64_t m, const double *__restrict__ r, double *__restrict__ p,
                                                      const double *__restrict__ dinv, CgState *st,
                                                      double *__restrict__ part) {
    double d = 0.0;
    const int64_t stride = (int64_t)gridDim.x * kBlock;
    for (int64_t i = (int64_t)blockIdx.x * kBlock + threadIdx.x; i < m; i += stride) {
        const double ri = r[i], zi = dinv[i] * ri;
        p[i] = zi;
        d += ri * zi;
    }
    d = block_sum(d);
    if (threadIdx.x == 0) part[blockIdx.x] = d;
}

// one workgroup: rr = r.r from the start test, rho = r.z
__global__ __launch_bounds__(kBlock) void k_pcg_start_fin(const double *__restrict__ part, int n, CgState *st) {
    const double rz = sum_partials(part, n);
    if (threadIdx.x != 0) return;
    st->rr = st->rho;
    st->rho = rz;
    if (st->status == kRunning && !(rz > 0.0 && isfinite(rz))) st->status = kBreakdown;
}

__global__ __launch_bounds__(kBlock) void k_pupdate_r(int64_t m, double *__restrict__ r, const double *__restrict__ q,
                                                      const double *__restrict__ dinv, CgState *st,
                                                      const double *__restrict__ pq_part, int n_pq,
                                                      double *__restrict__ part) {
    if (st->status != kRunning) return;
    const double pq = sum_partials(pq_part, n_pq);
    const double rho = st->rho;
    if (!(pq > 0.0) || !isfinite(pq)) {
        if (blockIdx.x == 0 && threadIdx.x == 0) {
            st->pq = pq;
            st->status = kBreakdown;
        }
        return;
    }
    const double alpha = rho / pq;
    if (blockIdx.x == 0 && threadIdx.x == 0) {
        st->pq = pq;
        st->alpha = alpha;
        st->rho_old = rho;
        st->active = 1;
    }
    double rz = 0.0, rr = 0.0;
    const int64_t stride = (int64_t)gridDim.x * kBlock;
    for (int64_t i = (int64_t)blockIdx.x * kBlock + threadIdx.x; i < m; i += stride) {
        const double ri = r[i] - alpha * q[i];
        r[i] = ri;
        rz += ri * (dinv[i] * ri);
        rr += ri * ri;
    }
    rz = block_sum(rz);
    rr = block_sum(rr);
    if (threadIdx.x == 0) {
        part[blockIdx.x] = rz;
        part[kMaxPartials + blockIdx.x] = rr;
    }
}

__global__ __launch_bounds__(kBlock) void k_pupdate_xp(int64_t m, double *__restrict__ x, double *__restrict__ p,
                                                       const double *__restrict__ r, const double *__restrict__ dinv,
                                                       CgState *st, const double *__restrict__ part, int n) {
    if (!st->active) return;
    const double rz = sum_partials(part, n);
    const double rr = sum_partials(part + kMaxPartials, n);  // a workgroup collective: every thread calls it
    const double alpha = st->alpha, beta = rz / st->rho_old;
    if (blockIdx.x == 0 && threadIdx.x == 0) {
        const int it = st->iters + 1;
        const double res = sqrt(rr) / st->bnorm;
        st->iters = it;
        st->rho = rz;
        st->rr = rr;
        if (st->hist) st->hist[it] = res;
        if (!isfinite(res)) st->status = kBreakdown;
        else if (res <= st->tol) st->status = kConverged;
        else if (it >= st->max_iter) st->status = kCapped;
    }
    const int64_t stride = (int64_t)gridDim.x * kBlock;
    for (int64_t i = (int64_t)blockIdx.x * kBlock + threadIdx.x; i < m; i += stride) {
        const double pi = p[i];
        x[i] += alpha * pi;
        p[i] = dinv[i] * r[i] + beta * pi;
    }
}

// 1 / A_ii from the FP64 CRS rows; bad[0] = 1 if a diagonal entry is zero,
// missing or not finite
__global__ __launch_bounds__(kBlock) void k_dinv(int64_t m, const int32_t *__restrict__ ptr,
                                                 const int32_t *__restrict__ col, const double *__restrict__ val,
                                                 double *__restrict__ dinv, int *__restrict__ bad) {
    const int64_t stride = (int64_t)gridDim.x * kBlock;
    for (int64_t i = (int64_t)blockIdx.x * kBlock + threadIdx.x; i < m; i += stride) {
        double d = 0.0;
        for (int32_t j = ptr[i]; j < ptr[i + 1]; ++j)
            if (col[j] == i) d = val[j];
        const bool ok = d != 0.0 && isfinite(d);
        dinv[i] = ok ? 1.0 / d : 0.0;
        if (!ok) bad[0] = 1;
    }
}

// One workgroup: reduce partials into the solver state.
template <int KIND>
__global__ __launch_bounds__(kBlock) void k_finalize(const double *__restrict__ part, int n, CgState *st) {
    const double s1 = sum_partials(part, n);
    double s2 = 0.0;
    if (KIND == kFinStart) s2 = sum_partials(part + kMaxPartials, n);
    if (threadIdx.x != 0) return;
    if (KIND == kFinStart) {
        // s1 = r0.r0, s2 = b.b: the start test of CG
        const double bnorm = sqrt(s2);
        st->bnorm = bnorm;
        st->iters = 0;
        st->active = 0;
        if (bnorm == 0.0) {
            st->rho = 0.0;
            st->zero_x = 1;
            st->status = kConverged;
            if (st->hist) st->hist[0] = 0.0;
        } else {
            double rho = s1;
            if (st->warm && s1 >= s2) {
                // the guess is no closer than x0 = 0: restart from zero (r = b)
                st->zero_x = 2;
                rho = s2;
            }
            st->rho = rho;
            const double res = sqrt(rho) / bnorm;
            if (st->hist) st->hist[0] = res;
            if (!isfinite(res)) st->status = kBreakdown;
            else if (res <= st->tol) st->status = kConverged;
            else if (st->max_iter <= 0) st->status = kCapped;
            else st->status = kRunning;
        }
    } else if (KIND == kFinTrue) {
        st->rr_true = s1;
    } else {
        st->pq = s1;
        if (st->dot_out) *st->dot_out = s1;
    }
}

__global__ __launch_bounds__(kBlock) void k_zero_if(int64_t m, double *__restrict__ x, double *__restrict__ r,
                                                    double *__restrict__ p, const double *__restrict__ b,
                                                    const CgState *st) {
    const int z = st->zero_x;
    if (!z) return;
    const int64_t stride = (int64_t)gridDim.x * kBlock;
    for (int64_t i = (int64_t)blockIdx.x * kBlock + threadIdx.x; i < m; i += stride) {
        x[i] = 0.0;
        if (z == 2) {
            const double bi = b[i];
            r[i] = bi;
            p[i] = bi;
        }
    }
}

__global__ __launch_bounds__(kBlock) void k_dot(int64_t n, const double *__restrict__ x,
                                                const double *__restrict__ y, double *__restrict__ part) {
    double d = 0.0;
    const int64_t stride = (int64_t)gridDim.x * kBlock;
    for (int64_t i = (int64_t)blockIdx.x * kBlock + threadIdx.x; i < n; i += stride) d += x[i] * y[i];
    d = block_sum(d);
    if (threadIdx.x == 0) part[blockIdx.x] = d;
}

__global__ void k_state_reset(CgState *st, double *dot_out) {
    st->rho = 1.0;
    st->status = kRunning;
    st->dot_out = dot_out;
}

int vec_grid(const void *kern, int64_t m, int num_cu) {
    return resident_grid((long)num_cu * resident_per_cu(kern), (long)((m + kBlock - 1) / kBlock));
}

// Streaming bandwidth probes (a reference for the bandwidth the kernels above
// reach): grid-stride 16-byte non-temporal accesses over n doubles.
__global__ __launch_bounds__(kBlock) void k_stream_copy(int64_t n, const double *__restrict__ src,
                                                        double *__restrict__ dst) {
    using V = Vec16<double>;
    const int64_t nv = n / 2, stride = (int64_t)gridDim.x * kBlock;
    const int64_t gid = (int64_t)blockIdx.x * kBlock + threadIdx.x;
    for (int64_t i = gid; i < nv; i += stride)
        __builtin_nontemporal_store(__builtin_nontemporal_load((const V::t *)src + i), (V::t *)dst + i);
    if (gid == 0 && (n & 1)) dst[n - 1] = src[n - 1];
}

// Reads n doubles and writes one partial sum per workgroup (so that no load
// can be dropped).
__global__ __launch_bounds__(kBlock) void k_stream_read(int64_t n, const double *__restrict__ src,
                                                        double *__restrict__ part) {
    using V = Vec16<double>;
    const int64_t nv = n / 2, stride = (int64_t)gridDim.x * kBlock;
    const int64_t gid = (int64_t)blockIdx.x * kBlock + threadIdx.x;
    double s = 0.0;
    for (int64_t i = gid; i < nv; i += stride) {
        const V::t v = __builtin_nontemporal_load((const V::t *)src + i);
        s += v[0] + v[1];
    }
    if (gid == 0 && (n & 1)) s += src[n - 1];
    s = block_sum(s);
    if (threadIdx.x == 0) part[blockIdx.x] = s;
}

}  // namespace

int launch_stream_probe(mfe_ctx *ctx, int kind, int64_t n, const double *src, double *dst) {
    const void *kern = kind == 0 ? (const void *)k_stream_copy : (const void *)k_stream_read;
    const int g = vec_grid(kern, (n + 1) / 2, ctx->num_cu);  // at most kMaxPartials workgroups
    if (kind == 0)
        hipLaunchKernelGGL(k_stream_copy, dim3(g), dim3(kBlock), 0, ctx->stream, n, src, dst);
    else
        hipLaunchKernelGGL(k_stream_read, dim3(g), dim3(kBlock), 0, ctx->stream, n, src, dst);
    MFE_HIP_TRY(hipGetLastError());
    return MFE_OK;
}

template <typename T, bool NT>
int update_r_as(const mfe_problem *P, void *r, const void *q, CgState *st, const double *pq_partials, int n_pq,
                double *rr_partials, hipStream_t s, int *grid) {
    // one thread per 16-byte chunk: a grid sized by elements would leave the
    // workgroups past m / W without rows (half of them in FP64, three
    // quarters in FP32) and their zero partials to the next kernel's sum;
    // the other workgroups keep their rows, so the sums are unchanged
    const int g = vec_grid((const void *)k_update_r<T, NT>, (P->m + Vec16<T>::W - 1) / Vec16<T>::W,
                           P->ctx->num_cu);
    hipLaunchKernelGGL((k_update_r<T, NT>), dim3(g), dim3(kBlock), 0, s, P->m, (T *)r, (const T *)q, st, pq_partials,
                       n_pq, rr_partials);
    MFE_HIP_TRY(hipGetLastError());
    if (grid) *grid = g;
    return MFE_OK;
}

template <typename T, bool NT>
int update_xp_as(const mfe_problem *P, void *x, void *p, const void *r, CgState *st, const double *rr_partials,
                 int n_rr, hipStream_t s) {
    // one thread per 16-byte chunk, as the r update
    const int g = vec_grid((const void *)k_update_xp<T, NT>, (P->m + Vec16<T>::W - 1) / Vec16<T>::W,
                           P->ctx->num_cu);
    hipLaunchKernelGGL((k_update_xp<T, NT>), dim3(g), dim3(kBlock), 0, s, P->m, (T *)x, (T *)p, (const T *)r, st,
                       rr_partials, n_rr);
    MFE_HIP_TRY(hipGetLastError());
    return MFE_OK;
}

int launch_update_r(const mfe_problem *P, bool f32, void *r, const void *q, CgState *st,
                    const double *pq_partials, int n_pq, double *rr_partials, hipStream_t s, int *grid) {
    const bool nt = vectors_stream_nt(P->m);
    if (f32)
        return nt ? update_r_as<float, true>(P, r, q, st, pq_partials, n_pq, rr_partials, s, grid)
                  : update_r_as<float, false>(P, r, q, st, pq_partials, n_pq, rr_partials, s, grid);
    return nt ? update_r_as<double, true>(P, r, q, st, pq_partials, n_pq, rr_partials, s, grid)
              : update_r_as<double, false>(P, r, q, st, pq_partials, n_pq, rr_partials, s, grid);
}

int launch_update_xp(const mfe_problem *P, bool f32, void *x, void *p, const void *r, CgState *st,
                     const double *rr_partials, int n_rr, hipStream_t s) {
    const bool nt = vectors_stream_nt(P->m);
    if (f32)
        return nt ? update_xp_as<float, true>(P, x, p, r, st, rr_partials, n_rr, s)
                  : update_xp_as<float, false>(P, x, p, r, st, rr_partials, n_rr, s);
    return nt ? update_xp_as<double, true>(P, x, p, r, st, rr_partials, n_rr, s)
              : update_xp_as<double, false>(P, x, p, r, st, rr_partials, n_rr, s);
}

int launch_pcg_start(const mfe_problem *P, const double *r, double *p, const double *dinv, CgState *st,
                     double *partials, hipStream_t s) {
    const int g = vec_grid((const void *)k_pcg_start, P->m, P->ctx->num_cu);
    hipLaunchKernelGGL(k_pcg_start, dim3(g), dim3(kBlock), 0, s, P->m, r, p, dinv, st, partials);
    hipLaunchKernelGGL(k_pcg_start_fin, dim3(1), dim3(kBlock), 0, s, (const double *)partials, g, st);
    MFE_HIP_TRY(hipGetLastError());
    return MFE_OK;
}

int launch_pupdate_r(const mfe_problem *P, double *r, const double *q, const double *dinv, CgState *st,
                     const double *pq_part, int n_pq, double *part, int *grid, hipStream_t s) {
    const int g = vec_grid((const void *)k_pupdate_r, P->m, P->ctx->num_cu);
    hipLaunchKernelGGL(k_pupdate_r, dim3(g), dim3(kBlock), 0, s, P->m, r, q, dinv, st, pq_part, n_pq, part);
    MFE_HIP_TRY(hipGetLastError());
    if (grid) *grid = g;
    return MFE_OK;
}

int launch_pupdate_xp(const mfe_problem *P, double *x, double *p, const double *r, const double *dinv, CgState *st,
                      const double *part, int n, hipStream_t s) {
    const int g = vec_grid((const void *)k_pupdate_xp, P->m, P->ctx->num_cu);
    hipLaunchKernelGGL(k_pupdate_xp, dim3(g), dim3(kBlock), 0, s, P->m, x, p, r, dinv, st, part, n);
    MFE_HIP_TRY(hipGetLastError());
    return MFE_OK;
}

int build_dinv(mfe_problem *P) {
    if (P->dinv.ptr) return MFE_OK;
    mfe_ctx *ctx = P->ctx;
    hipStream_t s = ctx->stream;
    MFE_TRY(dev_alloc(ctx, &P->dinv, (size_t)P->m * sizeof(double)));
    int *bad = (int *)ctx->scratch.ptr;
    int *hbad = (int *)((CgState *)ctx->pinned + 3);
    *hbad = 0;
    MFE_HIP_TRY(hipMemcpyAsync(bad, hbad, sizeof(int), hipMemcpyHostToDevice, s));
    const int g = vec_grid((const void *)k_dinv, P->m, ctx->num_cu);
    hipLaunchKernelGGL(k_dinv, dim3(g), dim3(kBlock), 0, s, P->m, (const int32_t *)P->ptr.ptr,
                       (const int32_t *)P->col.ptr, (const double *)P->val64.ptr, (double *)P->dinv.ptr, bad);
    MFE_HIP_TRY(hipGetLastError());
    MFE_HIP_TRY(hipMemcpyAsync(hbad, bad, sizeof(int), hipMemcpyDeviceToHost, s));
    MFE_HIP_TRY(hipStreamSynchronize(s));
    if (*hbad) {
        dev_free(ctx, &P->dinv);
        set_error("Jacobi preconditioner: a diagonal entry is zero, missing or not finite");
        return MFE_EINVAL;
    }
    return MFE_OK;
}

int launch_sr_update(const mfe_problem *P, double *x, double *r, double *p, double *s, const double *w, CgState *st,
                     const double *partials, int n, hipStream_t stream) {
    const int g = vec_grid((const void *)k_sr_update, P->m, P->ctx->num_cu);
    hipLaunchKernelGGL(k_sr_update, dim3(g), dim3(kBlock), 0, stream, P->m, x, r, p, s, w, st, partials, n);
    MFE_HIP_TRY(hipGetLastError());
    return MFE_OK;
}

int launch_finalize(FinalizeKind kind, const double *partials, int n, CgState *st, hipStream_t s) {
    switch (kind) {
        case kFinStart:
            hipLaunchKernelGGL(k_finalize<kFinStart>, dim3(1), dim3(kBlock), 0, s, partials, n, st);
            break;
        case kFinTrue:
            hipLaunchKernelGGL(k_finalize<kFinTrue>, dim3(1), dim3(kBlock), 0, s, partials, n, st);
            break;
        case kFinDot:
            hipLaunchKernelGGL(k_finalize<kFinDot>, dim3(1), dim3(kBlock), 0, s, partials, n, st);
            break;
    }
    MFE_HIP_TRY(hipGetLastError());
    return MFE_OK;
}

int launch_zero_if(int64_t m, double *x, double *r, double *p, const double *b, const CgState *st, int num_cu,
                   hipStream_t s) {
    const int g = vec_grid((const void *)k_zero_if, m, num_cu);
    hipLaunchKernelGGL(k_zero_if, dim3(g), dim3(kBlock), 0, s, m, x, r, p, b, st);
    MFE_HIP_TRY(hipGetLastError());
    return MFE_OK;
}

int launch_state_reset(CgState *st, double *dot_out, hipStream_t s) {
    hipLaunchKernelGGL(k_state_reset, dim3(1), dim3(1), 0, s, st, dot_out);
    MFE_HIP_TRY(hipGetLastError());
    return MFE_OK;
}

int launch_dot(mfe_ctx *ctx, int64_t n, const double *x, const double *y, double *partials, hipStream_t s,
               int *grid) {
    const int g = vec_grid((const void *)k_dot, n, ctx->num_cu);
    hipLaunchKernelGGL(k_dot, dim3(g), dim3(kBlock), 0, s, n, x, y, partials);
    MFE_HIP_TRY(hipGetLastError());
    if (grid) *grid = g;
    return MFE_OK;
}

}  // namespace mfe
