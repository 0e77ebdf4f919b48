// Batched CG over many box meshes of uneven size (the batched extension of
// the Sec. 1 CG module): every system follows exactly the single-system CG
// recurrence with its own alpha, beta, norm and stopping test, and a
// converged system is frozen while the others continue.
//
// The systems are assembled into one block-diagonal matrix.  Workgroups are
// assigned to systems in proportion to their rows (each workgroup owns one
// contiguous row chunk of one system), so every per-system reduction is the
// fixed-order sum of that system's workgroup partials, formed at the start of
// the consuming kernel by each of the system's workgroups: one iteration of
// all systems is three kernels (SpMV + p.q, r update + r.r, x/p update), K
// iterations are captured in one HIP graph, and the host polls the system
// states once per graph.  The grid is a multiple of the resident capacity so
// that CUs freed by frozen systems take on the remaining work.  An autotuner
// picks the CRS lanes per row (rows per wavefront) and the grid multiple by
// timing the SpMV kernel on the batch itself.
#include <algorithm>
#include <chrono>
#include <cmath>
#include <new>
#include <vector>

#include "common.hpp"
#include "device_util.hpp"
#include "spmv_rows.hpp"

#ifndef MFE_CG_TAIL
#define MFE_CG_TAIL 1  // short graphs at the forecast end of a solve (0: fixed length)
#endif
#ifndef MFE_BATCH_SCALAR_WALK
#define MFE_BATCH_SCALAR_WALK 1  // 1x3 BCRS, one slice per wavefront: the scalar read-ahead walk
#endif

namespace mfe {
namespace {

struct Map {
    const int32_t *wg_sys;  // system of each workgroup
    const int64_t *wg_lo;   // first row of each workgroup's chunk
    const int64_t *wg_hi;   // one past its last row
    const int32_t *sys_wg;  // first workgroup of each system [nsys + 1]
};

struct Tuning {
    int lanes = 32;   // CRS lanes per row
    int factor = 1;   // grid = factor x resident workgroups
};

// Sum of the partials of system `sys` (its workgroups' entries), fixed order,
// returned to every thread.
__device__ __forceinline__ double sys_sum(const double *__restrict__ part, const Map &M, int sys) {
    return sum_partials(part + M.sys_wg[sys], M.sys_wg[sys + 1] - M.sys_wg[sys]);
}

// ------------------------------------------------------------------ SpMV

template <typename T, int FMT, int L, int MODE>
__global__ __launch_bounds__(kBlock) void k_bspmv(const int32_t *__restrict__ ptr, const int32_t *__restrict__ col,
                                                  const T *__restrict__ cval, const int32_t *__restrict__ slot_base,
                                                  const int32_t *__restrict__ jas,
                                                  const B13Desc *__restrict__ desc, const T *__restrict__ bval,
                                                  const T *__restrict__ x, T *__restrict__ y, T *__restrict__ pout,
                                                  const double *__restrict__ b, CgState *st, Map M,
                                                  double *__restrict__ part, int nwg) {
    const int w = blockIdx.x;
    const int sys = M.wg_sys[w];
    if (MODE == kSpmvDot) {
        if (w == M.sys_wg[sys] && threadIdx.x == 0) st[sys].active = 0;
        if (st[sys].status != kRunning) return;
    }
    const int64_t lo = M.wg_lo[w], hi = M.wg_hi[w];
    double d1 = 0.0, d2 = 0.0;
    // the row's epilogue operand (x[row] or b[row]) is loaded before its
    // gathers, not after the y store (which would add a memory round trip)
    auto operand = [&](int64_t row) -> double { return MODE == kSpmvDot ? (double)x[row] : b[row]; };
    auto emit = [&](int64_t row, T sum, double opnd) {
        if (MODE == kSpmvDot) {
            y[row] = sum;
            d1 += opnd * (double)sum;
        } else if (MODE == kSpmvResid) {
            const double bi = opnd, r = bi - (double)sum;
            y[row] = (T)r;
            pout[row] = (T)r;
            d1 += r * r;
            d2 += bi * bi;
        } else {  // kSpmvTrue
            const double r = opnd - (double)sum;
            d1 += r * r;
        }
    };
    if (FMT == MFE_BCRS13) {
        // the 64-row slices overlapping [lo, hi) (system offsets are not
        // slice aligned), L per wavefront per pass (wavefront w takes slices
        // sb + w, sb + w + 4, ...: rows per wavefront 64 L); rows outside
        // [lo, hi) belong to the neighbouring workgroup.  The next pass's
        // column indices are requested before this pass's values and gathers.
        const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6), lane = threadIdx.x & 63;
        const int64_t s_lo = lo >> 6, s_hi = (hi + 63) >> 6;
        constexpr int W = kBlock / 64;
        if constexpr (L == 1 && MFE_BATCH_SCALAR_WALK) {
            // one slice per wavefront: the scalar read-ahead walk of the
            // single-system FP64 product (only the next slice's bounds and
            // descriptor are read ahead, with scalar loads)
            B13Ahead cur, nxt;
            b13_ahead(slot_base, desc, s_lo + wave < s_hi ? s_lo + wave : -1, cur);
            for (int64_t sl = s_lo + wave; sl < s_hi; sl += W) {
                b13_ahead(slot_base, desc, sl + W < s_hi ? sl + W : -1, nxt);
                const int64_t row = sl * 64 + lane;
                if (row >= lo && row < hi) {
                    const double opnd = operand(row);
                    emit(row, b13_row_ahead<T>(cur, jas, bval, sl, lane, x), opnd);
                }
                cur = nxt;
            }
        } else {
        constexpr int SP = W * L;  // slices per pass
        B13Idx cur[L], nxt[L];
        auto fetch = [&](int64_t sb, B13Idx *r) {
#pragma unroll
            for (int j = 0; j < L; ++j) {
                const int64_t sl = sb + j * W + wave, row = sl * 64 + lane;
                r[j].sl.S = 0;
                if (sl >= s_hi) continue;
                r[j].sl = b13_slice(slot_base[sl], slot_base[sl + 1]);
                if (row >= lo && row < hi) b13_cols(jas, desc, sl, lane, r[j]);
            }
        };
        if (s_lo < s_hi) fetch(s_lo, cur);
        for (int64_t sb = s_lo; sb < s_hi; sb += SP) {
#pragma unroll
            for (int j = 0; j < L; ++j) nxt[j].sl.S = 0;
            if (sb + SP < s_hi) fetch(sb + SP, nxt);
#pragma unroll
            for (int j = 0; j < L; ++j) {
                const int64_t sl = sb + j * W + wave, row = sl * 64 + lane;
                if (sl < s_hi && row >= lo && row < hi) {
                    const double opnd = operand(row);
                    const T sum = cur[j].sl.S == 9 ? b13_row9_idx(cur[j].c, bval, cur[j].sl, lane, x)
                                                   : b13_row_generic(jas, bval, cur[j].sl, lane, x);
                    emit(row, sum, opnd);
                }
            }
#pragma unroll
            for (int j = 0; j < L; ++j) cur[j] = nxt[j];
        }
        }
    } else {
        constexpr int R = kBlock / L;  // rows per pass
        const int g = threadIdx.x / L, sub = threadIdx.x % L;
        for (int64_t base = lo; base < hi; base += R) {
            const int64_t row = base + g;
            const double opnd = sub == 0 && row < hi ? operand(row) : 0.0;
            const T sum = csr_row<T, L>(ptr, col, cval, row < hi ? row : -1, sub, x);
            if (sub != 0 || row >= hi) continue;
            emit(row, sum, opnd);
        }
    }
    d1 = block_sum(d1);
    if (MODE == kSpmvResid) d2 = block_sum(d2);
    if (threadIdx.x == 0) {
        part[w] = d1;
        if (MODE == kSpmvResid) part[nwg + w] = d2;
    }
}

// ------------------------------------------------------------------ vector updates

template <typename T>
__global__ __launch_bounds__(kBlock) void k_bupdate_r(T *__restrict__ r, const T *__restrict__ q, CgState *st, Map M,
                                                      const double *__restrict__ pq_part,
                                                      double *__restrict__ rr_part) {
    const int w = blockIdx.x;
    const int sys = M.wg_sys[w];
    CgState &S = st[sys];
    if (S.status != kRunning) return;
    const double pq = sys_sum(pq_part, M, sys);
    const double rho = S.rho;
    const bool first = w == M.sys_wg[sys] && threadIdx.x == 0;
    if (!(pq > 0.0) || !isfinite(pq)) {
        if (first) {
            S.pq = pq;
            S.status = kBreakdown;
        }
        return;
    }
    const double alpha = rho / pq;
    if (first) {
        S.pq = pq;
        S.alpha = alpha;
        S.rho_old = rho;
        S.active = 1;
    }
    const T a = (T)alpha;
    double d = 0.0;
    for (int64_t i = M.wg_lo[w] + threadIdx.x; i < M.wg_hi[w]; i += kBlock) {
        const T ri = r[i] - a * q[i];
        r[i] = ri;
        d += (double)ri * (double)ri;
    }
    d = block_sum(d);
    if (threadIdx.x == 0) rr_part[w] = d;
}

template <typename T>
__global__ __launch_bounds__(kBlock) void k_bupdate_xp(T *__restrict__ x, T *__restrict__ p, const T *__restrict__ r,
                                                       CgState *st, Map M, const double *__restrict__ rr_part) {
    const int w = blockIdx.x;
    const int sys = M.wg_sys[w];
    CgState &S = st[sys];
    if (!S.active) return;
    const double rho_new = sys_sum(rr_part, M, sys);
    const double alpha = S.alpha, beta = rho_new / S.rho_old;
    if (w == M.sys_wg[sys] && threadIdx.x == 0) {
        const int it = S.iters + 1;
        const double res = sqrt(rho_new) / S.bnorm;
        S.iters = it;
        S.rho = rho_new;
        if (S.hist) S.hist[it] = res;
        if (!isfinite(res)) S.status = kBreakdown;
        else if (res <= S.tol) S.status = kConverged;
        else if (it >= S.max_iter) S.status = kCapped;
    }
    const T a = (T)alpha, be = (T)beta;
    for (int64_t i = M.wg_lo[w] + threadIdx.x; i < M.wg_hi[w]; i += kBlock) {
        const T pi = p[i];
        x[i] += a * pi;
        p[i] = r[i] + be * pi;
    }
}

// One workgroup per system.  kind kFinStart: the CG start test from the
// partials (r.r, b.b); kFinTrue: ||b - A x||^2.  With `gate` non-null a
// system whose gate state is not running is marked converged (frozen).
template <int KIND>
__global__ __launch_bounds__(kBlock) void k_bfinalize(const double *__restrict__ part, int nwg, CgState *st, Map M,
                                                      const CgState *gate) {
    const int sys = blockIdx.x;
    const double s1 = sys_sum(part, M, sys);
    double s2 = 0.0;
    if (KIND == kFinStart) s2 = sys_sum(part + nwg, M, sys);
    if (threadIdx.x != 0) return;
    CgState &S = st[sys];
    if (KIND == kFinTrue) {
        S.rr_true = s1;
        return;
    }
    if (gate && gate[sys].status != kRunning) {
        S.status = kConverged;
        S.iters = 0;
        S.active = 0;
        return;
    }
    const double bnorm = sqrt(s2);
    S.bnorm = bnorm;
    S.iters = 0;
    S.active = 0;
    if (bnorm == 0.0) {
        S.rho = 0.0;
        S.zero_x = 1;
        S.status = kConverged;
    } else {
        S.rho = s1;
        const double res = sqrt(s1) / bnorm;
        if (!isfinite(res)) S.status = kBreakdown;
        else if (res <= S.tol) S.status = kConverged;
        else if (S.max_iter <= 0) S.status = kCapped;
        else S.status = kRunning;
    }
}

__global__ __launch_bounds__(kBlock) void k_bzero_if(double *__restrict__ x, const CgState *st, Map M) {
    const int w = blockIdx.x;
    if (!st[M.wg_sys[w]].zero_x) return;
    for (int64_t i = M.wg_lo[w] + threadIdx.x; i < M.wg_hi[w]; i += kBlock) x[i] = 0.0;
}

// mixed precision: r32 = fl32(r / s_sys), p32 = r32, d32 = 0 for running systems; a system whose inner
// state carries scale = s_old > 0 keeps its inner direction instead (as the single-system refinement
// does): p32 = r32 + fl32(s_old / s_sys) (p32 - r32_old)
__global__ __launch_bounds__(kBlock) void k_bmixed_start(const double *__restrict__ r, const CgState *outer,
                                                         const CgState *inner, Map M, float *__restrict__ r32,
                                                         float *__restrict__ p32, float *__restrict__ d32,
                                                         double *__restrict__ part, int nwg) {
    const int w = blockIdx.x;
    const int sys = M.wg_sys[w];
    double acc = 0.0;
    if (outer[sys].status == kRunning) {
        const double s = sqrt(outer[sys].rho);
        const double s_old = inner[sys].scale;
        const float c = s_old > 0.0 ? (float)(s_old / s) : 0.0f;
        for (int64_t i = M.wg_lo[w] + threadIdx.x; i < M.wg_hi[w]; i += kBlock) {
            const float v = (float)(r[i] / s);
            p32[i] = s_old > 0.0 ? v + c * (p32[i] - r32[i]) : v;
            r32[i] = v;
            d32[i] = 0.0f;
            acc += (double)v * (double)v;
        }
    }
    acc = block_sum(acc);
    if (threadIdx.x == 0) {
        part[w] = acc;
        part[nwg + w] = acc;
    }
}

// x += s_sys d for systems refined in this outer step
__global__ __launch_bounds__(kBlock) void k_bmixed_update(double *__restrict__ x, const float *__restrict__ d32,
                                                          const CgState *outer, Map M) {
    const int w = blockIdx.x;
    const int sys = M.wg_sys[w];
    if (outer[sys].status != kRunning) return;
    const double s = sqrt(outer[sys].rho);
    for (int64_t i = M.wg_lo[w] + threadIdx.x; i < M.wg_hi[w]; i += kBlock) x[i] += s * (double)d32[i];
}

}  // namespace
}  // namespace mfe

using namespace mfe;

struct mfe_batch {
    mfe_ctx *ctx = nullptr;
    int nsys = 0;
    std::vector<int> N;         // 3 per system
    std::vector<int64_t> row0;  // nsys + 1
    mfe_problem *P = nullptr;   // block-diagonal matrix and workspace
    Buffer wg_sys, wg_lo, wg_hi, sys_wg, states, part_a, part_b, r32, p32, q32, d32;
    int nwg = 0;
    int map_format = 0;
    Tuning map_tuning;
    Tuning tuned[3];  // per format (index = format flag)
    bool has_tuning[3] = {false, false, false};
    void *pinned = nullptr;  // nsys CgState
    struct GraphEntry {
        int format, lanes, factor, k;
        bool f32;
        const void *x;
        const void *st;
        hipGraphExec_t exec;
    };
    std::vector<GraphEntry> graphs;
    // per system: mean d log(residual) / d iteration of its last FP64 solve
    // and of its last FP32 inner solve (the forecast priors; 0: none yet)
    std::vector<double> rate64, rate32;
};

namespace mfe {
namespace {

Map map_of(const mfe_batch *B) {
    return Map{(const int32_t *)B->wg_sys.ptr, (const int64_t *)B->wg_lo.ptr, (const int64_t *)B->wg_hi.ptr,
               (const int32_t *)B->sys_wg.ptr};
}

template <typename T, int FMT, int L, int MODE>
const void *bspmv_kernel() {
    return (const void *)k_bspmv<T, FMT, L, MODE>;
}

int resident_for(int format, int lanes) {
    const void *k = format == MFE_BCRS13 ? (lanes == 2 ? bspmv_kernel<double, MFE_BCRS13, 2, kSpmvDot>()
                                                       : bspmv_kernel<double, MFE_BCRS13, 1, kSpmvDot>())
                    : lanes == 8        ? bspmv_kernel<double, MFE_CSR, 8, kSpmvDot>()
                    : lanes == 16       ? bspmv_kernel<double, MFE_CSR, 16, kSpmvDot>()
                                        : bspmv_kernel<double, MFE_CSR, 32, kSpmvDot>();
    return resident_per_cu(k);
}

void release_batch_graphs(mfe_batch *B) {
    for (auto &g : B->graphs) (void)hipGraphExecDestroy(g.exec);
    B->graphs.clear();
}

struct MapPlan {
    std::vector<int32_t> wsys, swg;
    std::vector<int64_t> wlo, whi;
};

// Workgroup -> (system, row chunk) map of every system for a grid of about
// `target` groups, in proportion to rows (chunks of whole 64-row slices).
MapPlan plan_full(const mfe_batch *B, long target) {
    MapPlan m;
    m.swg.resize(B->nsys + 1);
    const int64_t mt = B->row0[B->nsys];
    for (int j = 0; j < B->nsys; ++j) {
        const int64_t mj = B->row0[j + 1] - B->row0[j];
        int64_t gj = (int64_t)std::llround((double)target * (double)mj / (double)mt);
        if (gj < 1) gj = 1;
        int64_t chunk = (mj + gj - 1) / gj;
        chunk = (chunk + 63) / 64 * 64;
        m.swg[j] = (int32_t)m.wsys.size();
        for (int64_t a = 0; a < mj; a += chunk) {
            m.wsys.push_back(j);
            m.wlo.push_back(B->row0[j] + a);
            m.whi.push_back(B->row0[j] + std::min(mj, a + chunk));
        }
    }
    m.swg[B->nsys] = (int32_t)m.wsys.size();
    return m;
}

// The same grid of exactly nwg workgroups spread over the systems with
// on[j] set only, in proportion to their rows (at least one each; a
// workgroup may get an empty chunk); the other systems get none, so the
// iteration kernels leave them untouched.  Needs nwg >= the number of
// systems on.
MapPlan plan_active(const mfe_batch *B, int nwg, const std::vector<char> &on) {
    const int ns = B->nsys;
    std::vector<int64_t> g(ns, 0);
    int64_t ma = 0;
    for (int j = 0; j < ns; ++j)
        if (on[j]) ma += B->row0[j + 1] - B->row0[j];
    int64_t used = 0;
    for (int j = 0; j < ns; ++j)
        if (on[j]) {
            g[j] = std::max<int64_t>(1, (int64_t)((double)nwg * (double)(B->row0[j + 1] - B->row0[j]) / (double)ma));
            used += g[j];
        }
    // the rounding left over goes to (or comes from) the systems in order of size
    std::vector<int> order;
    for (int j = 0; j < ns; ++j)
        if (on[j]) order.push_back(j);
    std::sort(order.begin(), order.end(), [&](int a, int b) {
        return B->row0[a + 1] - B->row0[a] > B->row0[b + 1] - B->row0[b];
    });
    for (size_t i = 0; used < nwg; i = (i + 1) % order.size(), ++used) ++g[order[i]];
    for (size_t i = 0; used > nwg; i = (i + 1) % order.size())
        if (g[order[i]] > 1) {
            --g[order[i]];
            --used;
        }
    MapPlan m;
    m.swg.resize(ns + 1);
    for (int j = 0; j < ns; ++j) {
        m.swg[j] = (int32_t)m.wsys.size();
        const int64_t mj = B->row0[j + 1] - B->row0[j];
        if (g[j] == 0) continue;
        int64_t chunk = (mj + g[j] - 1) / g[j];
        chunk = (chunk + 63) / 64 * 64;
        for (int64_t i = 0; i < g[j]; ++i) {
            m.wsys.push_back(j);
            m.wlo.push_back(B->row0[j] + std::min(mj, i * chunk));
            m.whi.push_back(B->row0[j] + std::min(mj, (i + 1) * chunk));
        }
    }
    m.swg[ns] = (int32_t)m.wsys.size();
    return m;
}

// Upload a plan of B->nwg workgroups into the map buffers (graphs keep their grid).
int upload_map(mfe_batch *B, const MapPlan &m) {
    const int nwg = (int)m.wsys.size();
    if (nwg != B->nwg) {
        set_error("internal: a workgroup map of another grid size");
        return MFE_EINVAL;
    }
    hipStream_t s = B->ctx->stream;
    MFE_HIP_TRY(hipMemcpyAsync(B->wg_sys.ptr, m.wsys.data(), nwg * sizeof(int32_t), hipMemcpyHostToDevice, s));
    MFE_HIP_TRY(hipMemcpyAsync(B->wg_lo.ptr, m.wlo.data(), nwg * sizeof(int64_t), hipMemcpyHostToDevice, s));
    MFE_HIP_TRY(hipMemcpyAsync(B->wg_hi.ptr, m.whi.data(), nwg * sizeof(int64_t), hipMemcpyHostToDevice, s));
    MFE_HIP_TRY(hipMemcpyAsync(B->sys_wg.ptr, m.swg.data(), (B->nsys + 1) * sizeof(int32_t), hipMemcpyHostToDevice, s));
    MFE_HIP_TRY(hipStreamSynchronize(s));
    return MFE_OK;
}

long map_target(const mfe_batch *B, int format, const Tuning &t) {
    return (long)B->ctx->num_cu * resident_for(format, t.lanes) * t.factor;
}

// Workgroup -> (system, row chunk) map for a grid of about `target` groups.
int build_map(mfe_batch *B, int format, const Tuning &t) {
    if (B->nwg > 0 && B->map_format == format && B->map_tuning.lanes == t.lanes && B->map_tuning.factor == t.factor)
        return MFE_OK;
    mfe_ctx *ctx = B->ctx;
    const MapPlan plan = plan_full(B, map_target(B, format, t));
    const std::vector<int32_t> &wsys = plan.wsys, &swg = plan.swg;
    const std::vector<int64_t> &wlo = plan.wlo, &whi = plan.whi;
    const int nwg = (int)wsys.size();
    if (nwg > B->nwg || !B->wg_sys.ptr) {
        dev_free(ctx, &B->wg_sys);
        dev_free(ctx, &B->wg_lo);
        dev_free(ctx, &B->wg_hi);
        dev_free(ctx, &B->part_a);
        dev_free(ctx, &B->part_b);
        MFE_TRY(dev_alloc(ctx, &B->wg_sys, nwg * sizeof(int32_t)));
        MFE_TRY(dev_alloc(ctx, &B->wg_lo, nwg * sizeof(int64_t)));
        MFE_TRY(dev_alloc(ctx, &B->wg_hi, nwg * sizeof(int64_t)));
        MFE_TRY(dev_alloc(ctx, &B->part_a, 2 * nwg * sizeof(double)));
        MFE_TRY(dev_alloc(ctx, &B->part_b, 2 * nwg * sizeof(double)));
    }
    hipStream_t s = ctx->stream;
    MFE_HIP_TRY(hipMemcpyAsync(B->wg_sys.ptr, wsys.data(), nwg * sizeof(int32_t), hipMemcpyHostToDevice, s));
    MFE_HIP_TRY(hipMemcpyAsync(B->wg_lo.ptr, wlo.data(), nwg * sizeof(int64_t), hipMemcpyHostToDevice, s));
    MFE_HIP_TRY(hipMemcpyAsync(B->wg_hi.ptr, whi.data(), nwg * sizeof(int64_t), hipMemcpyHostToDevice, s));
    MFE_HIP_TRY(hipMemcpyAsync(B->sys_wg.ptr, swg.data(), (B->nsys + 1) * sizeof(int32_t), hipMemcpyHostToDevice, s));
    MFE_HIP_TRY(hipStreamSynchronize(s));
    B->nwg = nwg;
    B->map_format = format;
    B->map_tuning = t;
    release_batch_graphs(B);  // graphs bake the old map's grid size
    return MFE_OK;
}

template <typename T, int FMT, int L, int MODE>
void launch_b(const mfe_batch *B, const T *x, T *y, T *pout, const double *b, CgState *st, double *part,
              hipStream_t s) {
    const mfe_problem *P = B->P;
    const T *cval = std::is_same<T, double>::value ? (const T *)P->val64.ptr : (const T *)P->val32.ptr;
    const T *bval = std::is_same<T, double>::value ? (const T *)P->bval64.ptr : (const T *)P->bval32.ptr;
    hipLaunchKernelGGL((k_bspmv<T, FMT, L, MODE>), dim3(B->nwg), dim3(kBlock), 0, s, (const int32_t *)P->ptr.ptr,
                       (const int32_t *)P->col.ptr, cval, (const int32_t *)P->slot_base.ptr,
                       (const int32_t *)P->jas.ptr, (const B13Desc *)P->bdesc.ptr, bval, x, y, pout, b, st,
                       map_of(B), part, B->nwg);
}

template <typename T, int MODE>
int bspmv(const mfe_batch *B, int format, const Tuning &t, const void *x, void *y, void *pout, const double *b,
          CgState *st, double *part, hipStream_t s) {
    const T *xx = (const T *)x;
    T *yy = (T *)y, *pp = (T *)pout;
    if (format == MFE_BCRS13 && t.lanes == 2) launch_b<T, MFE_BCRS13, 2, MODE>(B, xx, yy, pp, b, st, part, s);
    else if (format == MFE_BCRS13) launch_b<T, MFE_BCRS13, 1, MODE>(B, xx, yy, pp, b, st, part, s);
    else if (t.lanes == 8) launch_b<T, MFE_CSR, 8, MODE>(B, xx, yy, pp, b, st, part, s);
    else if (t.lanes == 16) launch_b<T, MFE_CSR, 16, MODE>(B, xx, yy, pp, b, st, part, s);
    else launch_b<T, MFE_CSR, 32, MODE>(B, xx, yy, pp, b, st, part, s);
    MFE_HIP_TRY(hipGetLastError());
    return MFE_OK;
}

int bfinalize(const mfe_batch *B, FinalizeKind kind, const double *part, CgState *st, const CgState *gate,
              hipStream_t s) {
    if (kind == kFinStart)
        hipLaunchKernelGGL(k_bfinalize<kFinStart>, dim3(B->nsys), dim3(kBlock), 0, s, part, B->nwg, st, map_of(B),
                           gate);
    else
        hipLaunchKernelGGL(k_bfinalize<kFinTrue>, dim3(B->nsys), dim3(kBlock), 0, s, part, B->nwg, st, map_of(B),
                           gate);
    MFE_HIP_TRY(hipGetLastError());
    return MFE_OK;
}

template <typename T>
int capture_iterations(mfe_batch *B, int format, const Tuning &t, T *x, T *r, T *p, T *q, CgState *st, int k,
                       hipGraphExec_t *out) {
    hipStream_t cs = B->ctx->cap_stream;
    double *pa = (double *)B->part_a.ptr, *pb = (double *)B->part_b.ptr;
    MFE_HIP_TRY(hipStreamBeginCapture(cs, hipStreamCaptureModeThreadLocal));
    int rc = MFE_OK;
    const Map M = map_of(B);
    for (int i = 0; i < k && rc == MFE_OK; ++i) {
        rc = bspmv<T, kSpmvDot>(B, format, t, p, q, nullptr, nullptr, st, pa, cs);
        if (rc == MFE_OK) {
            hipLaunchKernelGGL(k_bupdate_r<T>, dim3(B->nwg), dim3(kBlock), 0, cs, r, (const T *)q, st, M,
                               (const double *)pa, pb);
            hipLaunchKernelGGL(k_bupdate_xp<T>, dim3(B->nwg), dim3(kBlock), 0, cs, x, p, (const T *)r, st, M,
                               (const double *)pb);
            if (hipGetLastError() != hipSuccess) rc = MFE_EHIP;
        }
    }
    hipGraph_t g = nullptr;
    const hipError_t e = hipStreamEndCapture(cs, &g);
    if (rc != MFE_OK || e != hipSuccess) {
        if (g) (void)hipGraphDestroy(g);
        set_error("batched iteration capture failed");
        return rc != MFE_OK ? rc : MFE_EHIP;
    }
    const hipError_t e2 = hipGraphInstantiate(out, g, nullptr, nullptr, 0);
    (void)hipGraphDestroy(g);
    if (e2 != hipSuccess) {
        set_error(std::string("hipGraphInstantiate failed: ") + hipGetErrorString(e2));
        return MFE_EHIP;
    }
    return MFE_OK;
}

constexpr int kMaxBatchGraphs = 32;

template <typename T>
int graph_for_batch(mfe_batch *B, int format, const Tuning &t, bool f32, T *x, T *r, T *p, T *q, CgState *st, int k,
                    hipGraphExec_t *out) {
    for (auto &g : B->graphs)
        if (g.format == format && g.lanes == t.lanes && g.factor == t.factor && g.k == k && g.f32 == f32 &&
            g.x == x && g.st == st) {
            *out = g.exec;
            return MFE_OK;
        }
    hipGraphExec_t ex = nullptr;
    MFE_TRY(capture_iterations<T>(B, format, t, x, r, p, q, st, k, &ex));
    // bounded cache, as for single problems: drop the oldest graph once no
    // work of the context uses it
    if (B->graphs.size() >= (size_t)kMaxBatchGraphs) {
        const hipError_t e = hipStreamSynchronize(B->ctx->stream);
        if (e != hipSuccess) {
            (void)hipGraphExecDestroy(ex);
            set_error(std::string("hipStreamSynchronize failed: ") + hipGetErrorString(e));
            return MFE_EHIP;
        }
        (void)hipGraphExecDestroy(B->graphs.front().exec);
        B->graphs.erase(B->graphs.begin());
    }
    B->graphs.push_back({format, t.lanes, t.factor, k, f32, x, st, ex});
    *out = ex;
    return MFE_OK;
}

// The iteration graphs of a batched solve: k iterations, and kt for the end
// of the solve (tail = nullptr when k <= kTailIters).
struct BatchGraphs {
    hipGraphExec_t exec = nullptr, tail = nullptr;
    int k = 0, kt = 0;
};

template <typename T>
int batch_graphs(mfe_batch *B, int format, const Tuning &t, bool f32, T *x, T *r, T *p, T *q, CgState *st,
                 int max_iter, BatchGraphs *G) {
    G->k = std::min(kGraphIters, max_iter);
    MFE_TRY(graph_for_batch<T>(B, format, t, f32, x, r, p, q, st, G->k, &G->exec));
    G->tail = nullptr;
    G->kt = 0;
    if (MFE_CG_TAIL && G->k > kTailIters) {
        G->kt = kTailIters;
        MFE_TRY(graph_for_batch<T>(B, format, t, f32, x, r, p, q, st, G->kt, &G->tail));
    }
    return MFE_OK;
}

// Copy all system states to the host.
int read_states(mfe_batch *B, const CgState *st, std::vector<CgState> &out) {
    hipStream_t s = B->ctx->stream;
    MFE_HIP_TRY(hipMemcpyAsync(B->pinned, st, B->nsys * sizeof(CgState), hipMemcpyDeviceToHost, s));
    MFE_HIP_TRY(hipStreamSynchronize(s));
    const CgState *h = (const CgState *)B->pinned;
    out.assign(h, h + B->nsys);
    return MFE_OK;
}

int set_states(mfe_batch *B, CgState *st, double tol, int max_iter, const std::vector<double> *tols = nullptr,
               const std::vector<double> *scales = nullptr) {
    std::vector<CgState> h(B->nsys);
    for (int j = 0; j < B->nsys; ++j) {
        CgState &x = h[j];
        x = CgState{};
        x.tol = tols ? (*tols)[j] : tol;
        x.max_iter = max_iter;
        x.status = kRunning;
        x.scale = scales ? (*scales)[j] : 0.0;
    }
    CgState *pin = (CgState *)B->pinned;
    std::copy(h.begin(), h.end(), pin);
    MFE_HIP_TRY(hipMemcpyAsync(st, pin, B->nsys * sizeof(CgState), hipMemcpyHostToDevice, B->ctx->stream));
    MFE_HIP_TRY(hipStreamSynchronize(B->ctx->stream));
    return MFE_OK;
}

bool any_running(const std::vector<CgState> &v) {
    for (const auto &s : v)
        if (s.status == kRunning) return true;
    return false;
}

#ifndef MFE_BATCH_REMAP
#define MFE_BATCH_REMAP 1  // spread the grid over the running systems only once their rows fall below 60 %
#endif

// Replay the iteration graphs until no system runs.  fin holds the start
// states on entry and the final ones on return.  Each system's residual is
// forecast as in the single-system driver (prior: rates, updated here); the
// tail graph is launched once every running system is forecast to stop
// within one long graph, so that few frozen iterations follow the last
// system's end.  Once the running systems hold at most 60 % of the rows the
// grid is spread over, the same grid is spread over them alone (the graphs
// keep their launch shape and read the map at replay), so the systems that
// remain take the whole GPU; this is decided at multiples of kGraphIters
// iterations only, and the full map is restored at the end.
int run_batch(mfe_batch *B, const BatchGraphs &G, const CgState *st, int max_iter, std::vector<double> &rates,
              std::vector<CgState> &fin) {
    hipStream_t s = B->ctx->stream;
    const int ns = B->nsys;
    if ((int)rates.size() != ns) rates.assign(ns, 0.0);
    std::vector<Forecast> fc(ns);
    std::vector<double> res0(ns, 0.0);
    double rem = 0.0;  // the largest forecast over the running systems
    for (int j = 0; j < ns; ++j) {
        fc[j].slope = rates[j];
        res0[j] = stop_residual(fin[j], 0);
        if (fin[j].status == kRunning) rem = std::max(rem, fc[j].observe(0, res0[j], fin[j].tol));
    }
    const long limit = (long)max_iter + 2L * G.k;  // iterations; the device cap ends the loop first
    int64_t spread = B->row0[B->nsys];  // rows the current map spreads the grid over
    bool partial = false;
    int rc = MFE_OK;
    for (long launched = 0;;) {
        if (launched > limit) {
            set_error("batched CG still running after the iteration cap");
            rc = MFE_EHIP;
            break;
        }
        const bool tail = G.tail && std::min(rem, (double)(max_iter - launched)) <= (double)G.k;
        if (hipGraphLaunch(tail ? G.tail : G.exec, s) != hipSuccess) {
            set_error("hipGraphLaunch failed");
            rc = MFE_EHIP;
            break;
        }
        launched += tail ? G.kt : G.k;
        rc = read_states(B, st, fin);
        if (rc != MFE_OK || !any_running(fin)) break;
        rem = 0.0;
        for (int j = 0; j < ns; ++j)
            if (fin[j].status == kRunning)
                rem = std::max(rem, fc[j].observe(fin[j].iters, stop_residual(fin[j], 0), fin[j].tol));
        // the map decides each system's reduction order: it changes only at
        // multiples of kGraphIters iterations, so that results do not depend
        // on the graph lengths the forecast picks
        if (MFE_BATCH_REMAP && launched % kGraphIters == 0) {
            std::vector<char> on(B->nsys, 0);
            int64_t active = 0, nact = 0;
            for (int j = 0; j < B->nsys; ++j)
                if (fin[j].status == kRunning) {
                    on[j] = 1;
                    active += B->row0[j + 1] - B->row0[j];
                    ++nact;
                }
            if (active * 10 <= spread * 6 && nact <= B->nwg) {
                rc = upload_map(B, plan_active(B, B->nwg, on));
                if (rc != MFE_OK) break;
                spread = active;
                partial = true;
            }
        }
    }
    if (partial) {
        const int r2 = upload_map(B, plan_full(B, map_target(B, B->map_format, B->map_tuning)));
        if (rc == MFE_OK) rc = r2;
    }
    if (rc == MFE_OK)
        for (int j = 0; j < ns; ++j) {
            const double res = stop_residual(fin[j], 0);
            if (fin[j].iters > 0 && res0[j] > 0.0 && res > 0.0 && std::isfinite(res) && std::isfinite(res0[j])) {
                const double r = (std::log(res) - std::log(res0[j])) / fin[j].iters;
                if (r < 0.0) rates[j] = r;
            }
        }
    return rc;
}

// FP64 batched CG on all systems from x.  out_states: final states.
int batch_cg_fp64(mfe_batch *B, int format, const Tuning &t, double *x, double tol, int max_iter,
                  std::vector<CgState> &fin, std::vector<double> &rel_true) {
    mfe_problem *P = B->P;
    hipStream_t s = B->ctx->stream;
    CgState *st = (CgState *)B->states.ptr;
    double *pa = (double *)B->part_a.ptr;
    MFE_TRY(set_states(B, st, tol, max_iter));
    MFE_TRY(bspmv<double, kSpmvResid>(B, format, t, x, P->r.ptr, P->p.ptr, (const double *)P->b.ptr, st, pa, s));
    MFE_TRY(bfinalize(B, kFinStart, pa, st, nullptr, s));
    hipLaunchKernelGGL(k_bzero_if, dim3(B->nwg), dim3(kBlock), 0, s, x, (const CgState *)st, map_of(B));
    MFE_HIP_TRY(hipGetLastError());
    MFE_TRY(read_states(B, st, fin));
    if (any_running(fin)) {
        BatchGraphs G;
        MFE_TRY(batch_graphs<double>(B, format, t, false, x, (double *)P->r.ptr, (double *)P->p.ptr,
                                     (double *)P->q.ptr, st, max_iter, &G));
        MFE_TRY(run_batch(B, G, st, max_iter, B->rate64, fin));
    }
    MFE_TRY(bspmv<double, kSpmvTrue>(B, format, t, x, nullptr, nullptr, (const double *)P->b.ptr, st, pa, s));
    MFE_TRY(bfinalize(B, kFinTrue, pa, st, nullptr, s));
    std::vector<CgState> tr;
    MFE_TRY(read_states(B, st, tr));
    rel_true.resize(B->nsys);
    for (int j = 0; j < B->nsys; ++j)
        rel_true[j] = fin[j].bnorm > 0 ? std::sqrt(tr[j].rr_true) / fin[j].bnorm : 0.0;
    return MFE_OK;
}

int ensure_batch_ws(mfe_batch *B, bool mixed) {
    MFE_TRY(ensure_workspace(B->P));
    mfe_ctx *ctx = B->ctx;
    if (!B->states.ptr) MFE_TRY(dev_alloc(ctx, &B->states, 2 * B->nsys * sizeof(CgState)));
    if (mixed) {
        const size_t fb = (size_t)B->P->m * sizeof(float);
        if (!B->r32.ptr) MFE_TRY(dev_alloc(ctx, &B->r32, fb));
        if (!B->p32.ptr) MFE_TRY(dev_alloc(ctx, &B->p32, fb));
        if (!B->q32.ptr) MFE_TRY(dev_alloc(ctx, &B->q32, fb));
        if (!B->d32.ptr) MFE_TRY(dev_alloc(ctx, &B->d32, fb));
    }
    return MFE_OK;
}

int status_of(const CgState &s) {
    if (s.status == kCapped) return MFE_NOT_CONVERGED;
    if (s.status == kBreakdown) return MFE_EBREAKDOWN;
    return MFE_OK;
}

// Time the batched SpMV kernel under tuning t (ms per launch).
int time_spmv(mfe_batch *B, int format, const Tuning &t, double *ms) {
    MFE_TRY(build_map(B, format, t));
    MFE_TRY(ensure_batch_ws(B, false));
    mfe_problem *P = B->P;
    hipStream_t s = B->ctx->stream;
    CgState *st = (CgState *)B->states.ptr;
    MFE_TRY(set_states(B, st, 0.0, 1));  // running states so the Dot kernel works
    hipEvent_t e0, e1;
    MFE_HIP_TRY(hipEventCreate(&e0));
    MFE_HIP_TRY(hipEventCreate(&e1));
    const int reps = 5;
    int rc = bspmv<double, kSpmvDot>(B, format, t, P->b.ptr, P->q.ptr, nullptr, nullptr, st,
                                     (double *)B->part_a.ptr, s);  // warm-up
    if (rc == MFE_OK && hipEventRecord(e0, s) != hipSuccess) rc = MFE_EHIP;
    for (int i = 0; i < reps && rc == MFE_OK; ++i)
        rc = bspmv<double, kSpmvDot>(B, format, t, P->b.ptr, P->q.ptr, nullptr, nullptr, st, (double *)B->part_a.ptr,
                                     s);
    float f = 0.f;
    if (rc == MFE_OK && (hipEventRecord(e1, s) != hipSuccess || hipEventSynchronize(e1) != hipSuccess ||
                         hipEventElapsedTime(&f, e0, e1) != hipSuccess))
        rc = MFE_EHIP;
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    if (rc != MFE_OK) {
        if (rc == MFE_EHIP) set_error("autotune timing failed");
        return rc;
    }
    *ms = f / reps;
    return MFE_OK;
}

int tuning_for(mfe_batch *B, int format, Tuning *t) {
    if (B->has_tuning[format]) {
        *t = B->tuned[format];
        return MFE_OK;
    }
    *t = Tuning{};
    return MFE_OK;
}

}  // namespace
}  // namespace mfe

namespace {

// A batch object with the block-diagonal CRS storage allocated (rows row0,
// entries nnz0 per system), not yet filled.
int alloc_batch(mfe_ctx *ctx, int nsys, const std::vector<int64_t> &row0, const std::vector<int64_t> &nnz0,
                int formats, int precisions, mfe_batch **out) {
    if (nnz0[nsys] >= ((int64_t)1 << 31) - 1 || row0[nsys] >= ((int64_t)1 << 31) - 1) {
        set_error("batch too large for 32-bit row pointers");
        return MFE_EUNSUPPORTED;
    }
    if (hipSetDevice(ctx->device) != hipSuccess) {
        set_error("hipSetDevice failed");
        return MFE_EHIP;
    }
    mfe_batch *B = new (std::nothrow) mfe_batch();
    mfe_problem *P = new (std::nothrow) mfe_problem();
    if (!B || !P) {
        delete B;
        delete P;
        set_error("host allocation failed");
        return MFE_ENOMEM;
    }
    B->ctx = ctx;
    B->nsys = nsys;
    B->N.assign(3 * (size_t)nsys, 0);
    B->row0 = row0;
    B->P = P;
    P->ctx = ctx;
    P->m = row0[nsys];
    P->nnz = nnz0[nsys];
    P->formats = formats | MFE_CSR;
    P->precisions = precisions | MFE_F64;
    int rc = dev_alloc(ctx, &P->ptr, (size_t)(P->m + 1) * sizeof(int32_t));
    if (rc == MFE_OK) rc = dev_alloc(ctx, &P->col, (size_t)P->nnz * sizeof(int32_t));
    if (rc == MFE_OK) rc = dev_alloc(ctx, &P->val64, (size_t)P->nnz * sizeof(double));
    if (rc == MFE_OK) rc = dev_alloc(ctx, &P->b, (size_t)P->m * sizeof(double));
    if (rc == MFE_OK) rc = dev_alloc(ctx, &B->sys_wg, (nsys + 1) * sizeof(int32_t));
    if (rc != MFE_OK) {
        mfe_batch_destroy(B);
        return rc;
    }
    *out = B;
    return MFE_OK;
}

// Derived formats of the filled CRS and the pinned state slots; registers the batch.
int finish_batch(mfe_batch *B, mfe_batch **out) {
    int rc = finish_problem(B->P);
    if (rc == MFE_OK && hipHostMalloc(&B->pinned, B->nsys * sizeof(CgState), hipHostMallocDefault) != hipSuccess) {
        set_error("hipHostMalloc failed");
        rc = MFE_EHIP;
    }
    if (rc != MFE_OK) {
        mfe_batch_destroy(B);
        return rc;
    }
    B->ctx->batches.push_back(B);
    *out = B;
    return MFE_OK;
}

// dst[i] = src[i] + add (column indices and row pointers moved into the block-diagonal matrix)
__global__ __launch_bounds__(256) void k_shift_copy(int64_t n, const int32_t *__restrict__ src, int32_t add,
                                                    int32_t *__restrict__ dst) {
    for (int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x; i < n; i += (int64_t)gridDim.x * 256)
        dst[i] = src[i] + add;
}

int shift_copy(hipStream_t s, int64_t n, const int32_t *src, int64_t add, int32_t *dst) {
    if (n <= 0) return MFE_OK;
    const int grid = (int)std::min<int64_t>(4096, (n + 255) / 256);
    hipLaunchKernelGGL(k_shift_copy, dim3(grid), dim3(256), 0, s, n, src, (int32_t)add, dst);
    MFE_HIP_TRY(hipGetLastError());
    return MFE_OK;
}

}  // namespace

extern "C" {

int mfe_batch_create(mfe_ctx *ctx, int nsys, const int32_t *sizes, const double *face_vals, int formats,
                     int precisions, mfe_batch **out) {
    clear_error();
    if (!ctx || !out || !sizes || nsys < 1) {
        set_error("ctx, sizes and out must be non-NULL and nsys >= 1");
        return MFE_EINVAL;
    }
    *out = nullptr;
    if ((formats & ~(MFE_CSR | MFE_BCRS13)) || (precisions & ~(MFE_F64 | MFE_F32))) {
        set_error("unknown format or precision flag");
        return MFE_EINVAL;
    }
    std::vector<int64_t> row0(nsys + 1, 0), nnz0(nsys + 1, 0);
    for (int j = 0; j < nsys; ++j) {
        const int Nx = sizes[3 * j], Ny = sizes[3 * j + 1], Nz = sizes[3 * j + 2];
        if (Nx < 1 || Ny < 1 || Nz < 1) {
            set_error("every mesh needs Nx, Ny, Nz >= 1");
            return MFE_EINVAL;
        }
        row0[j + 1] = row0[j] + (int64_t)(Nx + 1) * (Ny + 1) * (Nz + 1);
        nnz0[j + 1] = nnz0[j] + (3 * (int64_t)Nx + 1) * (3 * (int64_t)Ny + 1) * (3 * (int64_t)Nz + 1);
    }
    mfe_batch *B = nullptr;
    MFE_TRY(alloc_batch(ctx, nsys, row0, nnz0, formats, precisions, &B));
    B->N.assign(sizes, sizes + 3 * nsys);
    mfe_problem *P = B->P;
    int rc = MFE_OK;
    for (int j = 0; j < nsys && rc == MFE_OK; ++j)
        rc = launch_assemble_into(ctx->stream, sizes[3 * j], sizes[3 * j + 1], sizes[3 * j + 2],
                                  face_vals ? face_vals + 6 * j : nullptr, nullptr, row0[j], nnz0[j],
                                  (int32_t *)P->ptr.ptr, (int32_t *)P->col.ptr, (double *)P->val64.ptr,
                                  (double *)P->b.ptr, false);
    if (rc != MFE_OK) {
        mfe_batch_destroy(B);
        return rc;
    }
    return finish_batch(B, out);
}

int mfe_batch_from_problems(mfe_ctx *ctx, int nsys, mfe_problem *const *sys, int formats, int precisions,
                            mfe_batch **out) {
    clear_error();
    if (!ctx || !out || !sys || nsys < 1) {
        set_error("ctx, sys and out must be non-NULL and nsys >= 1");
        return MFE_EINVAL;
    }
    *out = nullptr;
    if ((formats & ~(MFE_CSR | MFE_BCRS13)) || (precisions & ~(MFE_F64 | MFE_F32))) {
        set_error("unknown format or precision flag");
        return MFE_EINVAL;
    }
    std::vector<int64_t> row0(nsys + 1, 0), nnz0(nsys + 1, 0);
    for (int j = 0; j < nsys; ++j) {
        if (!sys[j] || sys[j]->ctx != ctx) {
            set_error("every system must be a problem of this context");
            return MFE_EINVAL;
        }
        row0[j + 1] = row0[j] + sys[j]->m;
        nnz0[j + 1] = nnz0[j] + sys[j]->nnz;
    }
    mfe_batch *B = nullptr;
    MFE_TRY(alloc_batch(ctx, nsys, row0, nnz0, formats, precisions, &B));
    mfe_problem *P = B->P;
    hipStream_t s = ctx->stream;
    int rc = MFE_OK;
    for (int j = 0; j < nsys && rc == MFE_OK; ++j) {
        const mfe_problem *Q = sys[j];
        if (Q->is_mesh) {
            B->N[3 * j] = Q->Nx;
            B->N[3 * j + 1] = Q->Ny;
            B->N[3 * j + 2] = Q->Nz;
        }
        // rows 0..m-1 of system j; ptr[m] of the last system closes the matrix
        rc = shift_copy(s, Q->m + (j == nsys - 1 ? 1 : 0), (const int32_t *)Q->ptr.ptr, nnz0[j],
                        (int32_t *)P->ptr.ptr + row0[j]);
        if (rc == MFE_OK) rc = shift_copy(s, Q->nnz, (const int32_t *)Q->col.ptr, row0[j], (int32_t *)P->col.ptr + nnz0[j]);
        if (rc == MFE_OK &&
            (hipMemcpyAsync((double *)P->val64.ptr + nnz0[j], Q->val64.ptr, Q->nnz * sizeof(double),
                            hipMemcpyDeviceToDevice, s) != hipSuccess ||
             hipMemcpyAsync((double *)P->b.ptr + row0[j], Q->b.ptr, Q->m * sizeof(double), hipMemcpyDeviceToDevice,
                            s) != hipSuccess)) {
            set_error("copy of a system's CRS arrays failed");
            rc = MFE_EHIP;
        }
    }
    if (rc != MFE_OK) {
        mfe_batch_destroy(B);
        return rc;
    }
    return finish_batch(B, out);
}

int mfe_batch_destroy(mfe_batch *B) {
    if (!B) return MFE_OK;
    mfe_ctx *ctx = B->ctx;
    (void)hipSetDevice(ctx->device);
    (void)hipStreamSynchronize(ctx->stream);
    release_batch_graphs(B);
    Buffer *bufs[] = {&B->wg_sys, &B->wg_lo, &B->wg_hi, &B->sys_wg, &B->states, &B->part_a, &B->part_b,
                      &B->r32,    &B->p32,   &B->q32,   &B->d32};
    for (Buffer *b : bufs) dev_free(ctx, b);
    if (B->P) {
        free_problem_storage(B->P);
        delete B->P;
    }
    if (B->pinned) (void)hipHostFree(B->pinned);
    unregister(ctx->batches, B);
    delete B;
    return MFE_OK;
}

int mfe_batch_info(const mfe_batch *B, int64_t *m_total, int64_t *nnz_total, int64_t *row_offsets) {
    clear_error();
    if (!B) {
        set_error("batch is NULL");
        return MFE_EINVAL;
    }
    if (m_total) *m_total = B->P->m;
    if (nnz_total) *nnz_total = B->P->nnz;
    if (row_offsets)
        for (int j = 0; j <= B->nsys; ++j) row_offsets[j] = B->row0[j];
    return MFE_OK;
}

int mfe_batch_bcrs13_layout(const mfe_batch *B, int64_t *slices, int64_t *slots, int64_t *compressed_slices,
                            int64_t *compressed_blocks) {
    clear_error();
    if (!B) {
        set_error("batch is NULL");
        return MFE_EINVAL;
    }
    return mfe_problem_bcrs13_layout(B->P, slices, slots, compressed_slices, compressed_blocks);
}

int mfe_batch_export_csr(const mfe_batch *B, int32_t *ptr_dev, int32_t *col_dev, double *val_dev, double *b_dev) {
    clear_error();
    if (!B) {
        set_error("batch is NULL");
        return MFE_EINVAL;
    }
    return mfe_problem_export_csr(B->P, ptr_dev, col_dev, val_dev, b_dev);
}

int mfe_batch_set_bc(mfe_batch *B, const double *face_vals, const double *node_g_dev) {
    clear_error();
    if (!B) {
        set_error("batch is NULL");
        return MFE_EINVAL;
    }
    for (int j = 0; j < B->nsys; ++j)
        if (B->N[3 * j] < 1) {
            set_error("boundary data can only be re-imposed when every system is a mesh");
            return MFE_EINVAL;
        }
    if (hipSetDevice(B->ctx->device) != hipSuccess) return MFE_EHIP;
    mfe_problem *P = B->P;
    for (int j = 0; j < B->nsys; ++j)
        MFE_TRY(launch_assemble_into(B->ctx->stream, B->N[3 * j], B->N[3 * j + 1], B->N[3 * j + 2],
                                     face_vals ? face_vals + 6 * j : nullptr,
                                     node_g_dev ? node_g_dev + B->row0[j] : nullptr, B->row0[j], 0,
                                     (int32_t *)P->ptr.ptr, (int32_t *)P->col.ptr, (double *)P->val64.ptr,
                                     (double *)P->b.ptr, true));
    return MFE_OK;
}

int mfe_batch_autotune(mfe_batch *B, int format, int *lanes_out, int *factor_out) {
    clear_error();
    if (!B || (format != MFE_CSR && format != MFE_BCRS13) || !(B->P->formats & format)) {
        set_error("batch must be non-NULL and the format built");
        return MFE_EINVAL;
    }
    if (hipSetDevice(B->ctx->device) != hipSuccess) return MFE_EHIP;
    // CRS: lanes per row 8 / 16 / 32 (rows per wavefront 8 / 4 / 2);
    // 1x3 BCRS: one lane per row, slices per wavefront and pass 1 / 2 (rows
    // per wavefront 64 / 128); both with grids of 1, 2, 4 x resident
    static const int lanes_c[3] = {8, 16, 32};
    static const int slices_b[2] = {1, 2};
    static const int factors[3] = {1, 2, 4};
    Tuning best{};
    double best_ms = 1e300;
    const int nl = format == MFE_BCRS13 ? 2 : 3;
    for (int li = 0; li < nl; ++li) {
        for (int fi = 0; fi < 3; ++fi) {
            Tuning t;
            t.lanes = format == MFE_BCRS13 ? slices_b[li] : lanes_c[li];
            t.factor = factors[fi];
            double ms = 0;
            MFE_TRY(time_spmv(B, format, t, &ms));
            if (ms < best_ms) {
                best_ms = ms;
                best = t;
            }
        }
    }
    B->tuned[format] = best;
    B->has_tuning[format] = true;
    if (lanes_out) *lanes_out = best.lanes;
    if (factor_out) *factor_out = best.factor;
    return MFE_OK;
}

int mfe_batch_cg(mfe_batch *B, int format, double *x_dev, double tol, int max_iter, mfe_cg_stats *stats) {
    clear_error();
    if (!B || !x_dev || !(tol >= 0.0) || max_iter < 0 || (format != MFE_CSR && format != MFE_BCRS13) ||
        !(B->P->formats & format)) {
        set_error("need batch, x, tol >= 0, max_iter >= 0 and a built format");
        return MFE_EINVAL;
    }
    if (hipSetDevice(B->ctx->device) != hipSuccess) return MFE_EHIP;
    const auto t0 = std::chrono::steady_clock::now();
    Tuning t;
    MFE_TRY(tuning_for(B, format, &t));
    MFE_TRY(build_map(B, format, t));
    MFE_TRY(ensure_batch_ws(B, false));
    std::vector<CgState> fin;
    std::vector<double> rel;
    MFE_TRY(batch_cg_fp64(B, format, t, x_dev, tol, max_iter, fin, rel));
    const double secs = std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
    int rc = MFE_OK;
    for (int j = 0; j < B->nsys; ++j) {
        const int sj = status_of(fin[j]);
        if (sj == MFE_EBREAKDOWN || (sj == MFE_NOT_CONVERGED && rc == MFE_OK)) rc = sj;
        if (stats) {
            stats[j].status = sj;
            stats[j].iterations = fin[j].iters;
            stats[j].outer = 0;
            stats[j].spmv_count = fin[j].iters + 2;
            stats[j].rel_res_recurrence = fin[j].bnorm > 0 ? std::sqrt(fin[j].rho) / fin[j].bnorm : 0.0;
            stats[j].rel_res_true = rel[j];
            stats[j].seconds = secs;
            stats[j].guess_rejected = 0;
            stats[j].reserved_ = 0;
        }
    }
    return rc;
}

int mfe_batch_cg_mixed(mfe_batch *B, int format, double *x_dev, double tol, double inner_tol, int max_outer,
                       int max_inner, mfe_cg_stats *stats) {
    return mfe_batch_cg_mixed_ex(B, format, x_dev, tol, inner_tol, max_outer, max_inner, 0, stats);
}

int mfe_batch_cg_mixed_ex(mfe_batch *B, int format, double *x_dev, double tol, double inner_tol, int max_outer,
                          int max_inner, int flags, mfe_cg_stats *stats) {
    clear_error();
    if (!B || !x_dev || !(tol >= 0.0) || !(inner_tol > 0.0 && inner_tol < 1.0) || max_outer < 1 || max_inner < 1 ||
        (format != MFE_CSR && format != MFE_BCRS13) || !(B->P->formats & format)) {
        set_error("need batch, x, tol >= 0, 0 < inner_tol < 1, max_outer, max_inner >= 1 and a built format");
        return MFE_EINVAL;
    }
    if (flags & ~MFE_MIXED_KEEP_DIRECTION) {
        set_error("flags: only MFE_MIXED_KEEP_DIRECTION applies to a batch");
        return MFE_EINVAL;
    }
    const bool keep = (flags & MFE_MIXED_KEEP_DIRECTION) != 0;
    if (!(B->P->precisions & MFE_F32)) {
        set_error("FP32 values were not built for this batch");
        return MFE_EUNSUPPORTED;
    }
    if (hipSetDevice(B->ctx->device) != hipSuccess) return MFE_EHIP;
    const auto t0 = std::chrono::steady_clock::now();
    Tuning t;
    MFE_TRY(tuning_for(B, format, &t));
    MFE_TRY(build_map(B, format, t));
    MFE_TRY(ensure_batch_ws(B, true));
    mfe_problem *P = B->P;
    hipStream_t s = B->ctx->stream;
    const int ns = B->nsys;
    CgState *outer = (CgState *)B->states.ptr, *inner = outer + ns;
    double *pa = (double *)B->part_a.ptr;
    const Map M = map_of(B);
    std::vector<int> outer_steps(ns, 0), inner_its(ns, 0);
    std::vector<CgState> o, in;
    std::vector<double> bnorm(ns), prev(ns), scales(ns, 0.0);
    auto outer_residual = [&]() -> int {
        MFE_TRY(set_states(B, outer, tol, 1));
        MFE_TRY(bspmv<double, kSpmvResid>(B, format, t, x_dev, P->r.ptr, P->p.ptr, (const double *)P->b.ptr, outer,
                                          pa, s));
        MFE_TRY(bfinalize(B, kFinStart, pa, outer, nullptr, s));
        return read_states(B, outer, o);
    };
    MFE_TRY(outer_residual());
    hipLaunchKernelGGL(k_bzero_if, dim3(B->nwg), dim3(kBlock), 0, s, x_dev, (const CgState *)outer, M);
    for (int j = 0; j < ns; ++j) {
        bnorm[j] = o[j].bnorm;
        prev[j] = std::sqrt(o[j].rho);
    }
    bool fallback = false;
    int step = 0;
    while (any_running(o)) {
        if (step >= max_outer) break;
        // per-system inner tolerance: no tighter than its outer target needs
        std::vector<double> eff(ns, inner_tol);
        for (int j = 0; j < ns; ++j)
            if (o[j].status == kRunning && prev[j] > 0)
                eff[j] = std::min(0.5, std::max(inner_tol, 0.5 * tol * bnorm[j] / prev[j]));
        MFE_TRY(set_states(B, inner, inner_tol, max_inner, &eff, &scales));
        hipLaunchKernelGGL(k_bmixed_start, dim3(B->nwg), dim3(kBlock), 0, s, (const double *)P->r.ptr,
                           (const CgState *)outer, (const CgState *)inner, M, (float *)B->r32.ptr,
                           (float *)B->p32.ptr, (float *)B->d32.ptr, pa, B->nwg);
        MFE_HIP_TRY(hipGetLastError());
        MFE_TRY(bfinalize(B, kFinStart, pa, inner, outer, s));
        BatchGraphs G;
        MFE_TRY(batch_graphs<float>(B, format, t, true, (float *)B->d32.ptr, (float *)B->r32.ptr,
                                    (float *)B->p32.ptr, (float *)B->q32.ptr, inner, max_inner, &G));
        MFE_TRY(read_states(B, inner, in));  // the start states seed the forecast
        if (any_running(in)) MFE_TRY(run_batch(B, G, inner, max_inner, B->rate32, in));
        bool breakdown = false;
        for (int j = 0; j < ns; ++j) {
            // the next step keeps the direction of an inner solve that met its tolerance (scale = its s)
            scales[j] = keep && o[j].status == kRunning && in[j].status == kConverged ? prev[j] : 0.0;
            if (o[j].status == kRunning) {
                inner_its[j] += in[j].iters;
                outer_steps[j] += 1;
                breakdown = breakdown || in[j].status == kBreakdown;
            }
        }
        hipLaunchKernelGGL(k_bmixed_update, dim3(B->nwg), dim3(kBlock), 0, s, x_dev, (const float *)B->d32.ptr,
                           (const CgState *)outer, M);
        MFE_HIP_TRY(hipGetLastError());
        ++step;
        std::vector<CgState> before = o;
        MFE_TRY(outer_residual());
        bool stagnated = false;
        for (int j = 0; j < ns; ++j)
            if (before[j].status == kRunning) {
                const double cur = std::sqrt(o[j].rho);
                if (o[j].status == kRunning && !(cur <= 0.5 * prev[j])) stagnated = true;
                prev[j] = cur;
            }
        if (breakdown || stagnated) {
            fallback = true;
            break;
        }
    }
    std::vector<double> rel(ns);
    for (int j = 0; j < ns; ++j) rel[j] = bnorm[j] > 0 ? std::sqrt(o[j].rho) / bnorm[j] : 0.0;
    std::vector<int> st_code(ns, MFE_OK), fb_its(ns, 0);
    for (int j = 0; j < ns; ++j)
        if (o[j].status == kRunning) st_code[j] = MFE_NOT_CONVERGED;
    if (fallback) {
        std::vector<CgState> fin;
        MFE_TRY(batch_cg_fp64(B, format, t, x_dev, tol, max_inner * max_outer, fin, rel));
        for (int j = 0; j < ns; ++j) {
            st_code[j] = status_of(fin[j]);
            fb_its[j] = fin[j].iters;
        }
    }
    const double secs = std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
    int rc = MFE_OK;
    for (int j = 0; j < ns; ++j) {
        if (st_code[j] == MFE_EBREAKDOWN || (st_code[j] == MFE_NOT_CONVERGED && rc == MFE_OK)) rc = st_code[j];
        if (stats) {
            stats[j].status = st_code[j];
            stats[j].iterations = inner_its[j] + fb_its[j];
            stats[j].outer = outer_steps[j];
            stats[j].spmv_count = inner_its[j] + fb_its[j] + outer_steps[j] + 1;
            stats[j].rel_res_recurrence = rel[j];
            stats[j].rel_res_true = rel[j];
            stats[j].seconds = secs;
            stats[j].guess_rejected = 0;
            stats[j].reserved_ = 0;
        }
    }
    return rc;
}

int mfe_cg_batched(mfe_ctx *ctx, int nsys, mfe_problem *const *sys, int format, double *const *x_dev, double tol,
                   int max_iter, int mixed, mfe_cg_stats *stats) {
    clear_error();
    if (!ctx || !sys || !x_dev || nsys < 1 || !(tol >= 0.0) || max_iter < 0 || (mixed != 0 && mixed != 1) ||
        (format != MFE_CSR && format != MFE_BCRS13)) {
        set_error("need ctx, sys, x, nsys >= 1, tol >= 0, max_iter >= 0, mixed 0 or 1, format CSR or BCRS13");
        return MFE_EINVAL;
    }
    for (int j = 0; j < nsys; ++j)
        if (!x_dev[j]) {
            set_error("every system needs its x");
            return MFE_EINVAL;
        }
    if (mixed && max_iter < 1) {
        set_error("the mixed-precision solve needs max_iter >= 1");
        return MFE_EINVAL;
    }
    mfe_batch *B = nullptr;
    MFE_TRY(mfe_batch_from_problems(ctx, nsys, sys, format, mixed ? (MFE_F64 | MFE_F32) : MFE_F64, &B));
    hipStream_t s = ctx->stream;
    int rc = MFE_OK;
    {
        TempBuffer x(ctx);
        rc = x.alloc((size_t)B->P->m * sizeof(double));
        double *xb = (double *)x.ptr();
        for (int j = 0; j < nsys && rc == MFE_OK; ++j)
            if (hipMemcpyAsync(xb + B->row0[j], x_dev[j], sys[j]->m * sizeof(double), hipMemcpyDeviceToDevice, s) !=
                hipSuccess) {
                set_error("gather of the initial guesses failed");
                rc = MFE_EHIP;
            }
        if (rc == MFE_OK)
            rc = mixed ? mfe_batch_cg_mixed(B, format, xb, tol, 1e-4, 50, max_iter, stats)
                       : mfe_batch_cg(B, format, xb, tol, max_iter, stats);
        // results (the last iterates after a breakdown) back to each system's x
        if (rc == MFE_OK || rc == MFE_NOT_CONVERGED || rc == MFE_EBREAKDOWN)
            for (int j = 0; j < nsys; ++j)
                if (hipMemcpyAsync(x_dev[j], xb + B->row0[j], sys[j]->m * sizeof(double), hipMemcpyDeviceToDevice,
                                   s) != hipSuccess) {
                    set_error("scatter of the solutions failed");
                    rc = MFE_EHIP;
                    break;
                }
    }
    mfe_batch_destroy(B);
    return rc;
}

}  // extern "C"
