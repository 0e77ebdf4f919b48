// Result verification (Sec. 1): the computed nodal values against the
// separation-of-variables solution of the paper's problem (Laplace equation
// on the unit cube, u = 1 on x = 1, u = 0 on the other five faces):
//
//   u(x, y, z) = sum over odd p, q of  16 / (pi^2 p q) sin(p pi y) sin(q pi z)
//                                      sinh(g x) / sinh(g),   g = pi sqrt(p^2 + q^2).
//
// The sinh ratio is evaluated as e^{g(x-1)} (1 - e^{-2gx}) / (1 - e^{-2g}),
// which never overflows.  For fixed p the term bound 16/(pi^2 p q) e^{g(x-1)}
// decreases in q, and its q = 1 value decreases in p, so both loops stop at
// the first term whose bound is below 1e-18.  Near x = 1 the series
// converges slowly (the boundary data jump at the edges of the x = 1 face),
// so only nodes with x <= x_max are evaluated.
#include <cmath>

#include "common.hpp"
#include "device_util.hpp"

namespace mfe {
namespace {

constexpr double kPi = 3.14159265358979323846;

__device__ double series_u(double x, double y, double z) {
    const double c0 = 16.0 / (kPi * kPi);
    double u = 0.0;
    for (int p = 1;; p += 2) {
        if (c0 / p * exp(kPi * p * (x - 1.0)) < 1e-18) break;
        const double sp = sinpi(p * y);
        for (int q = 1;; q += 2) {
            const double g = kPi * sqrt((double)p * p + (double)q * q);
            const double e = exp(g * (x - 1.0));
            const double bound = c0 / ((double)p * q) * e;
            if (bound < 1e-18) break;
            const double ratio = e * (1.0 - exp(-2.0 * g * x)) / (1.0 - exp(-2.0 * g));
            u += bound / e * sp * sinpi(q * z) * ratio;
        }
    }
    return u;
}

// Nodes with ix <= ixmax: series value (optional store), and per-workgroup
// partials of max |x - u|, sum (x - u)^2 and the node count.
__global__ __launch_bounds__(kBlock) void k_verify(int Nx, int Ny, int Nz, int ixmax, const double *__restrict__ xs,
                                                   double *__restrict__ u_out, double *__restrict__ part) {
    const int nx = Nx + 1, ny = Ny + 1;
    const int64_t m = (int64_t)nx * ny * (Nz + 1);
    double emax = 0.0, esq = 0.0, cnt = 0.0;
    const int64_t stride = (int64_t)gridDim.x * kBlock;
    for (int64_t i = (int64_t)blockIdx.x * kBlock + threadIdx.x; i < m; i += stride) {
        const int ix = (int)(i % nx), iy = (int)((i / nx) % ny), iz = (int)(i / ((int64_t)nx * ny));
        if (ix > ixmax) {
            if (u_out) u_out[i] = NAN;
            continue;
        }
        const double u = series_u((double)ix / Nx, (double)iy / Ny, (double)iz / Nz);
        if (u_out) u_out[i] = u;
        const double e = xs[i] - u;
        emax = fmax(emax, fabs(e));
        esq += e * e;
        cnt += 1.0;
    }
    __shared__ double red[3][kBlock / 64];
    const int w = threadIdx.x >> 6;
    // wavefront reductions: max by xor butterfly, sums by wave_sum
    for (int off = 32; off > 0; off >>= 1) emax = fmax(emax, __shfl_xor(emax, off, 64));
    esq = wave_sum(esq);
    cnt = wave_sum(cnt);
    if ((threadIdx.x & 63) == 0) {
        red[0][w] = emax;
        red[1][w] = esq;
        red[2][w] = cnt;
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        double a = 0.0, b = 0.0, c = 0.0;
        for (int k = 0; k < kBlock / 64; ++k) {
            a = fmax(a, red[0][k]);
            b += red[1][k];
            c += red[2][k];
        }
        part[blockIdx.x] = a;
        part[kMaxPartials + blockIdx.x] = b;
        part[2 * kMaxPartials + blockIdx.x] = c;
    }
}

// One workgroup: combine the partials in a fixed order into out[0..2].
__global__ __launch_bounds__(kBlock) void k_verify_fin(const double *__restrict__ part, int n, double *__restrict__ out) {
    const double b = sum_partials(part + kMaxPartials, n);
    const double c = sum_partials(part + 2 * kMaxPartials, n);
    if (threadIdx.x != 0) return;
    double a = 0.0;
    for (int k = 0; k < n; ++k) a = fmax(a, part[k]);
    out[0] = a;
    out[1] = b;
    out[2] = c;
}

}  // namespace
}  // namespace mfe

using namespace mfe;

extern "C" int mfe_verify_series(const mfe_problem *p, const double *x_dev, double x_max, double *u_dev,
                                 double *max_err, double *rms_err, int64_t *count) {
    clear_error();
    if (!p || !x_dev || !max_err || !rms_err || !count) {
        set_error("problem, x, max_err, rms_err and count must be non-NULL");
        return MFE_EINVAL;
    }
    if (!p->is_mesh) {
        set_error("verification needs a problem made by mfe_problem_create (mesh sizes)");
        return MFE_EUNSUPPORTED;
    }
    if (!(x_max > 0.0 && x_max < 1.0)) {
        set_error("x_max must lie in (0, 1)");
        return MFE_EINVAL;
    }
    mfe_ctx *ctx = p->ctx;
    MFE_HIP_TRY(hipSetDevice(ctx->device));
    hipStream_t s = ctx->stream;
    // largest ix with ix / Nx <= x_max
    int ixmax = (int)std::floor(x_max * p->Nx);
    while (ixmax + 1 <= p->Nx && (double)(ixmax + 1) / p->Nx <= x_max) ++ixmax;
    while (ixmax >= 0 && (double)ixmax / p->Nx > x_max) --ixmax;
    const int g = resident_grid((long)ctx->num_cu * resident_per_cu((const void *)k_verify),
                                (long)((p->m + kBlock - 1) / kBlock));
    double *part = (double *)p->partials.ptr;
    Buffer tmp;
    if (!part) {
        MFE_TRY(dev_alloc(ctx, &tmp, 3 * kMaxPartials * sizeof(double) + 4 * sizeof(double)));
        part = (double *)tmp.ptr;
    }
    double *out = (double *)ctx->scratch.ptr;
    hipLaunchKernelGGL(k_verify, dim3(g), dim3(kBlock), 0, s, p->Nx, p->Ny, p->Nz, ixmax, x_dev, u_dev, part);
    hipLaunchKernelGGL(k_verify_fin, dim3(1), dim3(kBlock), 0, s, (const double *)part, g, out);
    int rc = hipGetLastError() == hipSuccess ? MFE_OK : MFE_EHIP;
    double h[3] = {0, 0, 0};
    double *pin = (double *)((CgState *)ctx->pinned + 3);
    if (rc == MFE_OK && hipMemcpyAsync(pin, out, 3 * sizeof(double), hipMemcpyDeviceToHost, s) != hipSuccess)
        rc = MFE_EHIP;
    if (hipStreamSynchronize(s) != hipSuccess && rc == MFE_OK) rc = MFE_EHIP;
    if (rc == MFE_OK) {
        h[0] = pin[0];
        h[1] = pin[1];
        h[2] = pin[2];
    }
    if (tmp.ptr) dev_free(ctx, &tmp);
    if (rc != MFE_OK) {
        set_error("verification kernel failed");
        return rc;
    }
    *max_err = h[0];
    *count = (int64_t)h[2];
    *rms_err = h[2] > 0 ? std::sqrt(h[1] / h[2]) : 0.0;
    return MFE_OK;
}
