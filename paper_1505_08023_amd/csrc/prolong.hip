// Trilinear prolongation of nodal values from a box mesh to the mesh refined
// `factor` times per axis: the interpolant of the trilinear elements of the
// coarse mesh (Sec. 1 element space) evaluated at the fine nodes.  It turns a
// coarse solution (or a coarse prediction of the learned initial guess) into
// an initial guess on the fine mesh.  Optionally the fine boundary nodes take
// given values instead (the fine problem's Dirichlet data: the interpolant of
// a coarse face differs from the fine face data near the face's edges).
#include "common.hpp"

namespace mfe {
namespace {

__global__ __launch_bounds__(kBlock) void k_prolong(int Nx, int Ny, int Nz, int f, const double *__restrict__ xc,
                                                    const double *__restrict__ bnd, double *__restrict__ xf) {
    const int fx = Nx * f, fy = Ny * f, fz = Nz * f;
    const int64_t cnx = Nx + 1, cny = Ny + 1;
    const int64_t nx = fx + 1, ny = fy + 1;
    const int64_t m = nx * ny * (fz + 1);
    const int64_t stride = (int64_t)gridDim.x * kBlock;
    for (int64_t i = (int64_t)blockIdx.x * kBlock + threadIdx.x; i < m; i += stride) {
        const int ix = (int)(i % nx), iy = (int)((i / nx) % ny), iz = (int)(i / (nx * ny));
        if (bnd && (ix == 0 || iy == 0 || iz == 0 || ix == fx || iy == fy || iz == fz)) {
            xf[i] = bnd[i];
            continue;
        }
        // coarse cell (clamped so that the last node uses the last cell) and local coordinates
        const int cx = min(ix / f, Nx - 1), cy = min(iy / f, Ny - 1), cz = min(iz / f, Nz - 1);
        const double tx = (double)(ix - cx * f) / f, ty = (double)(iy - cy * f) / f, tz = (double)(iz - cz * f) / f;
        const double *c = xc + cx + cnx * (cy + cny * cz);
        const int64_t sy = cnx, sz = cnx * cny;
        const double v00 = c[0] + tx * (c[1] - c[0]);
        const double v10 = c[sy] + tx * (c[sy + 1] - c[sy]);
        const double v01 = c[sz] + tx * (c[sz + 1] - c[sz]);
        const double v11 = c[sz + sy] + tx * (c[sz + sy + 1] - c[sz + sy]);
        const double w0 = v00 + ty * (v10 - v00), w1 = v01 + ty * (v11 - v01);
        xf[i] = w0 + tz * (w1 - w0);
    }
}

}  // namespace
}  // namespace mfe

using namespace mfe;

extern "C" int mfe_prolong_trilinear(mfe_ctx *ctx, int Nx, int Ny, int Nz, const double *xc_dev, int factor,
                                     const double *bnd_dev, double *xf_dev) {
    clear_error();
    if (!ctx || !xc_dev || !xf_dev || Nx < 1 || Ny < 1 || Nz < 1 || factor < 1) {
        set_error("need ctx, xc, xf, Nx, Ny, Nz >= 1 and factor >= 1");
        return MFE_EINVAL;
    }
    const int64_t fx = (int64_t)Nx * factor, fy = (int64_t)Ny * factor, fz = (int64_t)Nz * factor;
    if ((fx + 1) * (fy + 1) * (fz + 1) >= ((int64_t)1 << 31) - 1) {
        set_error("fine mesh beyond 32-bit node numbering");
        return MFE_EUNSUPPORTED;
    }
    MFE_HIP_TRY(hipSetDevice(ctx->device));
    const int64_t m = (fx + 1) * (fy + 1) * (fz + 1);
    const int grid = resident_grid((long)ctx->num_cu * 8, (long)((m + kBlock - 1) / kBlock));
    hipLaunchKernelGGL(k_prolong, dim3(grid), dim3(kBlock), 0, ctx->stream, Nx, Ny, Nz, factor, xc_dev, bnd_dev,
                       xf_dev);
    MFE_HIP_TRY(hipGetLastError());
    return MFE_OK;
}
