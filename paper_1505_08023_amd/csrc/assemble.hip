// Mesh, matrix structure, element assembly and Dirichlet elimination on the
// GPU (Sec. 1 problem statement and assembly module; Fig 3.6 structure loop;
// Fig 3.7 element loop).
//
// The paper assembles element by element and scatters into the global CRS
// under a critical section.  Here each thread owns one matrix row (one mesh
// node) and gathers: for every in-range neighbour j of node i it sums, over
// the elements that contain both nodes in ascending element order, the
// element-matrix entry coupling them.  No atomics; every row is written by
// exactly one thread, so the result is deterministic.
#include "common.hpp"
#include "device_util.hpp"

namespace mfe {
namespace {

struct Mesh {
    int Nx, Ny, Nz;
    int nx, ny, nz;            // nodes per axis
    double kpat[8];            // element-matrix entry by coupling pattern (see below)
    double face[6];            // x0, x1, y0, y1, z0, z1
    const double *node_g;      // optional per-node boundary values
};

// Element stiffness of a brick with sides hx, hy, hz (trilinear shape
// functions, integral of grad N_a . grad N_b):
//   K_ab = (hy hz/hx) s_x m_y m_z + (hx hz/hy) m_x s_y m_z + (hx hy/hz) m_x m_y s_z
// per axis s = +1, m = 1/3 when a and b share that coordinate, s = -1,
// m = 1/6 when they differ.  The entry depends only on the pattern
// d = (a xor b) of differing axes (bit 0 x, bit 1 y, bit 2 z).
void element_patterns(double hx, double hy, double hz, double kpat[8]) {
    const double cx = hy * hz / hx, cy = hx * hz / hy, cz = hx * hy / hz;
    for (int d = 0; d < 8; ++d) {
        const bool dx = d & 1, dy = d & 2, dz = d & 4;
        const double sx = dx ? -1.0 : 1.0, sy = dy ? -1.0 : 1.0, sz = dz ? -1.0 : 1.0;
        const double mx = dx ? 1.0 / 6.0 : 1.0 / 3.0, my = dy ? 1.0 / 6.0 : 1.0 / 3.0,
                     mz = dz ? 1.0 / 6.0 : 1.0 / 3.0;
        kpat[d] = cx * sx * my * mz + cy * mx * sy * mz + cz * mx * my * sz;
    }
}

// Number of row entries contributed by line position i of an axis with N
// elements (in-range neighbours among i-1, i, i+1), and the prefix sum of
// those counts over positions 0..i-1.
__device__ __forceinline__ int line_count(int i, int N) { return (i == 0 || i == N) ? 2 : 3; }
__device__ __forceinline__ int64_t line_prefix(int i) { return i == 0 ? 0 : 2 + 3 * (int64_t)(i - 1); }

// Boundary value of a node, or false for an interior node.  A node on several
// faces takes the first face in the order x=1, x=0, y=1, y=0, z=1, z=0.
__device__ __forceinline__ bool boundary_value(const Mesh &M, int ix, int iy, int iz, int64_t id,
                                               double &g) {
    int f;
    if (ix == M.Nx) f = 1;
    else if (ix == 0) f = 0;
    else if (iy == M.Ny) f = 3;
    else if (iy == 0) f = 2;
    else if (iz == M.Nz) f = 5;
    else if (iz == 0) f = 4;
    else return false;
    g = M.node_g ? M.node_g[id] : M.face[f];
    return true;
}

// Number of elements containing node i and its neighbour at offset s along
// an axis with N elements: for s = 0 the elements left/right of i that exist,
// else the single element between them.
__device__ __forceinline__ int shared_elements(int i, int s, int N) {
    if (s != 0) return 1;
    return (i > 0) + (i < N);
}

// One thread per row, one 64-thread workgroup per 64 consecutive rows.
// mode 0: structure + values + rhs; mode 1: rhs only.  The rows of a
// workgroup own one contiguous run of the CRS arrays: each thread writes its
// row's entries into LDS at its offset in that run, then the workgroup copies
// the run to memory with coalesced stores.  The mesh's rows and entries are
// written at offsets row_off / nnz_off of the arrays (column indices shifted
// by row_off), so several meshes can form one block-diagonal matrix.
constexpr int kAsmRows = 64;
__global__ __launch_bounds__(kAsmRows) void k_assemble(Mesh M, int64_t row_off, int64_t nnz_off,
                                                       int32_t *__restrict__ ptr, int32_t *__restrict__ col,
                                                       double *__restrict__ val, double *__restrict__ b,
                                                       int rhs_only) {
    __shared__ int32_t scol[kAsmRows * 27];
    __shared__ double sval[kAsmRows * 27];
    const int64_t m = (int64_t)M.nx * M.ny * M.nz;
    const int64_t i0 = (int64_t)blockIdx.x * kAsmRows;
    const int64_t i = i0 + threadIdx.x;
    const bool live = i < m;
    const int64_t ic = live ? i : m - 1;  // rows past the end compute row m-1 and discard it
    const int ix = (int)(ic % M.nx);
    const int iy = (int)((ic / M.nx) % M.ny);
    const int iz = (int)(ic / ((int64_t)M.nx * M.ny));

    const int64_t SX = 3 * (int64_t)M.Nx + 1, SY = 3 * (int64_t)M.Ny + 1;
    const int cy = line_count(iy, M.Ny), cz = line_count(iz, M.Nz);
    const int64_t start = SX * SY * line_prefix(iz) + SX * line_prefix(iy) * cz +
                          line_prefix(ix) * (int64_t)cy * cz;
    const int64_t end = start + (int64_t)line_count(ix, M.Nx) * cy * cz;
    if (!rhs_only && live) {
        ptr[row_off + i] = (int32_t)(nnz_off + start);
        if (i == m - 1) ptr[row_off + m] = (int32_t)(nnz_off + end);
    }
    // the workgroup's run of entries: from its first row's start to its last live row's end
    const int64_t run_lo = __shfl(start, 0, 64);
    int64_t run_hi = live ? end : 0;
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) {
        const int64_t o = __shfl_xor(run_hi, off, 64);
        run_hi = o > run_hi ? o : run_hi;
    }

    double gi;
    const bool dir_i = boundary_value(M, ix, iy, iz, ic, gi);
    double bi = 0.0;  // zero source: element loads vanish
    int64_t k = start;
    for (int sz = -1; sz <= 1; ++sz) {
        const int jz = iz + sz;
        if (jz < 0 || jz > M.Nz) continue;
        for (int sy = -1; sy <= 1; ++sy) {
            const int jy = iy + sy;
            if (jy < 0 || jy > M.Ny) continue;
            for (int sx = -1; sx <= 1; ++sx) {
                const int jx = ix + sx;
                if (jx < 0 || jx > M.Nx) continue;
                const int64_t j = ic + sx + (int64_t)M.nx * (sy + (int64_t)M.ny * sz);
                // sum of the element entries over the shared elements
                const int ne = shared_elements(ix, sx, M.Nx) * shared_elements(iy, sy, M.Ny) *
                               shared_elements(iz, sz, M.Nz);
                const double kij = M.kpat[(sx != 0) | ((sy != 0) << 1) | ((sz != 0) << 2)];
                double raw = 0.0;
                for (int e = 0; e < ne; ++e) raw += kij;
                double v = raw;
                if (dir_i) {
                    v = (j == ic) ? 1.0 : 0.0;
                } else {
                    double gj;
                    if (boundary_value(M, jx, jy, jz, j, gj)) {
                        bi -= raw * gj;
                        v = 0.0;
                    }
                }
                if (!rhs_only && live) {
                    scol[k - run_lo] = (int32_t)(row_off + j);
                    sval[k - run_lo] = v;
                }
                ++k;
            }
        }
    }
    if (live) b[row_off + i] = dir_i ? gi : bi;
    if (rhs_only) return;  // uniform over the workgroup
    __syncthreads();
    for (int64_t t = run_lo + threadIdx.x; t < run_hi; t += kAsmRows) {
        col[nnz_off + t] = scol[t - run_lo];
        val[nnz_off + t] = sval[t - run_lo];
    }
}

}  // namespace

int launch_assemble_into(hipStream_t s, int Nx, int Ny, int Nz, const double *face_vals, const double *node_g,
                         int64_t row_off, int64_t nnz_off, int32_t *ptr, int32_t *col, double *val, double *b,
                         bool rhs_only) {
    Mesh M{};
    M.Nx = Nx;
    M.Ny = Ny;
    M.Nz = Nz;
    M.nx = Nx + 1;
    M.ny = Ny + 1;
    M.nz = Nz + 1;
    element_patterns(1.0 / Nx, 1.0 / Ny, 1.0 / Nz, M.kpat);
    static const double paper_faces[6] = {0.0, 1.0, 0.0, 0.0, 0.0, 0.0};
    const double *f = face_vals ? face_vals : paper_faces;
    for (int i = 0; i < 6; ++i) M.face[i] = f[i];
    M.node_g = node_g;
    const int64_t m = (int64_t)M.nx * M.ny * M.nz;
    const int64_t grid = (m + kAsmRows - 1) / kAsmRows;
    hipLaunchKernelGGL(k_assemble, dim3((unsigned)grid), dim3(kAsmRows), 0, s, M, row_off, nnz_off, ptr, col, val, b,
                       rhs_only ? 1 : 0);
    MFE_HIP_TRY(hipGetLastError());
    return MFE_OK;
}

int launch_assemble(mfe_problem *P, const double *face_vals, const double *node_g, bool values_and_rhs,
                    bool rhs_only) {
    (void)values_and_rhs;
    return launch_assemble_into(P->ctx->stream, P->Nx, P->Ny, P->Nz, face_vals, node_g, 0, 0, (int32_t *)P->ptr.ptr,
                                (int32_t *)P->col.ptr, (double *)P->val64.ptr, (double *)P->b.ptr, rhs_only);
}

}  // namespace mfe
