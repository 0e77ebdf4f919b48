// extern "C" entry points declared in include/mfe.h: argument checks,
// object lifetime, and dispatch to the kernel launchers.
#include <cstring>
#include <mutex>
#include <new>
#include <string>
#include <unordered_map>

#include "common.hpp"

namespace mfe {

namespace {
thread_local std::string g_error;
}

void set_error(const std::string &msg) { g_error = msg; }
void clear_error() { g_error.clear(); }

int dev_alloc(mfe_ctx *ctx, Buffer *b, size_t bytes) {
    if (bytes == 0) bytes = 256;
    void *p = nullptr;
    if (ctx->alloc) {
        p = ctx->alloc(bytes, ctx->alloc_user);
    } else if (hipMalloc(&p, bytes) != hipSuccess) {
        (void)hipGetLastError();
        p = nullptr;
    }
    if (!p) {
        set_error("device allocation of " + std::to_string(bytes) + " bytes failed");
        return MFE_ENOMEM;
    }
    b->ptr = p;
    b->bytes = bytes;
    return MFE_OK;
}

void dev_free(mfe_ctx *ctx, Buffer *b) {
    if (!b->ptr) return;
    if (ctx->free_fn) ctx->free_fn(b->ptr, ctx->alloc_user);
    else (void)hipFree(b->ptr);
    b->ptr = nullptr;
    b->bytes = 0;
}

TempBuffer::~TempBuffer() {
    if (!b.ptr) return;
    (void)hipStreamSynchronize(ctx->stream);
    dev_free(ctx, &b);
}

int resident_per_cu(const void *kernel) {
    static std::mutex mu;
    static std::unordered_map<const void *, int> cache;
    std::lock_guard<std::mutex> lock(mu);
    auto it = cache.find(kernel);
    if (it != cache.end()) return it->second;
    int n = 0;
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&n, kernel, kBlock, 0) != hipSuccess || n < 1) {
        (void)hipGetLastError();
        n = 1;
    }
    cache[kernel] = n;
    return n;
}

int resident_grid(long max_groups, long ntiles) {
    long g = max_groups < kMaxPartials ? max_groups : kMaxPartials;
    const long need = (ntiles + kNumXcd - 1) / kNumXcd * kNumXcd;
    if (need < g) g = need;
    if (g < kNumXcd) g = kNumXcd;
    return (int)(g / kNumXcd * kNumXcd);
}

}  // namespace mfe

using namespace mfe;

namespace {

bool fits_int32(int64_t v) { return v >= 0 && v < ((int64_t)1 << 31) - 1; }

int set_device(const mfe_ctx *ctx) {
    MFE_HIP_TRY(hipSetDevice(ctx->device));
    return MFE_OK;
}

}  // namespace

namespace mfe {

void free_problem_storage(mfe_problem *P) {
    mfe_ctx *ctx = P->ctx;
    release_graphs(P);
    Buffer *bufs[] = {&P->ptr, &P->col, &P->val64, &P->val32, &P->b, &P->slot_base, &P->jas, &P->bval64,
                      &P->bval32, &P->rowblocks, &P->bdesc, &P->cdesc, &P->citems, &P->crows, &P->r, &P->p, &P->q,
                      &P->state, &P->partials,
                      &P->r32, &P->p32, &P->q32, &P->d32, &P->ax, &P->s, &P->dinv};
    for (Buffer *b : bufs) dev_free(ctx, b);
}

// Derived formats and precisions after the FP64 CRS exists.
int finish_problem(mfe_problem *P) {
    // the wavefront tiles and their descriptors serve the CRS product only
    // where it does not walk row groups
    MFE_TRY(build_csr_groups(P));
    if (P->ncitems == 0) MFE_TRY(build_csr_tiles(P));
    if (P->formats & MFE_BCRS13) MFE_TRY(build_bcrs13(P));
    if (P->precisions & MFE_F32) MFE_TRY(cast_values_f32(P));
    MFE_HIP_TRY(hipStreamSynchronize(P->ctx->stream));
    return MFE_OK;
}

}  // namespace mfe

namespace {

int check_format(const mfe_problem *p, int format) {
    if (format != MFE_CSR && format != MFE_BCRS13) {
        set_error("format must be MFE_CSR or MFE_BCRS13");
        return MFE_EINVAL;
    }
    if (!(p->formats & format)) {
        set_error("format was not built for this problem");
        return MFE_EUNSUPPORTED;
    }
    return MFE_OK;
}

}  // namespace

extern "C" {

const char *mfe_last_error(void) { return g_error.c_str(); }

int mfe_version(void) { return 13; }

int mfe_ctx_create(int device, void *stream, mfe_alloc_fn alloc, mfe_free_fn free_fn, void *alloc_user,
                   mfe_ctx **out) {
    clear_error();
    if (!out) {
        set_error("out is NULL");
        return MFE_EINVAL;
    }
    *out = nullptr;
    if ((alloc == nullptr) != (free_fn == nullptr)) {
        set_error("alloc and free callbacks must be given together");
        return MFE_EINVAL;
    }
    int ndev = 0;
    MFE_HIP_TRY(hipGetDeviceCount(&ndev));
    if (device < 0 || device >= ndev) {
        set_error("device index out of range");
        return MFE_EINVAL;
    }
    MFE_HIP_TRY(hipSetDevice(device));
    mfe_ctx *c = new (std::nothrow) mfe_ctx();
    if (!c) {
        set_error("host allocation failed");
        return MFE_ENOMEM;
    }
    c->device = device;
    c->stream = (hipStream_t)stream;
    c->alloc = alloc;
    c->free_fn = free_fn;
    c->alloc_user = alloc_user;
    hipDeviceProp_t prop;
    int rc = MFE_OK;
    if (hipGetDeviceProperties(&prop, device) != hipSuccess ||
        hipStreamCreateWithFlags(&c->cap_stream, hipStreamNonBlocking) != hipSuccess ||
        hipHostMalloc(&c->pinned, kPinnedSlots * sizeof(CgState), hipHostMallocDefault) != hipSuccess ||
        hipEventCreateWithFlags(&c->ev[0], hipEventDisableTiming) != hipSuccess ||
        hipEventCreateWithFlags(&c->ev[1], hipEventDisableTiming) != hipSuccess) {
        set_error(std::string("context setup failed: ") + hipGetErrorString(hipGetLastError()));
        rc = MFE_EHIP;
    }
    if (rc == MFE_OK) rc = noalloc_init(device);
    if (rc == MFE_OK) {
        c->num_cu = prop.multiProcessorCount;
        rc = dev_alloc(c, &c->scratch, kMaxPartials * sizeof(double));
    }
    if (rc == MFE_OK) rc = dev_alloc(c, &c->dot_state, sizeof(CgState));
    if (rc == MFE_OK) rc = dev_alloc(c, &c->spmv_dot_state, sizeof(CgState));
    if (rc == MFE_OK && (hipMemsetAsync(c->dot_state.ptr, 0, sizeof(CgState), c->stream) != hipSuccess ||
                         hipMemsetAsync(c->spmv_dot_state.ptr, 0, sizeof(CgState), c->stream) != hipSuccess)) {
        set_error("hipMemsetAsync failed");
        rc = MFE_EHIP;
    }
    if (rc != MFE_OK) {
        mfe_ctx_destroy(c);
        return rc;
    }
    *out = c;
    return MFE_OK;
}

int mfe_ctx_destroy(mfe_ctx *ctx) {
    if (!ctx) return MFE_OK;
    (void)hipSetDevice(ctx->device);
    (void)hipStreamSynchronize(ctx->stream);
    while (!ctx->nets.empty()) mfe_net_destroy(ctx->nets.back());
    while (!ctx->batches.empty()) mfe_batch_destroy(ctx->batches.back());
    while (!ctx->problems.empty()) mfe_problem_destroy(ctx->problems.back());
    dev_free(ctx, &ctx->scratch);
    dev_free(ctx, &ctx->dot_state);
    dev_free(ctx, &ctx->spmv_dot_state);
    if (ctx->ev[0]) (void)hipEventDestroy(ctx->ev[0]);
    if (ctx->ev[1]) (void)hipEventDestroy(ctx->ev[1]);
    if (ctx->pinned) (void)hipHostFree(ctx->pinned);
    if (ctx->cap_stream) (void)hipStreamDestroy(ctx->cap_stream);
    delete ctx;
    return MFE_OK;
}

int mfe_problem_create(mfe_ctx *ctx, int Nx, int Ny, int Nz, const double *face_vals, const double *node_g_dev,
                       int formats, int precisions, mfe_problem **out) {
    clear_error();
    if (!ctx || !out) {
        set_error("ctx and out must be non-NULL");
        return MFE_EINVAL;
    }
    *out = nullptr;
    if (Nx < 1 || Ny < 1 || Nz < 1) {
        set_error("Nx, Ny, Nz must be >= 1");
        return MFE_EINVAL;
    }
    if ((formats & ~(MFE_CSR | MFE_BCRS13)) || (precisions & ~(MFE_F64 | MFE_F32))) {
        set_error("unknown format or precision flag");
        return MFE_EINVAL;
    }
    const int64_t m = (int64_t)(Nx + 1) * (Ny + 1) * (Nz + 1);
    const int64_t nnz = (3 * (int64_t)Nx + 1) * (3 * (int64_t)Ny + 1) * (3 * (int64_t)Nz + 1);
    if (!fits_int32(m) || !fits_int32(nnz)) {
        set_error("mesh too large for 32-bit row pointers (nnz >= 2^31)");
        return MFE_EUNSUPPORTED;
    }
    MFE_TRY(set_device(ctx));
    mfe_problem *P = new (std::nothrow) mfe_problem();
    if (!P) {
        set_error("host allocation failed");
        return MFE_ENOMEM;
    }
    P->ctx = ctx;
    P->is_mesh = true;
    P->Nx = Nx;
    P->Ny = Ny;
    P->Nz = Nz;
    P->m = m;
    P->nnz = nnz;
    P->formats = formats | MFE_CSR;
    P->precisions = precisions | MFE_F64;
    int rc = dev_alloc(ctx, &P->ptr, (size_t)(m + 1) * sizeof(int32_t));
    if (rc == MFE_OK) rc = dev_alloc(ctx, &P->col, (size_t)nnz * sizeof(int32_t));
    if (rc == MFE_OK) rc = dev_alloc(ctx, &P->val64, (size_t)nnz * sizeof(double));
    if (rc == MFE_OK) rc = dev_alloc(ctx, &P->b, (size_t)m * sizeof(double));
    if (rc == MFE_OK) rc = launch_assemble(P, face_vals, node_g_dev, true, false);
    if (rc == MFE_OK) rc = finish_problem(P);
    if (rc != MFE_OK) {
        (void)hipStreamSynchronize(ctx->stream);
        free_problem_storage(P);
        delete P;
        return rc;
    }
    ctx->problems.push_back(P);
    *out = P;
    return MFE_OK;
}

int mfe_problem_from_csr(mfe_ctx *ctx, int64_t m, const int32_t *ptr_dev, const int32_t *col_dev,
                         const double *val_dev, const double *b_dev, int formats, int precisions,
                         mfe_problem **out) {
    clear_error();
    if (!ctx || !out || !ptr_dev || !col_dev || !val_dev) {
        set_error("ctx, out, ptr, col and val must be non-NULL");
        return MFE_EINVAL;
    }
    *out = nullptr;
    if (m < 1 || !fits_int32(m)) {
        set_error("m must be in [1, 2^31-1)");
        return MFE_EINVAL;
    }
    if ((formats & ~(MFE_CSR | MFE_BCRS13)) || (precisions & ~(MFE_F64 | MFE_F32))) {
        set_error("unknown format or precision flag");
        return MFE_EINVAL;
    }
    MFE_TRY(set_device(ctx));
    int32_t nnz32 = 0;
    MFE_HIP_TRY(hipMemcpyAsync(&nnz32, ptr_dev + m, sizeof(int32_t), hipMemcpyDeviceToHost, ctx->stream));
    MFE_HIP_TRY(hipStreamSynchronize(ctx->stream));
    if (nnz32 < 0) {
        set_error("ptr[m] must be >= 0");
        return MFE_EINVAL;
    }
    MFE_TRY(validate_csr(ctx, m, nnz32, ptr_dev, col_dev));
    mfe_problem *P = new (std::nothrow) mfe_problem();
    if (!P) {
        set_error("host allocation failed");
        return MFE_ENOMEM;
    }
    P->ctx = ctx;
    P->m = m;
    P->nnz = nnz32;
    P->formats = formats | MFE_CSR;
    P->precisions = precisions | MFE_F64;
    hipStream_t s = ctx->stream;
    int rc = dev_alloc(ctx, &P->ptr, (size_t)(m + 1) * sizeof(int32_t));
    if (rc == MFE_OK) rc = dev_alloc(ctx, &P->col, (size_t)nnz32 * sizeof(int32_t));
    if (rc == MFE_OK) rc = dev_alloc(ctx, &P->val64, (size_t)nnz32 * sizeof(double));
    if (rc == MFE_OK) rc = dev_alloc(ctx, &P->b, (size_t)m * sizeof(double));
    if (rc == MFE_OK &&
        (hipMemcpyAsync(P->ptr.ptr, ptr_dev, (m + 1) * sizeof(int32_t), hipMemcpyDeviceToDevice, s) != hipSuccess ||
         hipMemcpyAsync(P->col.ptr, col_dev, (size_t)nnz32 * sizeof(int32_t), hipMemcpyDeviceToDevice, s) !=
             hipSuccess ||
         hipMemcpyAsync(P->val64.ptr, val_dev, (size_t)nnz32 * sizeof(double), hipMemcpyDeviceToDevice, s) !=
             hipSuccess ||
         (b_dev ? hipMemcpyAsync(P->b.ptr, b_dev, m * sizeof(double), hipMemcpyDeviceToDevice, s)
                : hipMemsetAsync(P->b.ptr, 0, m * sizeof(double), s)) != hipSuccess)) {
        set_error("copy of the CRS arrays failed");
        rc = MFE_EHIP;
    }
    if (rc == MFE_OK) rc = finish_problem(P);
    if (rc != MFE_OK) {
        (void)hipStreamSynchronize(s);
        free_problem_storage(P);
        delete P;
        return rc;
    }
    ctx->problems.push_back(P);
    *out = P;
    return MFE_OK;
}

int mfe_problem_from_csr_host(mfe_ctx *ctx, int64_t m, const int32_t *ptr, const int32_t *col, const double *val,
                              const double *b, int formats, int precisions, mfe_problem **out) {
    clear_error();
    if (!ctx || !out || !ptr || !col || !val) {
        set_error("ctx, out, ptr, col and val must be non-NULL");
        return MFE_EINVAL;
    }
    if (m < 1 || !fits_int32(m) || ptr[0] != 0 || ptr[m] < 0) {
        set_error("m must be in [1, 2^31-1), ptr[0] = 0 and ptr[m] >= 0");
        return MFE_EINVAL;
    }
    MFE_TRY(set_device(ctx));
    const int64_t nnz = ptr[m];
    hipStream_t s = ctx->stream;
    TempBuffer dp(ctx), dc(ctx), dv(ctx), db(ctx);
    MFE_TRY(dp.alloc((size_t)(m + 1) * sizeof(int32_t)));
    MFE_TRY(dc.alloc((size_t)nnz * sizeof(int32_t)));
    MFE_TRY(dv.alloc((size_t)nnz * sizeof(double)));
    if (b) MFE_TRY(db.alloc((size_t)m * sizeof(double)));
    MFE_HIP_TRY(hipMemcpyAsync(dp.ptr(), ptr, (m + 1) * sizeof(int32_t), hipMemcpyHostToDevice, s));
    if (nnz > 0) {
        MFE_HIP_TRY(hipMemcpyAsync(dc.ptr(), col, nnz * sizeof(int32_t), hipMemcpyHostToDevice, s));
        MFE_HIP_TRY(hipMemcpyAsync(dv.ptr(), val, nnz * sizeof(double), hipMemcpyHostToDevice, s));
    }
    if (b) MFE_HIP_TRY(hipMemcpyAsync(db.ptr(), b, m * sizeof(double), hipMemcpyHostToDevice, s));
    // the host arrays must stay valid until the copies have run
    MFE_HIP_TRY(hipStreamSynchronize(s));
    return mfe_problem_from_csr(ctx, m, (const int32_t *)dp.ptr(), (const int32_t *)dc.ptr(),
                                (const double *)dv.ptr(), b ? (const double *)db.ptr() : nullptr, formats, precisions,
                                out);
}

int mfe_problem_set_bc(mfe_problem *p, const double *face_vals, const double *node_g_dev) {
    clear_error();
    if (!p) {
        set_error("problem is NULL");
        return MFE_EINVAL;
    }
    if (!p->is_mesh) {
        set_error("boundary data can only be re-imposed on a mesh problem");
        return MFE_EINVAL;
    }
    MFE_TRY(set_device(p->ctx));
    return launch_assemble(p, face_vals, node_g_dev, false, true);
}

int mfe_problem_info(const mfe_problem *p, int64_t *m, int64_t *nnz, int64_t *nblocks) {
    clear_error();
    if (!p) {
        set_error("problem is NULL");
        return MFE_EINVAL;
    }
    if (m) *m = p->m;
    if (nnz) *nnz = p->nnz;
    if (nblocks) *nblocks = (p->formats & MFE_BCRS13) ? p->nblocks : 0;
    return MFE_OK;
}

int mfe_problem_csr_layout(const mfe_problem *p, int64_t *tile_rows, int64_t *tiles, int64_t *compressed_tiles) {
    clear_error();
    if (!p) {
        set_error("problem is NULL");
        return MFE_EINVAL;
    }
    if (tile_rows) *tile_rows = kCsrsRows;
    if (tiles) *tiles = (p->m + kCsrsRows - 1) / kCsrsRows;
    if (compressed_tiles) *compressed_tiles = p->csr_ctiles;
    return MFE_OK;
}

int mfe_problem_csr_groups(const mfe_problem *p, int64_t *items, int64_t *groups, int64_t *group_rows,
                           int64_t *other_rows) {
    clear_error();
    if (!p) {
        set_error("problem is NULL");
        return MFE_EINVAL;
    }
    if (items) *items = p->ncitems;
    if (groups) *groups = p->ncgroups;
    if (group_rows) *group_rows = p->ncgroup_rows;
    if (other_rows) *other_rows = p->ncitems > 0 ? p->ncrows : 0;
    return MFE_OK;
}

int mfe_problem_bcrs13_layout(const mfe_problem *p, int64_t *slices, int64_t *slots, int64_t *compressed_slices,
                              int64_t *compressed_blocks) {
    clear_error();
    if (!p) {
        set_error("problem is NULL");
        return MFE_EINVAL;
    }
    const bool built = (p->formats & MFE_BCRS13) != 0;
    if (slices) *slices = built ? (p->m + 63) / 64 : 0;
    if (slots) *slots = built ? p->nslots : 0;
    if (compressed_slices) *compressed_slices = built ? p->b13_cslices : 0;
    if (compressed_blocks) *compressed_blocks = built ? p->b13_cblocks : 0;
    return MFE_OK;
}

int mfe_problem_export_csr(const mfe_problem *p, int32_t *ptr_dev, int32_t *col_dev, double *val_dev,
                           double *b_dev) {
    clear_error();
    if (!p) {
        set_error("problem is NULL");
        return MFE_EINVAL;
    }
    MFE_TRY(set_device(p->ctx));
    hipStream_t s = p->ctx->stream;
    if (ptr_dev)
        MFE_HIP_TRY(hipMemcpyAsync(ptr_dev, p->ptr.ptr, (p->m + 1) * sizeof(int32_t), hipMemcpyDeviceToDevice, s));
    if (col_dev)
        MFE_HIP_TRY(hipMemcpyAsync(col_dev, p->col.ptr, p->nnz * sizeof(int32_t), hipMemcpyDeviceToDevice, s));
    if (val_dev)
        MFE_HIP_TRY(hipMemcpyAsync(val_dev, p->val64.ptr, p->nnz * sizeof(double), hipMemcpyDeviceToDevice, s));
    if (b_dev) MFE_HIP_TRY(hipMemcpyAsync(b_dev, p->b.ptr, p->m * sizeof(double), hipMemcpyDeviceToDevice, s));
    return MFE_OK;
}

int mfe_problem_export_csr_host(const mfe_problem *p, int32_t *ptr, int32_t *col, double *val, double *b) {
    clear_error();
    if (!p) {
        set_error("problem is NULL");
        return MFE_EINVAL;
    }
    MFE_TRY(set_device(p->ctx));
    hipStream_t s = p->ctx->stream;
    if (ptr) MFE_HIP_TRY(hipMemcpyAsync(ptr, p->ptr.ptr, (p->m + 1) * sizeof(int32_t), hipMemcpyDeviceToHost, s));
    if (col) MFE_HIP_TRY(hipMemcpyAsync(col, p->col.ptr, p->nnz * sizeof(int32_t), hipMemcpyDeviceToHost, s));
    if (val) MFE_HIP_TRY(hipMemcpyAsync(val, p->val64.ptr, p->nnz * sizeof(double), hipMemcpyDeviceToHost, s));
    if (b) MFE_HIP_TRY(hipMemcpyAsync(b, p->b.ptr, p->m * sizeof(double), hipMemcpyDeviceToHost, s));
    MFE_HIP_TRY(hipStreamSynchronize(s));
    return MFE_OK;
}

int mfe_rhs(const mfe_problem *p, double *b_dev) {
    clear_error();
    if (!p || !b_dev) {
        set_error("problem and b must be non-NULL");
        return MFE_EINVAL;
    }
    MFE_TRY(set_device(p->ctx));
    MFE_HIP_TRY(hipMemcpyAsync(b_dev, p->b.ptr, p->m * sizeof(double), hipMemcpyDeviceToDevice, p->ctx->stream));
    return MFE_OK;
}

int mfe_problem_export_bcrs13(const mfe_problem *p, int32_t *bptr_dev, int32_t *bcol_dev, double *bval_dev) {
    clear_error();
    if (!p) {
        set_error("problem is NULL");
        return MFE_EINVAL;
    }
    MFE_TRY(check_format(p, MFE_BCRS13));
    MFE_TRY(set_device(p->ctx));
    return export_bcrs13(p, bptr_dev, bcol_dev, bval_dev);
}

int mfe_problem_destroy(mfe_problem *p) {
    if (!p) return MFE_OK;
    mfe_ctx *ctx = p->ctx;
    (void)hipSetDevice(ctx->device);
    (void)hipStreamSynchronize(ctx->stream);
    free_problem_storage(p);
    unregister(ctx->problems, p);
    delete p;
    return MFE_OK;
}

int mfe_spmv(const mfe_problem *p, int format, const double *x_dev, double *y_dev) {
    clear_error();
    if (!p || !x_dev || !y_dev) {
        set_error("problem, x and y must be non-NULL");
        return MFE_EINVAL;
    }
    MFE_TRY(check_format(p, format));
    MFE_TRY(set_device(p->ctx));
    SpmvArgs a{x_dev, y_dev, nullptr, nullptr, nullptr, nullptr};
    return launch_spmv(p, format, false, kSpmvPlain, a, p->ctx->stream);
}

int mfe_spmv_f32(const mfe_problem *p, int format, const float *x_dev, float *y_dev) {
    clear_error();
    if (!p || !x_dev || !y_dev) {
        set_error("problem, x and y must be non-NULL");
        return MFE_EINVAL;
    }
    MFE_TRY(check_format(p, format));
    if (!(p->precisions & MFE_F32)) {
        set_error("FP32 values were not built for this problem");
        return MFE_EUNSUPPORTED;
    }
    MFE_TRY(set_device(p->ctx));
    SpmvArgs a{x_dev, y_dev, nullptr, nullptr, nullptr, nullptr};
    return launch_spmv(p, format, true, kSpmvPlain, a, p->ctx->stream);
}

int mfe_spmv_dot(const mfe_problem *p, int format, const double *p_dev, double *q_dev, double *pq_dev,
                 void *ev_before, void *ev_after) {
    clear_error();
    if (!p || !p_dev || !q_dev || !pq_dev) {
        set_error("problem, p, q and pq must be non-NULL");
        return MFE_EINVAL;
    }
    MFE_TRY(check_format(p, format));
    MFE_TRY(set_device(p->ctx));
    mfe_ctx *ctx = p->ctx;
    CgState *st = (CgState *)ctx->spmv_dot_state.ptr;
    // a running state with rho = 1, so the kernel's CG epilogue only publishes p.q
    MFE_TRY(launch_state_reset(st, pq_dev, ctx->stream));
    if (ev_before) MFE_HIP_TRY(hipEventRecord((hipEvent_t)ev_before, ctx->stream));
    SpmvArgs a{p_dev, q_dev, nullptr, nullptr, st, (double *)ctx->scratch.ptr};
    int n = 0;
    MFE_TRY(launch_spmv(p, format, false, kSpmvDot, a, ctx->stream, &n));
    if (ev_after) MFE_HIP_TRY(hipEventRecord((hipEvent_t)ev_after, ctx->stream));
    return launch_finalize(kFinDot, (const double *)ctx->scratch.ptr, n, st, ctx->stream);
}

int mfe_spmv_dot_f32(const mfe_problem *p, int format, const float *p_dev, float *q_dev, double *pq_dev,
                     void *ev_before, void *ev_after) {
    clear_error();
    if (!p || !p_dev || !q_dev || !pq_dev) {
        set_error("problem, p, q and pq must be non-NULL");
        return MFE_EINVAL;
    }
    MFE_TRY(check_format(p, format));
    if (!(p->precisions & MFE_F32)) {
        set_error("FP32 values were not built for this problem");
        return MFE_EUNSUPPORTED;
    }
    MFE_TRY(set_device(p->ctx));
    mfe_ctx *ctx = p->ctx;
    CgState *st = (CgState *)ctx->spmv_dot_state.ptr;
    MFE_TRY(launch_state_reset(st, pq_dev, ctx->stream));
    if (ev_before) MFE_HIP_TRY(hipEventRecord((hipEvent_t)ev_before, ctx->stream));
    SpmvArgs a{p_dev, q_dev, nullptr, nullptr, st, (double *)ctx->scratch.ptr};
    int n = 0;
    MFE_TRY(launch_spmv(p, format, true, kSpmvDot, a, ctx->stream, &n));
    if (ev_after) MFE_HIP_TRY(hipEventRecord((hipEvent_t)ev_after, ctx->stream));
    return launch_finalize(kFinDot, (const double *)ctx->scratch.ptr, n, st, ctx->stream);
}

int mfe_dot(mfe_ctx *ctx, int64_t n, const double *x_dev, const double *y_dev, double *out_host) {
    clear_error();
    if (!ctx || !out_host || n < 0 || (n > 0 && (!x_dev || !y_dev))) {
        set_error("ctx, out (and x, y when n > 0) must be non-NULL and n >= 0");
        return MFE_EINVAL;
    }
    MFE_TRY(set_device(ctx));
    CgState *st = (CgState *)ctx->dot_state.ptr;
    int g = 0;
    MFE_TRY(launch_dot(ctx, n, x_dev, y_dev, (double *)ctx->scratch.ptr, ctx->stream, &g));
    MFE_TRY(launch_state_reset(st, nullptr, ctx->stream));
    MFE_TRY(launch_finalize(kFinDot, (const double *)ctx->scratch.ptr, g, st, ctx->stream));
    CgState *pin = (CgState *)ctx->pinned;
    MFE_HIP_TRY(hipMemcpyAsync(&pin[3], st, sizeof(CgState), hipMemcpyDeviceToHost, ctx->stream));
    MFE_HIP_TRY(hipStreamSynchronize(ctx->stream));
    *out_host = pin[3].pq;
    return MFE_OK;
}

int mfe_stream_probe(mfe_ctx *ctx, int kind, int64_t n, const double *src_dev, double *dst_dev, void *ev_before,
                     void *ev_after) {
    clear_error();
    if (!ctx || (kind != 0 && kind != 1) || n < 0 || (n > 0 && (!src_dev || !dst_dev))) {
        set_error("ctx, kind 0 or 1, n >= 0 and (when n > 0) src and dst must be given");
        return MFE_EINVAL;
    }
    MFE_TRY(set_device(ctx));
    if (n == 0) return MFE_OK;
    if (ev_before) MFE_HIP_TRY(hipEventRecord((hipEvent_t)ev_before, ctx->stream));
    MFE_TRY(launch_stream_probe(ctx, kind, n, src_dev, dst_dev));
    if (ev_after) MFE_HIP_TRY(hipEventRecord((hipEvent_t)ev_after, ctx->stream));
    return MFE_OK;
}

int mfe_cg(const mfe_problem *p, int format, double *x_dev, double tol, int max_iter, double *hist_dev,
           mfe_cg_stats *stats) {
    clear_error();
    if (!p || !x_dev) {
        set_error("problem and x must be non-NULL");
        return MFE_EINVAL;
    }
    if (!(tol >= 0.0) || max_iter < 0) {
        set_error("tol must be >= 0 and max_iter >= 0");
        return MFE_EINVAL;
    }
    MFE_TRY(check_format(p, format));
    MFE_TRY(set_device(p->ctx));
    return cg_solve(const_cast<mfe_problem *>(p), format, x_dev, tol, max_iter, hist_dev, stats, false);
}

int mfe_cg_single_reduction(const mfe_problem *p, int format, double *x_dev, double tol, int max_iter,
                            double *hist_dev, mfe_cg_stats *stats) {
    clear_error();
    if (!p || !x_dev) {
        set_error("problem and x must be non-NULL");
        return MFE_EINVAL;
    }
    if (!(tol >= 0.0) || max_iter < 0) {
        set_error("tol must be >= 0 and max_iter >= 0");
        return MFE_EINVAL;
    }
    MFE_TRY(check_format(p, format));
    MFE_TRY(set_device(p->ctx));
    return cg_sr_solve(const_cast<mfe_problem *>(p), format, x_dev, tol, max_iter, hist_dev, stats);
}

int mfe_cg_jacobi(const mfe_problem *p, int format, double *x_dev, double tol, int max_iter, double *hist_dev,
                  mfe_cg_stats *stats) {
    clear_error();
    if (!p || !x_dev) {
        set_error("problem and x must be non-NULL");
        return MFE_EINVAL;
    }
    if (!(tol >= 0.0) || max_iter < 0) {
        set_error("tol must be >= 0 and max_iter >= 0");
        return MFE_EINVAL;
    }
    MFE_TRY(check_format(p, format));
    MFE_TRY(set_device(p->ctx));
    return cg_jacobi_solve(const_cast<mfe_problem *>(p), format, x_dev, tol, max_iter, hist_dev, stats);
}

int mfe_cg_warm(const mfe_problem *p, int format, double *x_dev, double tol, int max_iter, double *hist_dev,
                mfe_cg_stats *stats) {
    clear_error();
    if (!p || !x_dev) {
        set_error("problem and x must be non-NULL");
        return MFE_EINVAL;
    }
    if (!(tol >= 0.0) || max_iter < 0) {
        set_error("tol must be >= 0 and max_iter >= 0");
        return MFE_EINVAL;
    }
    MFE_TRY(check_format(p, format));
    MFE_TRY(set_device(p->ctx));
    return cg_solve(const_cast<mfe_problem *>(p), format, x_dev, tol, max_iter, hist_dev, stats, true);
}

int mfe_cg_mixed(const mfe_problem *p, int format, double *x_dev, double tol, double inner_tol, int max_outer,
                 int max_inner, mfe_cg_stats *stats) {
    clear_error();
    if (!p || !x_dev) {
        set_error("problem and x must be non-NULL");
        return MFE_EINVAL;
    }
    if (!(tol >= 0.0) || !(inner_tol > 0.0 && inner_tol < 1.0) || max_outer < 1 || max_inner < 1) {
        set_error("need tol >= 0, 0 < inner_tol < 1, max_outer >= 1, max_inner >= 1");
        return MFE_EINVAL;
    }
    MFE_TRY(check_format(p, format));
    if (!(p->precisions & MFE_F32)) {
        set_error("FP32 values were not built for this problem");
        return MFE_EUNSUPPORTED;
    }
    MFE_TRY(set_device(p->ctx));
    return cg_mixed_solve(const_cast<mfe_problem *>(p), format, x_dev, tol, inner_tol, max_outer, max_inner,
                          stats);
}

int mfe_cg_mixed_warm(const mfe_problem *p, int format, double *x_dev, double tol, double inner_tol, int max_outer,
                      int max_inner, mfe_cg_stats *stats) {
    clear_error();
    if (!p || !x_dev) {
        set_error("problem and x must be non-NULL");
        return MFE_EINVAL;
    }
    if (!(tol >= 0.0) || !(inner_tol > 0.0 && inner_tol < 1.0) || max_outer < 1 || max_inner < 1) {
        set_error("need tol >= 0, 0 < inner_tol < 1, max_outer >= 1, max_inner >= 1");
        return MFE_EINVAL;
    }
    MFE_TRY(check_format(p, format));
    if (!(p->precisions & MFE_F32)) {
        set_error("FP32 values were not built for this problem");
        return MFE_EUNSUPPORTED;
    }
    MFE_TRY(set_device(p->ctx));
    return cg_mixed_solve(const_cast<mfe_problem *>(p), format, x_dev, tol, inner_tol, max_outer, max_inner,
                          stats, true);
}

int mfe_cg_mixed_ex(const mfe_problem *p, int format, double *x_dev, double tol, double inner_tol, int max_outer,
                    int max_inner, int flags, mfe_cg_stats *stats) {
    clear_error();
    if (!p || !x_dev) {
        set_error("problem and x must be non-NULL");
        return MFE_EINVAL;
    }
    if (!(tol >= 0.0) || !(inner_tol > 0.0 && inner_tol < 1.0) || max_outer < 1 || max_inner < 1) {
        set_error("need tol >= 0, 0 < inner_tol < 1, max_outer >= 1, max_inner >= 1");
        return MFE_EINVAL;
    }
    if (flags & ~(MFE_MIXED_WARM | MFE_MIXED_KEEP_DIRECTION)) {
        set_error("unknown flags");
        return MFE_EINVAL;
    }
    MFE_TRY(check_format(p, format));
    if (!(p->precisions & MFE_F32)) {
        set_error("FP32 values were not built for this problem");
        return MFE_EUNSUPPORTED;
    }
    MFE_TRY(set_device(p->ctx));
    return cg_mixed_solve(const_cast<mfe_problem *>(p), format, x_dev, tol, inner_tol, max_outer, max_inner,
                          stats, (flags & MFE_MIXED_WARM) != 0, (flags & MFE_MIXED_KEEP_DIRECTION) != 0);
}

}  // extern "C"
