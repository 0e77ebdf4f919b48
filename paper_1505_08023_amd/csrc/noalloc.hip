// The fused product q = A p with p.q (the kernel each CG iteration runs),
// through an entry point that allocates no device memory.
//
// mfe_spmv_dot keeps its reduction partials and its solver state in memory
// the context allocated.  mfe_spmv_dot_noalloc keeps them in `scratch`, a
// statically sized device array of this library: one per GPU, loaded with
// the code object, released when the process ends.  Host code never passes
// the array's name to a kernel (on the host it names a stand-in, not device
// memory): mfe_ctx_create looks up its device address once per device and
// the entry point passes that address.
#include <mutex>

#include "common.hpp"

namespace mfe {

// Scratch layout: the per-workgroup partials of p.q (room for kMaxPartials
// workgroups), then one CgState.
constexpr size_t kNoallocPartialBytes = (size_t)kMaxPartials * sizeof(double);
constexpr size_t kNoallocStateBytes = (sizeof(CgState) + 255) / 256 * 256;
constexpr size_t kNoallocBytes = kNoallocPartialBytes + kNoallocStateBytes;
static_assert(kNoallocBytes == 33024, "the size mfe.h states for mfe_spmv_dot_noalloc");

}  // namespace mfe

static __device__ __align__(256) unsigned char scratch[mfe::kNoallocBytes];

namespace mfe {
namespace {

constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
void *g_scratch_dev[kMaxDevices] = {};

}  // namespace

// Called by mfe_ctx_create with `device` current: the device address of this
// device's copy of `scratch`, looked up once per device.
int noalloc_init(int device) {
    if (device < 0 || device >= kMaxDevices) {
        set_error("device index beyond the library's table of " + std::to_string(kMaxDevices) + " devices");
        return MFE_EUNSUPPORTED;
    }
    std::lock_guard<std::mutex> lock(g_scratch_mu);
    if (g_scratch_dev[device]) return MFE_OK;
    void *ptr = nullptr;
    const hipError_t e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
    if (e != hipSuccess || !ptr) {
        set_error(std::string("hipGetSymbolAddress of the static scratch failed: ") + hipGetErrorString(e));
        return MFE_EHIP;
    }
    g_scratch_dev[device] = ptr;
    return MFE_OK;
}

namespace {

void *scratch_of(int device) {
    if (device < 0 || device >= kMaxDevices) return nullptr;
    std::lock_guard<std::mutex> lock(g_scratch_mu);
    return g_scratch_dev[device];
}

}  // namespace
}  // namespace mfe

using namespace mfe;

extern "C" int mfe_spmv_dot_noalloc(const mfe_problem *p, int format, const double *p_dev, double *q_dev,
                                    double *pq_dev) {
    clear_error();
    if (!p || !p_dev || !q_dev || !pq_dev) {
        set_error("problem, p, q and pq must be non-NULL");
        return MFE_EINVAL;
    }
    if (format != MFE_CSR && format != MFE_BCRS13) {
        set_error("format must be MFE_CSR or MFE_BCRS13");
        return MFE_EINVAL;
    }
    if (!(p->formats & format)) {
        set_error("format was not built for this problem");
        return MFE_EUNSUPPORTED;
    }
    mfe_ctx *ctx = p->ctx;
    MFE_HIP_TRY(hipSetDevice(ctx->device));
    unsigned char *base = (unsigned char *)scratch_of(ctx->device);
    if (!base) {
        set_error("the static scratch of this device was not set up (no context was created on it)");
        return MFE_EINVAL;
    }
    double *partials = (double *)base;
    CgState *st = (CgState *)(base + kNoallocPartialBytes);
    // every field the product and the finalizer read is set here: a running
    // state with rho = 1 whose finalizer publishes p.q to pq_dev
    MFE_TRY(launch_state_reset(st, pq_dev, ctx->stream));
    SpmvArgs a{p_dev, q_dev, nullptr, nullptr, st, partials};
    a.max_partials = kMaxPartials;
    int n = 0;
    MFE_TRY(launch_spmv(p, format, false, kSpmvDot, a, ctx->stream, &n));
    return launch_finalize(kFinDot, partials, n, st, ctx->stream);
}
