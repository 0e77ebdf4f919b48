// CRS -> fixed 1x3 BCRS conversion (Sec. 3.1: the matrix is converted at the
// start of CG; CRS stays the assembly format) and FP32 value copies.
//
// The paper's BCRS stores 1xn segments of variable length n with an offsets
// array and unrolls the segment loop with a switch on n (Figs 3.2, 3.3).  On
// a GPU the switch becomes divergence, so the segment length is fixed to 3
// (the length of almost every segment of this matrix) and shorter segments
// are zero padded: no offsets array, no branch.  Rows are grouped in slices
// of 64 (one wavefront); inside a slice the k-th block of every row is stored
// contiguously, so each block load of a wavefront is one coalesced access
// (layout in b13_layout.hpp).
#include <algorithm>
#include <vector>

#include "b13_layout.hpp"
#include "common.hpp"
#include "device_util.hpp"

namespace mfe {
namespace {

// Greedy 1x3 blocking of one CRS row: a block starts at the first stored
// column not yet covered (moved back to m-3 near the end of the matrix) and
// covers c, c+1, c+2.  Calls f(block, c, slot values) for every block.
template <typename F>
__device__ __forceinline__ int row_blocks(const int32_t *col, const double *val, int32_t lo, int32_t hi,
                                          int64_t m, F f) {
    int nb = 0;
    int32_t k = lo;
    while (k < hi) {
        int64_t c = col[k];
        if (c > m - 3) c = m - 3;
        double v[3] = {0.0, 0.0, 0.0};
        while (k < hi && col[k] <= c + 2) {
            if (val) v[col[k] - c] = val[k];
            ++k;
        }
        f(nb, (int32_t)c, v);
        ++nb;
    }
    return nb;
}

// One 64-thread workgroup per slice.  The slice's CRS runs, contiguous in
// the CRS arrays, are first copied to LDS with coalesced loads (a thread per
// row then walks its row in LDS instead of issuing loads 27 entries apart
// from its neighbours'); a slice with more than kConvCap entries reads
// global memory directly.
constexpr int kConvCap = 64 * 28;

// Blocks per row, and per slice the maximum over its 64 rows.
__global__ __launch_bounds__(64) void k_b13_count(int64_t m, const int32_t *__restrict__ ptr,
                                                  const int32_t *__restrict__ col,
                                                  int32_t *__restrict__ rowblocks,
                                                  int32_t *__restrict__ slice_n) {
    __shared__ int32_t sc[kConvCap];
    const int64_t s = blockIdx.x;
    const int64_t i = s * 64 + threadIdx.x;
    const int64_t r1 = s * 64 + 64 < m ? s * 64 + 64 : m;
    const int32_t tlo = ptr[s * 64], thi = ptr[r1];
    const bool staged = thi - tlo <= kConvCap;
    if (staged)
        for (int32_t j = tlo + (int32_t)threadIdx.x; j < thi; j += 64) sc[j - tlo] = col[j];
    __syncthreads();
    int nb = 0;
    if (i < m) {
        auto none = [](int, int32_t, const double *) {};
        nb = staged ? row_blocks(sc, nullptr, ptr[i] - tlo, ptr[i + 1] - tlo, m, none)
                    : row_blocks(col, nullptr, ptr[i], ptr[i + 1], m, none);
        rowblocks[i] = nb;
    }
    int mx = nb;
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) mx = max(mx, __shfl_xor(mx, off, 64));
    if (threadIdx.x == 0) slice_n[s] = mx;
}

// Exclusive prefix sum of n int32 counts into out[0..n] (out[n] = total),
// by a single workgroup of 1024 threads: each thread scans a contiguous
// chunk, the chunk totals are scanned in LDS, then each chunk is written.
// scale multiplies every count (e.g. rows per slice).
__global__ __launch_bounds__(1024) void k_scan1(int64_t n, const int32_t *__restrict__ in,
                                                int32_t *__restrict__ out, int scale,
                                                int64_t *__restrict__ total) {
    __shared__ int64_t sums[1024];
    const int t = threadIdx.x;
    const int64_t chunk = (n + 1023) / 1024;
    const int64_t lo = min(n, t * chunk), hi = min(n, lo + chunk);
    int64_t s = 0;
    for (int64_t i = lo; i < hi; ++i) s += (int64_t)in[i] * scale;
    sums[t] = s;
    __syncthreads();
    if (t == 0) {
        int64_t acc = 0;
        for (int j = 0; j < 1024; ++j) {
            int64_t v = sums[j];
            sums[j] = acc;
            acc += v;
        }
        out[n] = (int32_t)acc;
        *total = acc;
    }
    __syncthreads();
    int64_t acc = sums[t];
    for (int64_t i = lo; i < hi; ++i) {
        out[i] = (int32_t)acc;
        acc += (int64_t)in[i] * scale;
    }
}

// Multi-workgroup exclusive scan of int32 counts: chunks of kScanChunk
// elements, 8 consecutive ones per thread of a 1024-thread workgroup.
// Phase 1 writes each chunk's total, k_scan1 scans the chunk totals, phase 2
// scans inside each chunk from its offset.  Sums are formed in int64.
constexpr int kScanThreads = 1024, kScanPer = 8, kScanChunk = kScanThreads * kScanPer;

// Exclusive scan of one value per thread over the workgroup; *sum receives
// the workgroup total (every thread).
__device__ __forceinline__ int64_t wg_exclusive_scan(int64_t v, int64_t *sum) {
    __shared__ int64_t wsum[kScanThreads / 64 + 1];
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
    int64_t x = v;
#pragma unroll
    for (int off = 1; off < 64; off <<= 1) {
        const int64_t y = __shfl_up(x, off, 64);
        if (lane >= off) x += y;
    }
    if (lane == 63) wsum[w] = x;
    __syncthreads();
    if (threadIdx.x == 0) {
        int64_t acc = 0;
        for (int k = 0; k < kScanThreads / 64; ++k) {
            const int64_t t = wsum[k];
            wsum[k] = acc;
            acc += t;
        }
        wsum[kScanThreads / 64] = acc;
    }
    __syncthreads();
    *sum = wsum[kScanThreads / 64];
    return wsum[w] + x - v;
}

__global__ __launch_bounds__(kScanThreads) void k_scan_chunks(int64_t n, const int32_t *__restrict__ in,
                                                              int32_t *__restrict__ chunk_sum) {
    const int64_t lo = (int64_t)blockIdx.x * kScanChunk + (int64_t)threadIdx.x * kScanPer;
    int64_t v = 0;
    for (int j = 0; j < kScanPer; ++j)
        if (lo + j < n) v += in[lo + j];
    int64_t total;
    (void)wg_exclusive_scan(v, &total);
    if (threadIdx.x == 0) chunk_sum[blockIdx.x] = (int32_t)total;
}

__global__ __launch_bounds__(kScanThreads) void k_scan_apply(int64_t n, const int32_t *__restrict__ in,
                                                             const int32_t *__restrict__ chunk_off,
                                                             int32_t *__restrict__ out) {
    const int64_t lo = (int64_t)blockIdx.x * kScanChunk + (int64_t)threadIdx.x * kScanPer;
    int32_t vals[kScanPer];
    int64_t v = 0;
    for (int j = 0; j < kScanPer; ++j) {
        vals[j] = lo + j < n ? in[lo + j] : 0;
        v += vals[j];
    }
    int64_t total;
    int64_t acc = chunk_off[blockIdx.x] + wg_exclusive_scan(v, &total);
    for (int j = 0; j < kScanPer; ++j)
        if (lo + j < n) {
            out[lo + j] = (int32_t)acc;
            acc += vals[j];
        }
}

// Write every row's blocks into its slice; pad up to the slice's slot count
// with zero blocks that point at the row's last block column (a valid index
// whose x entries are already in cache).
template <typename T>
__global__ __launch_bounds__(64) void k_b13_fill(int64_t m, const int32_t *__restrict__ ptr,
                                                 const int32_t *__restrict__ col,
                                                 const double *__restrict__ val,
                                                 const int32_t *__restrict__ slot_base,
                                                 int32_t *__restrict__ jas, T *__restrict__ bval) {
    __shared__ int32_t sc[kConvCap];
    __shared__ double sv[kConvCap];
    const int64_t s = blockIdx.x;
    const int lane = (int)threadIdx.x;
    const int64_t i = s * 64 + lane;
    const int64_t r1 = s * 64 + 64 < m ? s * 64 + 64 : m;
    const int32_t tlo = ptr[s * 64], thi = ptr[r1];
    const bool staged = thi - tlo <= kConvCap;
    if (staged)
        for (int32_t j = tlo + lane; j < thi; j += 64) {
            sc[j - tlo] = col[j];
            sv[j - tlo] = val[j];
        }
    __syncthreads();
    const B13Slice sl = b13_slice(slot_base[s], slot_base[s + 1]);
    int32_t last_c = 0;
    int nb = 0;
    if (i < m) {
        auto put = [&](int blk, int32_t c, const double *v) {
            jas[b13_jas(sl, blk, lane)] = c;
            for (int j = 0; j < 3; ++j) bval[b13_val(sl, blk, j, lane)] = (T)v[j];
            last_c = c;
        };
        nb = staged ? row_blocks(sc, sv, ptr[i] - tlo, ptr[i + 1] - tlo, m, put)
                    : row_blocks(col, val, ptr[i], ptr[i + 1], m, put);
    }
    // pad up to the slice's slot count with zero blocks that point at the
    // row's last block column (a valid index whose x entries are in cache)
    for (int k = nb; k < sl.S; ++k) {
        jas[b13_jas(sl, k, lane)] = last_c;
        for (int j = 0; j < 3; ++j) bval[b13_val(sl, k, j, lane)] = (T)0;
    }
}

// Slice descriptors (B13Desc): one 64-thread workgroup per slice.  Only
// full 9-slot slices are candidates.  d[0] is the smallest offset of slot 0
// over the lanes, e_l a lane's excess over it; the slice is uniform when
// every e_l is 0 or 1 and, for each slot, column - row - e_l is one value
// over the lanes.  cnt[s] receives the slice's real blocks when uniform
// (else 0) and flag[s] whether it is.
__device__ __forceinline__ int32_t wave_min_i(int32_t v) {
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) v = min(v, __shfl_xor(v, off, 64));
    return v;
}
__device__ __forceinline__ int32_t wave_max_i(int32_t v) {
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) v = max(v, __shfl_xor(v, off, 64));
    return v;
}
__device__ __forceinline__ int32_t wave_sum_i(int32_t v) {
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, 64);
    return v;
}

__global__ __launch_bounds__(64) void k_b13_desc(int64_t m, const int32_t *__restrict__ slot_base,
                                                 const int32_t *__restrict__ jas,
                                                 const int32_t *__restrict__ rowblocks, B13Desc *__restrict__ desc,
                                                 int32_t *__restrict__ cnt, int32_t *__restrict__ flag) {
    const int64_t s = blockIdx.x;
    const int lane = (int)threadIdx.x;
    const B13Slice sl = b13_slice(slot_base[s], slot_base[s + 1]);
    B13Desc D{};
    int uniform = 0, blocks = 0;
    if (sl.S == 9 && s * 64 + 64 <= m) {  // wavefront-uniform condition
        const int64_t row = s * 64 + lane;
        int32_t c[9];
#pragma unroll
        for (int k = 0; k < 9; ++k) c[k] = jas[b13_jas(sl, k, lane)];
        const int32_t d0 = (int32_t)(c[0] - row);  // |column - row| < m < 2^31
        const int32_t base = wave_min_i(d0);
        const int32_t e = d0 - base;
        bool ok = e == 0 || e == 1;
        D.d[0] = base;
#pragma unroll
        for (int k = 1; k < 9; ++k) {
            const int32_t t = (int32_t)(c[k] - row) - e;
            const int32_t lo = wave_min_i(t), hi = wave_max_i(t);
            ok = ok && lo == hi;
            D.d[k] = lo;
        }
        uniform = __all(ok) ? 1 : 0;
        const uint64_t bits = __ballot(e == 1);
        D.e_lo = (uint32_t)bits;
        D.e_hi = (uint32_t)(bits >> 32);
        D.uniform = uniform;
        blocks = wave_sum_i(rowblocks[row]);
    }
    if (lane == 0) {
        desc[s] = D;
        cnt[s] = uniform ? blocks : 0;
        flag[s] = uniform;
    }
}

// CRS tile descriptors (CsrDesc): one 64-thread workgroup per wavefront
// tile of kCsrsRows rows.  A full tile is uniform when each of its rows holds
// 27 entries and every column minus its row equals that of the tile's first
// row at the same entry.  flag[t] receives whether it is.
__global__ __launch_bounds__(64) void k_csr_desc(int64_t m, const int32_t *__restrict__ ptr,
                                                 const int32_t *__restrict__ col, CsrDesc *__restrict__ desc,
                                                 int32_t *__restrict__ flag) {
    const int64_t t = blockIdx.x;
    const int lane = (int)threadIdx.x;
    const int64_t r0 = t * kCsrsRows;
    // workgroup-uniform: a full tile of 27 kCsrsRows entries (checked before
    // any column is read, so the reads stay inside the tile's run)
    bool ok = r0 + kCsrsRows <= m;
    int32_t lo = 0;
    if (ok) {
        lo = ptr[r0];
        ok = ptr[r0 + kCsrsRows] - lo == 27 * kCsrsRows;
    }
    if (ok) {
        bool mine = true;
        if (lane < kCsrsRows) mine = ptr[r0 + lane + 1] - ptr[r0 + lane] == 27;
        for (int j = lane; j < 27 * kCsrsRows; j += 64) {
            const int64_t row = r0 + j / 27;
            mine = mine && (int64_t)col[lo + j] - row == (int64_t)col[lo + j % 27] - r0;
        }
        ok = __all(mine);
    }
    if (ok && lane < 27) desc[t].off[lane] = (int32_t)(col[lo + lane] - r0);
    if (lane == 0) {
        bool runs3 = ok;
        for (int i = 0; runs3 && i < 9; ++i)
            runs3 = col[lo + 3 * i + 1] == col[lo + 3 * i] + 1 && col[lo + 3 * i + 2] == col[lo + 3 * i] + 2;
        desc[t].uniform = ok ? (runs3 ? 2 : 1) : 0;
        flag[t] = ok ? 1 : 0;
    }
}

// FP32 copy of the 1x3 BCRS values: 9-slot slices into the packed layout
// (b13_val32_9), the others element by element.  One thread per (slice, lane).
__global__ __launch_bounds__(kBlock) void k_b13_cast_f32(int64_t nslices, const int32_t *__restrict__ slot_base,
                                                         const double *__restrict__ v64, float *__restrict__ v32) {
    const int64_t t = (int64_t)blockIdx.x * kBlock + threadIdx.x;
    const int64_t s = t >> 6;
    const int lane = (int)(t & 63);
    if (s >= nslices) return;
    const B13Slice sl = b13_slice(slot_base[s], slot_base[s + 1]);
    if (sl.S == 9) {
        for (int v = 0; v < 27; ++v) v32[b13_val32_9(sl, v, lane)] = (float)v64[b13_val(sl, v / 3, v % 3, lane)];
    } else {
        for (int k = 0; k < sl.S; ++k)
            for (int j = 0; j < 3; ++j) v32[b13_val(sl, k, j, lane)] = (float)v64[b13_val(sl, k, j, lane)];
    }
}

__global__ __launch_bounds__(kBlock) void k_cast_f32(int64_t n, const double *__restrict__ in,
                                                     float *__restrict__ out) {
    for (int64_t i = (int64_t)blockIdx.x * kBlock + threadIdx.x; i < n; i += (int64_t)gridDim.x * kBlock)
        out[i] = (float)in[i];
}

// Per-row block lists out of the slice layout (for inspection and tests).
__global__ __launch_bounds__(kBlock) void k_b13_export(int64_t m, const int32_t *__restrict__ slot_base,
                                                       const int32_t *__restrict__ rowblocks,
                                                       const int32_t *__restrict__ bptr,
                                                       const int32_t *__restrict__ jas,
                                                       const double *__restrict__ bv,
                                                       int32_t *__restrict__ bcol,
                                                       double *__restrict__ bval) {
    const int64_t i = (int64_t)blockIdx.x * kBlock + threadIdx.x;
    if (i >= m) return;
    const int64_t s = i >> 6;
    const int lane = (int)(i & 63);
    const B13Slice sl = b13_slice(slot_base[s], slot_base[s + 1]);
    for (int blk = 0; blk < rowblocks[i]; ++blk) {
        const int64_t o = bptr[i] + blk;
        if (bcol) bcol[o] = jas[b13_jas(sl, blk, lane)];
        if (bval)
            for (int j = 0; j < 3; ++j) bval[3 * o + j] = bv[b13_val(sl, blk, j, lane)];
    }
}

// Structure check of a caller-supplied CRS: ptr[0] = 0, ptr non-decreasing,
// ptr[m] = nnz, columns strictly ascending within a row and inside [0, m).
// Any violation sets *bad.
__global__ __launch_bounds__(kBlock) void k_validate_csr(int64_t m, int64_t nnz, const int32_t *__restrict__ ptr,
                                                         const int32_t *__restrict__ col, int *bad) {
    const int64_t i = (int64_t)blockIdx.x * kBlock + threadIdx.x;
    if (i >= m) return;
    const int64_t lo = ptr[i], hi = ptr[i + 1];
    bool ok = lo >= 0 && lo <= hi && hi <= nnz && (i != 0 || lo == 0) && (i != m - 1 || hi == nnz);
    for (int64_t k = lo; ok && k < hi; ++k) {
        const int32_t c = col[k];
        ok = c >= 0 && c < m && (k == lo || c > col[k - 1]);
    }
    if (!ok) atomicOr(bad, 1);
}

// flag[i] = 1 when row i holds 27 entries with column i + off[k] (k-th entry).
// One 64-thread workgroup per 64 rows: their column run is staged in LDS
// with coalesced loads (a run longer than 27 per row is read in place).
struct CsrOffsets {
    int32_t off[27];
};
__global__ __launch_bounds__(64) void k_csr_fullflag(int64_t m, const int32_t *__restrict__ ptr,
                                                     const int32_t *__restrict__ col, CsrOffsets O,
                                                     int32_t *__restrict__ flag) {
    __shared__ int32_t sc[64 * 27];
    const int64_t r0 = (int64_t)blockIdx.x * 64;
    const int lane = (int)threadIdx.x;
    const int64_t r1 = r0 + 64 < m ? r0 + 64 : m;
    const int32_t lo = ptr[r0], hi = ptr[r1];
    const bool staged = hi - lo <= 64 * 27;
    if (staged)
        for (int32_t j = lane; j < hi - lo; j += 64) sc[j] = col[lo + j];
    __syncthreads();
    const int64_t i = r0 + lane;
    if (i >= m) return;
    const int32_t a = ptr[i] - lo;
    bool ok = ptr[i + 1] - lo - a == 27;
    for (int k = 0; ok && k < 27; ++k)
        ok = (int64_t)(staged ? sc[a + k] : col[lo + a + k]) - i == (int64_t)O.off[k];
    flag[i] = ok ? 1 : 0;
}

// chg[i] = 1 where the flag changes between rows i - 1 and i (i = 0..m, with
// the flag taken as 0 outside the matrix): run starts and run ends alternate.
__global__ __launch_bounds__(kBlock) void k_flag_changes(int64_t m, const int32_t *__restrict__ flag,
                                                         int32_t *__restrict__ chg) {
    const int64_t i = (int64_t)blockIdx.x * kBlock + threadIdx.x;
    if (i > m) return;
    const int32_t cur = i < m ? flag[i] : 0, prev = i > 0 ? flag[i - 1] : 0;
    chg[i] = cur != prev ? 1 : 0;
}

// out[pos[i]] = i for every i with chg[i] set.
__global__ __launch_bounds__(kBlock) void k_compact_rows(int64_t n, const int32_t *__restrict__ chg,
                                                         const int32_t *__restrict__ pos, int32_t *__restrict__ out) {
    const int64_t i = (int64_t)blockIdx.x * kBlock + threadIdx.x;
    if (i < n && chg[i]) out[pos[i]] = (int32_t)i;
}

}  // namespace

int validate_csr(mfe_ctx *ctx, int64_t m, int64_t nnz, const int32_t *ptr, const int32_t *col) {
    TempBuffer bad(ctx);
    MFE_TRY(bad.alloc(sizeof(int)));
    MFE_HIP_TRY(hipMemsetAsync(bad.ptr(), 0, sizeof(int), ctx->stream));
    hipLaunchKernelGGL(k_validate_csr, dim3((unsigned)((m + kBlock - 1) / kBlock)), dim3(kBlock), 0,
                       ctx->stream, m, nnz, ptr, col, (int *)bad.ptr());
    MFE_HIP_TRY(hipGetLastError());
    int h = 0;
    MFE_HIP_TRY(hipMemcpyAsync(&h, bad.ptr(), sizeof(int), hipMemcpyDeviceToHost, ctx->stream));
    MFE_HIP_TRY(hipStreamSynchronize(ctx->stream));
    if (h) {
        set_error("CRS structure invalid: ptr must rise from 0 to nnz and columns ascend inside [0, m)");
        return MFE_EINVAL;
    }
    return MFE_OK;
}

// Exclusive scan of n >= 1 counts into out[0..n] (out may be NULL: total
// only) on the context's stream; *total_dev (device int64) receives the sum.
// The sum must fit int32.
int scan_counts(mfe_ctx *ctx, int64_t n, const int32_t *in, int32_t *out, int64_t *total_dev) {
    hipStream_t s = ctx->stream;
    const int64_t nchunks = (n + kScanChunk - 1) / kScanChunk;
    TempBuffer tmp(ctx);
    MFE_TRY(tmp.alloc((size_t)(2 * nchunks + 1) * sizeof(int32_t)));
    int32_t *csum = (int32_t *)tmp.ptr(), *coff = csum + nchunks;
    hipLaunchKernelGGL(k_scan_chunks, dim3((unsigned)nchunks), dim3(kScanThreads), 0, s, n, in, csum);
    hipLaunchKernelGGL(k_scan1, dim3(1), dim3(1024), 0, s, nchunks, (const int32_t *)csum, coff, 1, total_dev);
    if (out) {
        hipLaunchKernelGGL(k_scan_apply, dim3((unsigned)nchunks), dim3(kScanThreads), 0, s, n, in,
                           (const int32_t *)coff, out);
        // out[n] = total
        MFE_HIP_TRY(hipMemcpyAsync(out + n, coff + nchunks, sizeof(int32_t), hipMemcpyDeviceToDevice, s));
    }
    const hipError_t e = hipGetLastError();
    MFE_HIP_TRY(hipStreamSynchronize(s));
    if (e != hipSuccess) {
        set_error(std::string("scan launch failed: ") + hipGetErrorString(e));
        return MFE_EHIP;
    }
    return MFE_OK;
}

int build_csr_tiles(mfe_problem *P) {
    mfe_ctx *ctx = P->ctx;
    hipStream_t s = ctx->stream;
    const int64_t ntiles = (P->m + kCsrsRows - 1) / kCsrsRows;
    if (ntiles == 0) return MFE_OK;
    TempBuffer flag(ctx), total(ctx);
    MFE_TRY(dev_alloc(ctx, &P->cdesc, (size_t)ntiles * sizeof(CsrDesc)));
    MFE_TRY(flag.alloc((size_t)ntiles * sizeof(int32_t)));
    MFE_TRY(total.alloc(sizeof(int64_t)));
    hipLaunchKernelGGL(k_csr_desc, dim3((unsigned)ntiles), dim3(64), 0, s, P->m, (const int32_t *)P->ptr.ptr,
                       (const int32_t *)P->col.ptr, (CsrDesc *)P->cdesc.ptr, (int32_t *)flag.ptr());
    MFE_HIP_TRY(hipGetLastError());
    MFE_TRY(scan_counts(ctx, ntiles, (const int32_t *)flag.ptr(), nullptr, (int64_t *)total.ptr()));
    int64_t n = 0;
    MFE_HIP_TRY(hipMemcpyAsync(&n, total.ptr(), sizeof(int64_t), hipMemcpyDeviceToHost, s));
    MFE_HIP_TRY(hipStreamSynchronize(s));
    P->csr_ctiles = n;
    return MFE_OK;
}

// Work items of the CRS group walk of a mesh problem (see CsrRuns): full
// rows are flagged on the device, the run boundaries compacted and copied
// to the host, and the items built there in row order: each run of full rows
// cut into groups of at most 64, the rows between runs gathered into tiles
// of at most 16, a tile emitted when full (or at the end).
int build_csr_groups(mfe_problem *P) {
    P->ncitems = P->ncrows = P->ncgroups = P->ncgroup_rows = 0;
    if (!MFE_CSR_GROUPS || !P->is_mesh || P->Nx < 2 || P->Ny < 2 || P->Nz < 2) return MFE_OK;
    mfe_ctx *ctx = P->ctx;
    hipStream_t s = ctx->stream;
    const int64_t m = P->m, nx = P->Nx + 1, nxy = nx * (P->Ny + 1);
    CsrOffsets O{};
    int k = 0;
    for (int dz = -1; dz <= 1; ++dz)
        for (int dy = -1; dy <= 1; ++dy)
            for (int dx = -1; dx <= 1; ++dx) O.off[k++] = (int32_t)(dx + nx * dy + nxy * dz);
    for (int i = 0; i < 9; ++i) P->cruns.r[i] = O.off[3 * i];
    TempBuffer flag(ctx), chg(ctx), pos(ctx), total(ctx), edges(ctx);
    MFE_TRY(flag.alloc((size_t)m * sizeof(int32_t)));
    MFE_TRY(chg.alloc((size_t)(m + 1) * sizeof(int32_t)));
    MFE_TRY(pos.alloc((size_t)(m + 2) * sizeof(int32_t)));
    MFE_TRY(total.alloc(sizeof(int64_t)));
    const unsigned g1 = (unsigned)((m + 1 + kBlock - 1) / kBlock);
    hipLaunchKernelGGL(k_csr_fullflag, dim3((unsigned)((m + 63) / 64)), dim3(64), 0, s, m,
                       (const int32_t *)P->ptr.ptr, (const int32_t *)P->col.ptr, O, (int32_t *)flag.ptr());
    hipLaunchKernelGGL(k_flag_changes, dim3(g1), dim3(kBlock), 0, s, m, (const int32_t *)flag.ptr(),
                       (int32_t *)chg.ptr());
    MFE_HIP_TRY(hipGetLastError());
    MFE_TRY(scan_counts(ctx, m + 1, (const int32_t *)chg.ptr(), (int32_t *)pos.ptr(), (int64_t *)total.ptr()));
    int64_t nchg = 0;
    MFE_HIP_TRY(hipMemcpyAsync(&nchg, total.ptr(), sizeof(int64_t), hipMemcpyDeviceToHost, s));
    MFE_HIP_TRY(hipStreamSynchronize(s));
    if (nchg == 0) return MFE_OK;  // no full rows
    MFE_TRY(edges.alloc((size_t)nchg * sizeof(int32_t)));
    hipLaunchKernelGGL(k_compact_rows, dim3(g1), dim3(kBlock), 0, s, m + 1, (const int32_t *)chg.ptr(),
                       (const int32_t *)pos.ptr(), (int32_t *)edges.ptr());
    MFE_HIP_TRY(hipGetLastError());
    std::vector<int32_t> e((size_t)nchg);
    MFE_HIP_TRY(hipMemcpyAsync(e.data(), edges.ptr(), nchg * sizeof(int32_t), hipMemcpyDeviceToHost, s));
    MFE_HIP_TRY(hipStreamSynchronize(s));
    if (nchg % 2 != 0) {
        set_error("internal: unpaired run boundaries of the CRS row groups");
        return MFE_EINVAL;
    }
    std::vector<int32_t> items, rows;  // items as (a, b) pairs
    std::vector<int32_t> pending;
    auto flush = [&](bool all) {
        size_t at = 0;
        while (pending.size() - at >= 16 || (all && at < pending.size())) {
            const int n = (int)std::min<size_t>(16, pending.size() - at);
            items.push_back((int32_t)rows.size());
            items.push_back(-n);
            rows.insert(rows.end(), pending.begin() + (long)at, pending.begin() + (long)at + n);
            at += (size_t)n;
        }
        pending.erase(pending.begin(), pending.begin() + (long)at);
    };
    int64_t prev_end = 0, ngroups = 0, grows = 0;
    for (int64_t j = 0; j < nchg; j += 2) {
        const int64_t rs = e[(size_t)j], re = e[(size_t)j + 1];
        for (int64_t r = prev_end; r < rs; ++r) pending.push_back((int32_t)r);
        flush(false);
        for (int64_t r = rs; r < re; r += 64) {
            items.push_back((int32_t)r);
            items.push_back((int32_t)std::min<int64_t>(64, re - r));
            ++ngroups;
        }
        grows += re - rs;
        prev_end = re;
    }
    for (int64_t r = prev_end; r < m; ++r) pending.push_back((int32_t)r);
    flush(true);
    MFE_TRY(dev_alloc(ctx, &P->citems, items.size() * sizeof(int32_t)));
    MFE_TRY(dev_alloc(ctx, &P->crows, std::max<size_t>(rows.size(), 1) * sizeof(int32_t)));
    MFE_HIP_TRY(hipMemcpyAsync(P->citems.ptr, items.data(), items.size() * sizeof(int32_t), hipMemcpyHostToDevice, s));
    if (!rows.empty())
        MFE_HIP_TRY(hipMemcpyAsync(P->crows.ptr, rows.data(), rows.size() * sizeof(int32_t), hipMemcpyHostToDevice, s));
    MFE_HIP_TRY(hipStreamSynchronize(s));
    P->ncitems = (int64_t)items.size() / 2;
    P->ncrows = (int64_t)rows.size();
    P->ncgroups = ngroups;
    P->ncgroup_rows = grows;
    return MFE_OK;
}

int build_bcrs13(mfe_problem *P) {
    mfe_ctx *ctx = P->ctx;
    hipStream_t s = ctx->stream;
    const int64_t m = P->m;
    if (m < 3) {
        set_error("1x3 BCRS needs at least 3 rows");
        return MFE_EUNSUPPORTED;
    }
    const int64_t nslices = (m + 63) / 64;
    TempBuffer slice_buf(ctx), total_buf(ctx), cnt_buf(ctx);
    MFE_TRY(dev_alloc(ctx, &P->rowblocks, (size_t)m * sizeof(int32_t)));
    MFE_TRY(slice_buf.alloc((size_t)nslices * sizeof(int32_t)));
    MFE_TRY(dev_alloc(ctx, &P->slot_base, (size_t)(nslices + 1) * sizeof(int32_t)));
    MFE_TRY(total_buf.alloc(2 * sizeof(int64_t)));
    int32_t *slice_n = (int32_t *)slice_buf.ptr();
    int64_t *total = (int64_t *)total_buf.ptr();
    const unsigned grid = (unsigned)nslices;  // one 64-thread workgroup per slice
    hipLaunchKernelGGL(k_b13_count, dim3(grid), dim3(64), 0, s, m, (const int32_t *)P->ptr.ptr,
                       (const int32_t *)P->col.ptr, (int32_t *)P->rowblocks.ptr, slice_n);
    MFE_HIP_TRY(hipGetLastError());
    // slot rows per slice -> slot_base; the same counts x 1 give the total slot rows
    MFE_TRY(scan_counts(ctx, nslices, slice_n, (int32_t *)P->slot_base.ptr, total));
    int64_t nslots = 0;
    MFE_HIP_TRY(hipMemcpyAsync(&nslots, total, sizeof(int64_t), hipMemcpyDeviceToHost, s));
    MFE_HIP_TRY(hipStreamSynchronize(s));
    if (nslots * 64 * 3 >= ((int64_t)1 << 31)) {
        set_error("1x3 BCRS slot count exceeds 32-bit indexing");
        return MFE_EUNSUPPORTED;
    }
    P->nslots = nslots;
    MFE_TRY(dev_alloc(ctx, &P->jas, (size_t)nslots * 64 * sizeof(int32_t)));
    MFE_TRY(dev_alloc(ctx, &P->bval64, (size_t)nslots * 64 * 3 * sizeof(double)));
    hipLaunchKernelGGL(k_b13_fill<double>, dim3(grid), dim3(64), 0, s, m, (const int32_t *)P->ptr.ptr,
                       (const int32_t *)P->col.ptr, (const double *)P->val64.ptr,
                       (const int32_t *)P->slot_base.ptr, (int32_t *)P->jas.ptr, (double *)P->bval64.ptr);
    MFE_HIP_TRY(hipGetLastError());
    // number of real (unpadded) blocks: the sum of the per-row counts
    MFE_TRY(scan_counts(ctx, m, (const int32_t *)P->rowblocks.ptr, nullptr, total + 1));
    int64_t nb = 0;
    MFE_HIP_TRY(hipMemcpyAsync(&nb, total + 1, sizeof(int64_t), hipMemcpyDeviceToHost, s));
    MFE_HIP_TRY(hipStreamSynchronize(s));
    P->nblocks = nb;
    // slice descriptors; slice_n is reused for the per-slice flags
    MFE_TRY(dev_alloc(ctx, &P->bdesc, (size_t)nslices * sizeof(B13Desc)));
    MFE_TRY(cnt_buf.alloc((size_t)nslices * sizeof(int32_t)));
    int32_t *cnt = (int32_t *)cnt_buf.ptr();
    hipLaunchKernelGGL(k_b13_desc, dim3(grid), dim3(64), 0, s, m, (const int32_t *)P->slot_base.ptr,
                       (const int32_t *)P->jas.ptr, (const int32_t *)P->rowblocks.ptr, (B13Desc *)P->bdesc.ptr,
                       cnt, slice_n);
    MFE_HIP_TRY(hipGetLastError());
    MFE_TRY(scan_counts(ctx, nslices, slice_n, nullptr, total));
    MFE_TRY(scan_counts(ctx, nslices, cnt, nullptr, total + 1));
    int64_t counts[2] = {0, 0};
    MFE_HIP_TRY(hipMemcpyAsync(counts, total, 2 * sizeof(int64_t), hipMemcpyDeviceToHost, s));
    MFE_HIP_TRY(hipStreamSynchronize(s));
    P->b13_cslices = counts[0];
    P->b13_cblocks = counts[1];
    return MFE_OK;
}

int cast_values_f32(mfe_problem *P) {
    mfe_ctx *ctx = P->ctx;
    hipStream_t s = ctx->stream;
    MFE_TRY(dev_alloc(ctx, &P->val32, (size_t)P->nnz * sizeof(float)));
    hipLaunchKernelGGL(k_cast_f32, dim3(4096), dim3(kBlock), 0, s, P->nnz, (const double *)P->val64.ptr,
                       (float *)P->val32.ptr);
    MFE_HIP_TRY(hipGetLastError());
    if (P->formats & MFE_BCRS13) {
        const int64_t n = P->nslots * 64 * 3;
        MFE_TRY(dev_alloc(ctx, &P->bval32, (size_t)n * sizeof(float)));
        const int64_t nslices = (P->m + 63) / 64;
        hipLaunchKernelGGL(k_b13_cast_f32, dim3((unsigned)((nslices * 64 + kBlock - 1) / kBlock)), dim3(kBlock), 0, s,
                           nslices, (const int32_t *)P->slot_base.ptr, (const double *)P->bval64.ptr,
                           (float *)P->bval32.ptr);
        MFE_HIP_TRY(hipGetLastError());
    }
    return MFE_OK;
}

int export_bcrs13(const mfe_problem *P, int32_t *bptr_out, int32_t *bcol, double *bval) {
    mfe_ctx *ctx = P->ctx;
    hipStream_t s = ctx->stream;
    const int64_t m = P->m;
    TempBuffer bptr_buf(ctx), total_buf(ctx);
    MFE_TRY(bptr_buf.alloc((size_t)(m + 1) * sizeof(int32_t)));
    MFE_TRY(total_buf.alloc(sizeof(int64_t)));
    int32_t *bptr = (int32_t *)bptr_buf.ptr();
    MFE_TRY(scan_counts(ctx, m, (const int32_t *)P->rowblocks.ptr, bptr, (int64_t *)total_buf.ptr()));
    const unsigned grid = (unsigned)((m + kBlock - 1) / kBlock);
    hipLaunchKernelGGL(k_b13_export, dim3(grid), dim3(kBlock), 0, s, m, (const int32_t *)P->slot_base.ptr,
                       (const int32_t *)P->rowblocks.ptr, (const int32_t *)bptr,
                       (const int32_t *)P->jas.ptr, (const double *)P->bval64.ptr, bcol, bval);
    MFE_HIP_TRY(hipGetLastError());
    if (bptr_out)
        MFE_HIP_TRY(hipMemcpyAsync(bptr_out, bptr, (size_t)(m + 1) * sizeof(int32_t),
                                   hipMemcpyDeviceToDevice, s));
    MFE_HIP_TRY(hipStreamSynchronize(s));
    return MFE_OK;
}

}  // namespace mfe
