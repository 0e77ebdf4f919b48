// Device helpers: wavefront/workgroup reductions, the last-workgroup
// arrival test, XCD-aware tile ranges and streaming loads.
#pragma once

#include <hip/hip_runtime.h>

#include "common.hpp"

#ifndef MFE_XCD_REMAP
#define MFE_XCD_REMAP 1  // XCD-contiguous tile ranges for the CRS products (see tile_range)
#endif

namespace mfe {

// Sum over the 64 lanes of a wavefront by an xor butterfly: every lane ends
// with the same value, combined in a fixed order.
__device__ __forceinline__ double wave_sum(double v) {
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, 64);
    return v;
}

// Sum over the workgroup (kBlock threads).  Fixed order: lanes, then waves
// 0..3 in sequence.  Valid in thread 0 only.
__device__ __forceinline__ double block_sum(double v) {
    __shared__ double red[kBlock / 64];
    v = wave_sum(v);
    const int w = threadIdx.x >> 6;
    if ((threadIdx.x & 63) == 0) red[w] = v;
    __syncthreads();
    double s = 0.0;
    if (threadIdx.x == 0) {
#pragma unroll
        for (int i = 0; i < kBlock / 64; ++i) s += red[i];
    }
    __syncthreads();
    return s;
}

// Sum of the n partials written by the previous kernel, in a fixed order
// (lane-strided, then the workgroup tree), returned to every thread.  Every
// workgroup that calls it gets the bitwise-same value, so a scalar that a
// kernel needs (alpha, beta) is formed redundantly in each workgroup instead
// of by a separate launch or a cross-workgroup handshake.  Kernel
// boundaries make the previous kernel's stores visible on every XCD.
// Every thread of the workgroup must call it (it synchronises the workgroup).
__device__ __forceinline__ double sum_partials(const double *__restrict__ p, int n) {
    __shared__ double total;
    double s = 0.0;
    for (int i = threadIdx.x; i < n; i += kBlock) s += p[i];
    s = block_sum(s);
    if (threadIdx.x == 0) total = s;
    __syncthreads();
    return total;
}

// Tile range of this workgroup.  With XCD = true: workgroups are dispatched
// to the 8 XCDs round-robin (workgroup w runs on XCD w % 8), so XCD k takes
// the k-th contiguous eighth of the tiles and its workgroups stride through
// it together: each XCD's L2 then holds only the x entries near its own
// rows (gridDim.x must be a multiple of kNumXcd).  With XCD = false the
// whole grid strides through the tiles together, so that the chip reads
// one compact window of the matrix at a time.
struct TileRange {
    long t, end, step;
};
template <bool XCD = (MFE_XCD_REMAP != 0)>
__device__ __forceinline__ TileRange tile_range(long ntiles) {
    TileRange r;
    if (XCD) {
        const int xcd = blockIdx.x % kNumXcd;
        const int lid = blockIdx.x / kNumXcd;
        const int per = gridDim.x / kNumXcd;
        r.t = ntiles * xcd / kNumXcd + lid;
        r.end = ntiles * (xcd + 1) / kNumXcd;
        r.step = per;
    } else {
        r.t = blockIdx.x;
        r.end = ntiles;
        r.step = gridDim.x;
    }
    return r;
}

// Tile order of the 1x3 BCRS walks: the grid moves through the tiles in
// super-tiles of 8 S tiles (S = 2^sl), and inside each the XCD k takes the
// k-th run of S consecutive tiles, its workgroups striding through the XCD's
// runs in turn.  S = 1 is the grid-wide order, and S near ntiles / 8 comes
// close to the XCD-contiguous one; between them each XCD's L2 keeps the x
// entries of its runs while the chip still reads one region of the matrix at
// a time.  gridDim.x must be a multiple of kNumXcd.
struct TileSeq {
    long i, step, ntiles;
    int xcd, sl;
    __device__ __forceinline__ long tile(long j) const {
        return ((j >> sl) * kNumXcd + xcd) * (1L << sl) + (j & ((1L << sl) - 1));
    }
    __device__ __forceinline__ bool valid(long j) const { return tile(j) < ntiles; }
};
__device__ __forceinline__ TileSeq tile_seq(long ntiles, int sl) {
    TileSeq q;
    q.xcd = blockIdx.x % kNumXcd;
    q.i = blockIdx.x / kNumXcd;
    q.step = gridDim.x / kNumXcd;
    q.sl = sl;
    q.ntiles = ntiles;
    return q;
}

// Vector streams whose next use is more than one kernel away (or never).
// When the vectors of an iteration do not fit in the memory-side cache,
// loading and storing these non-temporally (nt = true) leaves that cache to
// the vector that the next SpMV gathers; when they fit, plain accesses keep
// them all cached.  nt is uniform over the launch.
template <typename T>
__device__ __forceinline__ T stream_load(const T *p, bool nt) {
    return nt ? __builtin_nontemporal_load(p) : *p;
}
template <typename T>
__device__ __forceinline__ void stream_store(T v, T *p, bool nt) {
    if (nt)
        __builtin_nontemporal_store(v, p);
    else
        *p = v;
}

// Matrix streams are read once per product.  A matrix larger than the
// memory-side cache is loaded non-temporally (NT = true) so that it does not
// evict the x entries that the gathers reuse; one that fits is loaded
// normally and stays cached from one product to the next (the launchers
// choose, see matrix_stream_nt).
template <bool NT = (MFE_MATRIX_NT != 0), typename T>
__device__ __forceinline__ T matrix_load(const T *p) {
    if constexpr (NT)
        return __builtin_nontemporal_load(p);
    else
        return *p;
}

}  // namespace mfe
