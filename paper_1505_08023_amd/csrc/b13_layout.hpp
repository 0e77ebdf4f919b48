// Slice layout of the fixed 1x3 BCRS (shared by the builder and the SpMV).
//
// Rows are grouped in slices of 64 (one wavefront, lane l = row 64 s + l).
// Slice s owns slot rows k0 = slot_base[s] .. k0 + S - 1 (S = blocks of its
// longest row); padding blocks have zero values.  Inside the slice's storage
// everything a wavefront loads is contiguous across lanes and 16-byte
// aligned, so one load instruction moves 16 bytes per lane:
//
//   column indices (64 S int32 from 64 k0):
//     slots 0..4Q-1 (Q = S/4) as quads   [q][lane][4]
//     slots 4Q..S-1 as singles           [k][lane]
//   values (192 S elements from 192 k0):
//     first two values of every block    [k][lane][2]          (S x 128)
//     third values of slots 0..2P-1      [p][lane][2], P = S/2 (P x 128)
//     third value of slot S-1 (S odd)    [lane]                (64)
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>

namespace mfe {

struct B13Slice {
    int64_t jbase;  // first column index of the slice (element offset)
    int64_t vbase;  // first value of the slice (element offset)
    int S;          // slots in the slice
};

__host__ __device__ __forceinline__ B13Slice b13_slice(int64_t k0, int64_t k1) {
    return B13Slice{k0 * 64, k0 * 192, (int)(k1 - k0)};
}

// element offset of the column index of slot k, lane l
__host__ __device__ __forceinline__ int64_t b13_jas(const B13Slice &sl, int k, int l) {
    const int Q = sl.S / 4;
    if (k < 4 * Q) return sl.jbase + (int64_t)(k / 4) * 256 + l * 4 + (k % 4);
    return sl.jbase + (int64_t)Q * 256 + (int64_t)(k - 4 * Q) * 64 + l;
}

// element offset of value j (0, 1, 2) of slot k, lane l
__host__ __device__ __forceinline__ int64_t b13_val(const B13Slice &sl, int k, int j, int l) {
    if (j < 2) return sl.vbase + (int64_t)k * 128 + l * 2 + j;
    const int P = sl.S / 2;
    if (k < 2 * P) return sl.vbase + (int64_t)sl.S * 128 + (int64_t)(k / 2) * 128 + l * 2 + (k % 2);
    return sl.vbase + (int64_t)sl.S * 128 + (int64_t)P * 128 + l;
}

// FP32 values of a 9-slot slice are stored packed instead, in the same
// region: the 27 values of a row in block order v = 3 k + j, as
// [q][lane][4] for q = 0..5 (v = 0..23) followed by [lane][3] (v = 24..26),
// so that a wavefront loads them with six 16-byte loads and one 12-byte load
// per lane rather than fourteen 8- or 4-byte ones.  Other slices keep the
// layout of b13_val in FP32 too.
__host__ __device__ __forceinline__ int64_t b13_val32_9(const B13Slice &sl, int v, int l) {
    if (v < 24) return sl.vbase + (int64_t)(v / 4) * 256 + l * 4 + (v % 4);
    return sl.vbase + 1536 + (int64_t)l * 3 + (v - 24);
}

}  // namespace mfe

namespace mfe {

// Column-index compression of a 9-slot slice.  When every block column of
// the slice has the form
//     jas(slot k, lane l) = 64 s + l + e_l + d[k],   e_l in {0, 1},
// (a structured-mesh slice: one offset per slot, one 0/1 shift per row, the
// shift being 1 for rows whose first stored column is the row itself) the
// SpMV forms the columns from this descriptor and does not read the slice's
// 576 column indices; the indices stay stored (export, other slices).  The
// reconstruction is exact, so results do not depend on which path a slice
// takes.  uniform = 0: read the indices.
struct B13Desc {
    int32_t d[9];
    uint32_t e_lo, e_hi;  // e_l of lanes 0..31 and 32..63
    int32_t uniform;
};
static_assert(sizeof(B13Desc) == 48, "B13Desc is 48 bytes");

}  // namespace mfe
