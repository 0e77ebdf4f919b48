// Row-level SpMV building blocks shared by the single-system and batched
// kernels (Sec. 3.1: CRS row of Fig 3.1; 1x3 segments of Figs 3.2/3.3).
#pragma once

#include <type_traits>

#include "b13_layout.hpp"
#include "common.hpp"
#include "device_util.hpp"

namespace mfe {

// CRS row by L lanes (L a power of two dividing 64): lane `sub` takes
// entries sub, sub+L, ...; the xor butterfly leaves the row sum in every lane
// of the group.  row < 0: no row (the lanes still join the butterfly).
template <typename T, int L, bool NT = (MFE_MATRIX_NT != 0)>
__device__ __forceinline__ T csr_row(const int32_t *__restrict__ ptr, const int32_t *__restrict__ col,
                                     const T *__restrict__ val, int64_t row, int sub, const T *__restrict__ x) {
    T sum = 0;
    if (row >= 0) {
        const int32_t lo = ptr[row], hi = ptr[row + 1];
        for (int32_t j = lo + sub; j < hi; j += L) sum += matrix_load<NT>(val + j) * x[matrix_load<NT>(col + j)];
    }
#pragma unroll
    for (int off = L / 2; off > 0; off >>= 1) sum += __shfl_xor(sum, off, L);
    return sum;
}

template <typename T>
using vec2_t = T __attribute__((ext_vector_type(2)));
typedef int32_t int4_t __attribute__((ext_vector_type(4)));

// Any slice: one block at a time.
template <typename T, bool NT = (MFE_MATRIX_NT != 0)>
__device__ __forceinline__ T b13_row_generic(const int32_t *jas, const T *val, const B13Slice &sl, int lane,
                                             const T *x) {
    T sum = 0;
    for (int k = 0; k < sl.S; ++k) {
        const T *xp = x + matrix_load<NT>(jas + b13_jas(sl, k, lane));
        sum += matrix_load<NT>(val + b13_val(sl, k, 0, lane)) * xp[0];
        sum += matrix_load<NT>(val + b13_val(sl, k, 1, lane)) * xp[1];
        sum += matrix_load<NT>(val + b13_val(sl, k, 2, lane)) * xp[2];
    }
    return sum;
}

// Column indices of one row of a 9-slot slice, loaded ahead of its values so
// that the next row's index loads overlap the current row's gathers.
struct B13Idx {
    B13Slice sl;
    int32_t c[9];
};

template <bool NT = (MFE_MATRIX_NT != 0)>
__device__ __forceinline__ void b13_load_idx(const int32_t *__restrict__ jas, int lane, B13Idx &r) {
    if (r.sl.S != 9) return;
    const int4_t q0 = matrix_load<NT>((const int4_t *)(jas + r.sl.jbase + lane * 4));
    const int4_t q1 = matrix_load<NT>((const int4_t *)(jas + r.sl.jbase + 256 + lane * 4));
    r.c[0] = q0.x, r.c[1] = q0.y, r.c[2] = q0.z, r.c[3] = q0.w;
    r.c[4] = q1.x, r.c[5] = q1.y, r.c[6] = q1.z, r.c[7] = q1.w;
    r.c[8] = matrix_load<NT>(jas + r.sl.jbase + 512 + lane);
}

// Column indices of one row of slice s (r.sl already set): formed from the
// slice descriptor when the slice is uniform, else loaded.  s must be
// wavefront-uniform (the descriptor is read with scalar loads).
template <bool NT = (MFE_MATRIX_NT != 0)>
__device__ __forceinline__ void b13_cols(const int32_t *__restrict__ jas, const B13Desc *__restrict__ desc,
                                         int64_t s, int lane, B13Idx &r) {
    if (r.sl.S != 9) return;
    const B13Desc &D = desc[s];
    if (D.uniform) {
        // both shift words as scalars, then a per-lane select (selecting the
        // address instead would turn the read into a vector load that the
        // tile's gathers wait for)
        const uint32_t e_lo = __builtin_amdgcn_readfirstlane(D.e_lo), e_hi = __builtin_amdgcn_readfirstlane(D.e_hi);
        const uint32_t bits = lane < 32 ? e_lo : e_hi;
        const int32_t base = (int32_t)(s * 64 + lane) + (int32_t)((bits >> (lane & 31)) & 1u);
#pragma unroll
        for (int k = 0; k < 9; ++k) r.c[k] = base + D.d[k];
    } else {
        b13_load_idx<NT>(jas, lane, r);
    }
}

typedef float float4_t __attribute__((ext_vector_type(4)));

// Values and gathers of a 9-slot row whose indices are already loaded.  FP32
// values come from the packed layout (b13_val32_9); the products are summed
// in the same order in both precisions.
template <typename T, bool NT = (MFE_MATRIX_NT != 0)>
__device__ __forceinline__ T b13_row9_idx(const int32_t *c, const T *val, const B13Slice &sl, int lane,
                                          const T *x) {
    if constexpr (std::is_same<T, float>::value) {
        float v[27];
#pragma unroll
        for (int q = 0; q < 6; ++q) {
            const float4_t t = matrix_load<NT>((const float4_t *)(val + sl.vbase + q * 256 + lane * 4));
            v[4 * q] = t.x, v[4 * q + 1] = t.y, v[4 * q + 2] = t.z, v[4 * q + 3] = t.w;
        }
#pragma unroll
        for (int j = 0; j < 3; ++j) v[24 + j] = matrix_load<NT>(val + sl.vbase + 1536 + lane * 3 + j);
        float sum = 0;
#pragma unroll
        for (int k = 0; k < 9; ++k) {
            const float *xp = x + c[k];
            sum += v[3 * k] * xp[0];
            sum += v[3 * k + 1] * xp[1];
            sum += v[3 * k + 2] * xp[2];
        }
        return sum;
    }
    vec2_t<T> a[9], b[4];
#pragma unroll
    for (int k = 0; k < 9; ++k) a[k] = matrix_load<NT>((const vec2_t<T> *)(val + sl.vbase + k * 128 + lane * 2));
#pragma unroll
    for (int p = 0; p < 4; ++p)
        b[p] = matrix_load<NT>((const vec2_t<T> *)(val + sl.vbase + 9 * 128 + p * 128 + lane * 2));
    const T w8 = matrix_load<NT>(val + sl.vbase + 13 * 128 + lane);
    const T v2[9] = {b[0].x, b[0].y, b[1].x, b[1].y, b[2].x, b[2].y, b[3].x, b[3].y, w8};
    T sum = 0;
#pragma unroll
    for (int k = 0; k < 9; ++k) {
        const T *xp = x + c[k];
        sum += a[k].x * xp[0];
        sum += a[k].y * xp[1];
        sum += v2[k] * xp[2];
    }
    return sum;
}

// Wavefront-uniform data of a slice, read one slice ahead with scalar loads
// (the scalar read-ahead walks): its slot range and descriptor.
struct B13Ahead {
    int32_t k0, k1;  // slot_base[s], slot_base[s + 1]
    B13Desc D;
};

// s wavefront-uniform; s < 0 (no slice) leaves an empty slot range.
__device__ __forceinline__ void b13_ahead(const int32_t *__restrict__ slot_base, const B13Desc *__restrict__ desc,
                                          int64_t s, B13Ahead &a) {
    a.k0 = a.k1 = 0;
    if (s < 0) return;
    a.k0 = slot_base[s];
    a.k1 = slot_base[s + 1];
    a.D = desc[s];
}

// Row 64 s + lane of slice s from its read-ahead data: descriptor slices form
// their column indices from it, the others load theirs here.
template <typename T, bool NT = (MFE_MATRIX_NT != 0)>
__device__ __forceinline__ T b13_row_ahead(const B13Ahead &a, const int32_t *__restrict__ jas,
                                           const T *__restrict__ val, int64_t s, int lane, const T *__restrict__ x) {
    B13Idx r;
    r.sl = b13_slice(a.k0, a.k1);
    if (r.sl.S != 9) return b13_row_generic<T, NT>(jas, val, r.sl, lane, x);
    if (a.D.uniform) {
        const uint32_t bits = lane < 32 ? a.D.e_lo : a.D.e_hi;
        const int32_t base = (int32_t)(s * 64 + lane) + (int32_t)((bits >> (lane & 31)) & 1u);
#pragma unroll
        for (int k = 0; k < 9; ++k) r.c[k] = base + a.D.d[k];
    } else {
        b13_load_idx<NT>(jas, lane, r);
    }
    return b13_row9_idx<T, NT>(r.c, val, r.sl, lane, x);
}

// 1x3 BCRS row 64 s + lane (one lane per row; s wavefront-uniform).
template <typename T, bool NT = (MFE_MATRIX_NT != 0)>
__device__ __forceinline__ T b13_row(const int32_t *__restrict__ slot_base, const int32_t *__restrict__ jas,
                                     const B13Desc *__restrict__ desc, const T *__restrict__ val, int64_t s,
                                     int lane, const T *__restrict__ x) {
    B13Idx r;
    r.sl = b13_slice(slot_base[s], slot_base[s + 1]);
    b13_cols<NT>(jas, desc, s, lane, r);
    return r.sl.S == 9 ? b13_row9_idx<T, NT>(r.c, val, r.sl, lane, x) : b13_row_generic<T, NT>(jas, val, r.sl, lane, x);
}

}  // namespace mfe
