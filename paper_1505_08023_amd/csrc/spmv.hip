// Sparse matrix-vector products (Sec. 3.1 MATVEC) with optional fused CG
// epilogues (the DOT that follows MATVEC in CG, Sec. 3.1 discussion of
// Fig 3.5, and the residual at CG start/exit).
//
//   CRS (Fig 3.1):  mesh problems by row groups (up to 64 consecutive
//                   full rows per wavefront, their values staged in LDS,
//                   one lane per row); other matrices by 16-row wavefront
//                   tiles staged in LDS, 4 lanes per row over the row's
//                   (val, col) pairs, an xor butterfly per row.
//   1x3 BCRS:       one lane per row; per block one column index and three
//                   values, all coalesced across the wavefront's 64 rows,
//                   and three consecutive x entries (the implicit column
//                   increment of Fig 3.2, unrolled as in Fig 3.3).
//   In both, tiles or slices whose column indices follow one offset per
//   entry (CsrDesc, B13Desc) form them from a small descriptor instead of
//   loading them; the sums are the same.
//
// Both kernels run a workgroup grid sized to stay resident.  The CRS kernels
// walk row tiles in XCD-contiguous ranges, so each XCD's L2 holds the x
// entries of the mesh planes its rows touch.  The 1x3 BCRS kernels walk
// super-tiles of 8 x 16 tiles with the whole grid in step, each XCD taking 16
// consecutive tiles of each (tile_seq; fewer on a matrix with fewer than 16
// tiles per workgroup): the chip reads one region of the matrix at a time,
// which measured faster for them, and each XCD's L2 still serves most of its
// x gathers.  The matrix streams past non-temporally when
// it is larger than the memory-side cache can usefully keep
// (matrix_stream_nt).
#include <type_traits>

#include "b13_layout.hpp"
#include "common.hpp"
#include "device_util.hpp"
#include "spmv_rows.hpp"

// Build-time tuning constants (swept on MI355X; defaults are the measured best).
#ifndef MFE_CSR_LANES
#define MFE_CSR_LANES 32      // lanes per row of the CRS kernel
#endif
#ifndef MFE_CSR_STREAM
#define MFE_CSR_STREAM 1      // CRS by LDS-staged wavefront tiles (0: MFE_CSR_LANES lanes per row)
#endif
#ifndef MFE_SPMV_Q_NT
#define MFE_SPMV_Q_NT 0       // q store of the dot mode: 0 by vector size, 1 always non-temporal, 2 never
#endif
#ifndef MFE_B13_PIPE_TILES
#define MFE_B13_PIPE_TILES 8  // tiles per workgroup from which the pipelined 1x3 BCRS walk is used
#endif
#ifndef MFE_B13_WALK
#define MFE_B13_WALK 2  // pipelined 1x3 BCRS walk: 0 column indices read ahead, 1 scalars read ahead, 2 by precision
#endif
#ifndef MFE_B13_SUPER
#define MFE_B13_SUPER 16      // 1x3 BCRS products: most consecutive tiles per XCD in a super-tile, a power of two (tile_seq)
#endif
#ifndef MFE_SPMV_WG_PER_CU
#define MFE_SPMV_WG_PER_CU 0  // resident workgroups per CU (0: as many as fit)
#endif
#ifndef MFE_B13_WAVES_PER_EU
#define MFE_B13_WAVES_PER_EU 0  // minimum wavefronts per SIMD the 1x3 BCRS kernels are built for (0: compiler's choice)
#endif
#if MFE_B13_WAVES_PER_EU > 0
#define MFE_B13_OCCUPANCY __attribute__((amdgpu_waves_per_eu(MFE_B13_WAVES_PER_EU, 8)))
#else
#define MFE_B13_OCCUPANCY
#endif

namespace mfe {
namespace {

template <typename T>
struct Epi {
    const T *__restrict__ x;
    T *__restrict__ y;
    T *__restrict__ pout;
    const double *__restrict__ b;
    bool nt;  // store y non-temporally (dot mode: y is read once, by the r update)
};

// The epilogue's own operand of a row: x[row] for the dot modes, b[row] for
// the residual modes.  The kernels load it before the row's gathers: read
// after the y store (finish_row's order of use) it would cost every tile a
// second memory round trip, since the vector memory counter that the wait
// for it uses also counts the store.
template <typename T, int MODE>
__device__ __forceinline__ double row_operand(const Epi<T> &E, int64_t row) {
    if (MODE == kSpmvDot || MODE == kSpmvDot2) return (double)E.x[row];
    if (MODE == kSpmvResid || MODE == kSpmvTrue) return E.b[row];
    return 0.0;
}

// The value a row's y entry receives, with the row's reduction terms
// accumulated in FP64 (`opnd` from row_operand).
template <typename T, int MODE>
__device__ __forceinline__ T row_result(T sum, double opnd, double &d1, double &d2) {
    if (MODE == kSpmvDot) {
        d1 += opnd * (double)sum;
    } else if (MODE == kSpmvDot2) {
        d1 += opnd * (double)sum;
        d2 += opnd * opnd;
    } else if (MODE == kSpmvResid) {
        const double r = opnd - (double)sum;
        d1 += r * r;
        d2 += opnd * opnd;
        return (T)r;
    } else if (MODE == kSpmvTrue) {
        const double r = opnd - (double)sum;
        d1 += r * r;
    }
    return sum;
}

// The row's stores (none for kSpmvTrue; y and p for kSpmvResid).
template <typename T, int MODE>
__device__ __forceinline__ void row_store(const Epi<T> &E, int64_t row, T v) {
    if (MODE == kSpmvTrue) return;
    if (MODE == kSpmvDot) {
#if MFE_SPMV_Q_NT == 1
        stream_store(v, E.y + row, true);
#elif MFE_SPMV_Q_NT == 2
        E.y[row] = v;
#else
        stream_store(v, E.y + row, E.nt);
#endif
    } else {
        E.y[row] = v;
    }
    if (MODE == kSpmvResid && E.pout) E.pout[row] = v;
}

// Per-row epilogue: the row's result, stored at once.
template <typename T, int MODE>
__device__ __forceinline__ void finish_row(const Epi<T> &E, int64_t row, T sum, double opnd, double &d1,
                                           double &d2) {
    row_store<T, MODE>(E, row, row_result<T, MODE>(sum, opnd, d1, d2));
}

// Workgroup partial(s) of the fused reductions; the consumer (the next
// kernel, or a finalize kernel) sums them.
template <int MODE>
__device__ __forceinline__ void store_partials(double d1, double d2, double *partials) {
    if (MODE == kSpmvPlain) return;
    constexpr bool two = MODE == kSpmvResid || MODE == kSpmvDot2;
    d1 = block_sum(d1);
    if (two) d2 = block_sum(d2);
    if (threadIdx.x == 0) {
        partials[blockIdx.x] = d1;
        if (two) partials[kMaxPartials + blockIdx.x] = d2;
    }
}

// In the CG loop the product runs only while the solve is running; it also
// opens the iteration (the vector updates check `active`) and records the
// iteration count for the single-reduction update, which rewrites it.
__device__ __forceinline__ bool cg_gate(CgState *st) {
    if (blockIdx.x == 0 && threadIdx.x == 0) {
        st->active = 0;
        st->iters_snap = st->iters;
        st->status_snap = st->status;
    }
    return st->status == kRunning;
}

// ---------------------------------------------------------------- CRS

template <typename T, int L, int MODE, bool MNT>
__global__ __launch_bounds__(kBlock) void k_spmv_csr(int64_t m, const int32_t *__restrict__ ptr,
                                                     const int32_t *__restrict__ col,
                                                     const T *__restrict__ val, Epi<T> E, CgState *st,
                                                     double *partials) {
    if ((MODE == kSpmvDot || MODE == kSpmvDot2) && st && !cg_gate(st)) return;
    constexpr int R = kBlock / L;  // rows per tile
    const int g = threadIdx.x / L, sub = threadIdx.x % L;
    const long ntiles = (m + R - 1) / R;
    double d1 = 0.0, d2 = 0.0;
    for (TileRange tr = tile_range(ntiles); tr.t < tr.end; tr.t += tr.step) {
        const int64_t row = tr.t * R + g;
        const double opnd = sub == 0 && row < m ? row_operand<T, MODE>(E, row) : 0.0;
        const T sum = csr_row<T, L, MNT>(ptr, col, val, row < m ? row : -1, sub, E.x);
        if (sub == 0 && row < m) finish_row<T, MODE>(E, row, sum, opnd, d1, d2);
    }
    store_partials<MODE>(d1, d2, partials);
}

// CRS by wavefront tiles staged in LDS: a wavefront takes kCsrsRows
// consecutive rows, loads their (value, column) runs, contiguous in the CRS
// arrays, with coalesced loads into LDS, then each row is summed by
// 64 / kCsrsRows lanes (strided entries, combined by an xor butterfly)
// reading LDS and gathering x.  A tile with a uniform descriptor (CsrDesc)
// stages only its values and forms the columns from the 27 offsets, in the
// same summation order, or, when the offsets form 9 runs of three
// consecutive columns, sums a run per step (a different order, the same
// products).  A tile whose entries exceed the LDS capacity is
// summed straight from global memory instead.
constexpr int kCsrsCap = kCsrsRows * 28;       // staged entries per wavefront tile (kCsrsRows: common.hpp)

__device__ __forceinline__ void wave_sync() {
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

template <typename T, int MODE, bool MNT>
__global__ __launch_bounds__(kBlock) void k_spmv_csrs(int64_t m, const int32_t *__restrict__ ptr,
                                                      const int32_t *__restrict__ col,
                                                      const CsrDesc *__restrict__ cdesc,
                                                      const T *__restrict__ val, Epi<T> E, CgState *st,
                                                      double *partials) {
    if ((MODE == kSpmvDot || MODE == kSpmvDot2) && st && !cg_gate(st)) return;
    __shared__ T sval[kBlock / 64][kCsrsCap];
    __shared__ int32_t scol[kBlock / 64][kCsrsCap];
    const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6), lane = threadIdx.x & 63;
    constexpr int LPR = 64 / kCsrsRows;  // lanes per row
    const int sub = lane % LPR, rl = lane / LPR;
    T *sv = sval[wave];
    int32_t *sc = scol[wave];
    constexpr int R = (kBlock / 64) * kCsrsRows;  // rows per workgroup tile
    const long ntiles = (m + R - 1) / R;
    double d1 = 0.0, d2 = 0.0;
    for (TileRange tr = tile_range(ntiles); tr.t < tr.end; tr.t += tr.step) {
        const int64_t r0 = tr.t * R + (int64_t)wave * kCsrsRows;
        if (r0 >= m) continue;  // wavefront-uniform
        const int64_t r1 = r0 + kCsrsRows < m ? r0 + kCsrsRows : m;
        const int32_t lo = ptr[r0], hi = ptr[r1];
        const int64_t row = r0 + rl;
        const CsrDesc &D = cdesc[tr.t * (kBlock / 64) + wave];  // this wavefront's tile
        const double opnd = sub == 0 && row < r1 ? row_operand<T, MODE>(E, row) : 0.0;
        T sum = 0;
        if (D.uniform == 2) {
            // 27 entries per row in 9 runs of three consecutive columns: stage
            // the values and the 9 run starts.  With LPR = 4 lanes per row,
            // lane `sub` takes runs sub and sub + 4 (each a 1x3 block: one
            // 16-byte and one 8-byte gather) and lanes 1..3 one entry each of
            // run 8, so no lane does more than 7 products; other lane counts
            // take runs sub, sub + LPR, ...
            for (int j = lane; j < 27 * kCsrsRows; j += 64) sv[j] = matrix_load<MNT>(val + lo + j);
            if (lane < 9) sc[lane] = D.off[3 * lane];
            wave_sync();
            const int a = rl * 27;
            constexpr int nfull = LPR == 4 ? 8 : 9;
            for (int i = sub; i < nfull; i += LPR) {
                const T *xp = E.x + row + sc[i];
                sum += sv[a + 3 * i] * xp[0];
                sum += sv[a + 3 * i + 1] * xp[1];
                sum += sv[a + 3 * i + 2] * xp[2];
            }
            if (LPR == 4 && sub > 0) sum += sv[a + 23 + sub] * E.x[row + sc[8] + sub - 1];
            wave_sync();
        } else if (D.uniform) {
            // 27 entries per row, columns row + off[k]: stage the values only
            for (int j = lane; j < 27 * kCsrsRows; j += 64) sv[j] = matrix_load<MNT>(val + lo + j);
            if (lane < 27) sc[lane] = D.off[lane];
            wave_sync();
            const int a = rl * 27;
            for (int j = sub; j < 27; j += LPR) sum += sv[a + j] * E.x[row + sc[j]];
            wave_sync();
        } else if (hi - lo <= kCsrsCap) {
            for (int32_t j = lo + lane; j < hi; j += 64) {
                sv[j - lo] = matrix_load<MNT>(val + j);
                sc[j - lo] = matrix_load<MNT>(col + j);
            }
            wave_sync();
            if (row < r1) {
                const int32_t a = ptr[row] - lo, b = ptr[row + 1] - lo;
                for (int32_t j = a + sub; j < b; j += LPR) sum += sv[j] * E.x[sc[j]];
            }
            wave_sync();
        } else if (row < r1) {
            for (int32_t j = ptr[row] + sub; j < ptr[row + 1]; j += LPR)
                sum += matrix_load<MNT>(val + j) * E.x[matrix_load<MNT>(col + j)];
        }
#pragma unroll
        for (int off = LPR / 2; off > 0; off >>= 1) sum += __shfl_xor(sum, off, 64);
        if (sub == 0 && row < r1) finish_row<T, MODE>(E, row, sum, opnd, d1, d2);
    }
    store_partials<MODE>(d1, d2, partials);
}

// CRS by row groups (mesh problems, see CsrRuns in common.hpp).  A group of
// up to 64 consecutive full rows owns a contiguous run of 27 n values: the
// wavefront stages it in LDS with 16-byte loads, all issued before the first
// LDS store (the run is read from the 16-byte boundary at or before its
// start; its end never reaches the matrix's end, whose last row is a corner
// row outside every group), then lane l sums row r0 + l in ascending column
// order, nine runs of three consecutive x entries, reading its 27 values from
// LDS at stride 27 (the lanes' accesses fall into distinct banks).  The other
// rows (mesh boundary rows) come 16 per wavefront from the row list and are
// summed by 4 lanes each from global memory.
constexpr int kCsrgVec = 16;  // bytes per staging load

template <typename T>
struct CsrgStage {
    static constexpr int V = kCsrgVec / (int)sizeof(T);        // values per staging load
    static constexpr int Q = (27 * 64 + V - 1 + 64 * V - 1) / (64 * V);  // staging loads per lane
    static constexpr int N = Q * 64 * V;                         // LDS values per wavefront
};

template <typename T, int MODE, bool MNT>
__global__ __launch_bounds__(kBlock) void k_spmv_csrg(const int32_t *__restrict__ ptr, const int32_t *__restrict__ col,
                                                      const T *__restrict__ val, const int2 *__restrict__ items,
                                                      long nitems, const int32_t *__restrict__ rows, CsrRuns R,
                                                      Epi<T> E, CgState *st, double *partials) {
    if ((MODE == kSpmvDot || MODE == kSpmvDot2) && st && !cg_gate(st)) return;
    using S = CsrgStage<T>;
    typedef T vec_t __attribute__((ext_vector_type(S::V)));
    __shared__ vec_t sval[kBlock / 64][S::N / S::V];
    const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6), lane = threadIdx.x & 63;
    vec_t *sv = sval[wave];
    const T *svs = (const T *)sv;
    const long ntiles = (nitems + kBlock / 64 - 1) / (kBlock / 64);
    double d1 = 0.0, d2 = 0.0;
    // one work item: its record and, for a group, its staged values in registers
    struct Cur {
        int2 item;
        int32_t lo;
        vec_t v[S::Q];
    };
    auto fetch = [&](long it, Cur &c) {
        c.item = items[it];
        if (c.item.y <= 0) return;
        c.lo = ptr[c.item.x];
        const int pad = c.lo % S::V;
        const int nv = (pad + 27 * c.item.y + S::V - 1) / S::V;
        const vec_t *src = (const vec_t *)(val + (c.lo - pad));
#pragma unroll
        for (int q = 0; q < S::Q; ++q)
            if (lane + 64 * q < nv) c.v[q] = matrix_load<MNT>(src + lane + 64 * q);
    };
    auto process = [&](Cur &c) {
        if (c.item.y > 0) {
            const int64_t r0 = c.item.x;
            const int n = c.item.y;
            const int pad = c.lo % S::V;
            const int nv = (pad + 27 * n + S::V - 1) / S::V;
#pragma unroll
            for (int q = 0; q < S::Q; ++q)
                if (lane + 64 * q < nv) sv[lane + 64 * q] = c.v[q];
            wave_sync();
            if (lane < n) {
                const int64_t row = r0 + lane;
                const double opnd = row_operand<T, MODE>(E, row);
                const T *a = svs + pad + 27 * lane;
                T sum = 0;
#pragma unroll
                for (int i = 0; i < 9; ++i) {
                    const T *xp = E.x + row + R.r[i];
                    sum += a[3 * i] * xp[0];
                    sum += a[3 * i + 1] * xp[1];
                    sum += a[3 * i + 2] * xp[2];
                }
                finish_row<T, MODE>(E, row, sum, opnd, d1, d2);
            }
            wave_sync();
        } else {
            const int rl = lane >> 2, sub = lane & 3;
            const int64_t row = rl < -c.item.y ? rows[c.item.x + rl] : -1;
            const double opnd = sub == 0 && row >= 0 ? row_operand<T, MODE>(E, row) : 0.0;
            const T sum = csr_row<T, 4, MNT>(ptr, col, val, row, sub, E.x);
            if (sub == 0 && row >= 0) finish_row<T, MODE>(E, row, sum, opnd, d1, d2);
        }
    };
    // (issuing the next item's staging loads before the current item's sums,
    // from a second register set, measured no faster: 0.916 against 0.912 ms)
    for (TileRange tr = tile_range(ntiles); tr.t < tr.end; tr.t += tr.step) {
        const long it = tr.t * (kBlock / 64) + wave;
        if (it >= nitems) continue;  // wavefront-uniform
        Cur c;
        fetch(it, c);
        process(c);
    }
    store_partials<MODE>(d1, d2, partials);
}

// ---------------------------------------------------------------- 1x3 BCRS

// Plain walk (the FP32 product on small grids): one slice per wavefront per
// tile; slice bounds, column indices, values, gathers, in that dependent
// order.
template <typename T, int MODE, bool MNT>
__global__ __launch_bounds__(kBlock) MFE_B13_OCCUPANCY void k_spmv_b13(int64_t m, const int32_t *__restrict__ slot_base,
                                                     const int32_t *__restrict__ jas,
                                                     const B13Desc *__restrict__ desc,
                                                     const T *__restrict__ val, Epi<T> E, CgState *st,
                                                     double *partials, int super_log2) {
    if ((MODE == kSpmvDot || MODE == kSpmvDot2) && st && !cg_gate(st)) return;
    const long ntiles = (m + kBlock - 1) / kBlock;
    const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6), lane = threadIdx.x & 63;
    double d1 = 0.0, d2 = 0.0;
    const TileSeq q = tile_seq(ntiles, super_log2);
    for (long j = q.i; q.valid(j); j += q.step) {
        const int64_t s = (int64_t)q.tile(j) * (kBlock / 64) + wave;
        const int64_t row = s * 64 + lane;
        if (row >= m) continue;
        const double opnd = row_operand<T, MODE>(E, row);
        const T sum = b13_row<T, MNT>(slot_base, jas, desc, val, s, lane, E.x);
        finish_row<T, MODE>(E, row, sum, opnd, d1, d2);
    }
    store_partials<MODE>(d1, d2, partials);
}

// Software-pipelined walk for grids whose workgroups take several tiles: a
// wavefront owns slice 4t + w of tile t.  The slice bounds and descriptor
// come from scalar loads (the slice index is wavefront-uniform) and the next
// tile's column indices are formed or requested before the current tile's
// values and gathers, so the index -> gather dependency of one tile overlaps
// the streaming of the previous one.  Arithmetic and summation order are
// those of k_spmv_b13.
template <typename T, int MODE, bool MNT>
__global__ __launch_bounds__(kBlock) MFE_B13_OCCUPANCY void k_spmv_b13p(int64_t m, const int32_t *__restrict__ slot_base,
                                                      const int32_t *__restrict__ jas,
                                                      const B13Desc *__restrict__ desc,
                                                      const T *__restrict__ val, Epi<T> E, CgState *st,
                                                      double *partials, int super_log2) {
    if ((MODE == kSpmvDot || MODE == kSpmvDot2) && st && !cg_gate(st)) return;
    const long ntiles = (m + kBlock - 1) / kBlock;
    const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6), lane = threadIdx.x & 63;
    double d1 = 0.0, d2 = 0.0;
    const TileSeq q = tile_seq(ntiles, super_log2);
    B13Idx cur, nxt;
    auto fetch = [&](long t, B13Idx &r) {
        const int64_t s = (int64_t)t * (kBlock / 64) + wave;
        const int64_t row = s * 64 + lane;
        r.sl.S = 0;
        if (s * 64 >= m) return;
        r.sl = b13_slice(slot_base[s], slot_base[s + 1]);
        if (row < m) b13_cols<MNT>(jas, desc, s, lane, r);
    };
    if (q.valid(q.i)) fetch(q.tile(q.i), cur);
    for (long j = q.i; q.valid(j); j += q.step) {
        nxt.sl.S = 0;
        if (q.valid(j + q.step)) fetch(q.tile(j + q.step), nxt);
        const int64_t row = q.tile(j) * kBlock + threadIdx.x;
        if (row < m) {
            const double opnd = row_operand<T, MODE>(E, row);
            const T sum = cur.sl.S == 9 ? b13_row9_idx<T, MNT>(cur.c, val, cur.sl, lane, E.x)
                                        : b13_row_generic<T, MNT>(jas, val, cur.sl, lane, E.x);
            finish_row<T, MODE>(E, row, sum, opnd, d1, d2);
        }
        cur = nxt;
    }
    store_partials<MODE>(d1, d2, partials);
}

// Scalar-prefetch walk: a wavefront owns slice 4t + w of tile t.  Only
// wavefront-uniform data is read ahead: the next tile's slice bounds and
// descriptor come from scalar loads issued before the current tile's vector
// loads, and nothing that a vector load wrote is carried into the next tile.
// A tile's row result is complete before its y store, so no wait on the
// vector memory counter (which also counts stores) falls between that store
// and the next tile's loads: the store's latency overlaps them.  Descriptor
// slices form their column indices from the carried scalars; the few others
// load theirs in place (b13_ahead, b13_row_ahead).  Arithmetic and
// summation order are those of k_spmv_b13.
template <typename T, int MODE, bool MNT>
__global__ __launch_bounds__(kBlock) MFE_B13_OCCUPANCY void k_spmv_b13s(int64_t m, const int32_t *__restrict__ slot_base,
                                                      const int32_t *__restrict__ jas,
                                                      const B13Desc *__restrict__ desc,
                                                      const T *__restrict__ val, Epi<T> E, CgState *st,
                                                      double *partials, int super_log2) {
    if ((MODE == kSpmvDot || MODE == kSpmvDot2) && st && !cg_gate(st)) return;
    const long ntiles = (m + kBlock - 1) / kBlock;
    const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6), lane = threadIdx.x & 63;
    double d1 = 0.0, d2 = 0.0;
    const TileSeq q = tile_seq(ntiles, super_log2);
    const int64_t nslices = (m + 63) / 64;
    auto slice = [&](long j) -> int64_t {  // this wavefront's slice of the j-th tile, or -1
        if (!q.valid(j)) return -1;
        const int64_t s = (int64_t)q.tile(j) * (kBlock / 64) + wave;
        return s < nslices ? s : -1;
    };
    B13Ahead cur, nxt;
    b13_ahead(slot_base, desc, slice(q.i), cur);
    for (long j = q.i; q.valid(j); j += q.step) {
        b13_ahead(slot_base, desc, slice(j + q.step), nxt);
        const int64_t s = (int64_t)q.tile(j) * (kBlock / 64) + wave;
        const int64_t row = s * 64 + lane;
        if (row < m) {
            const double opnd = row_operand<T, MODE>(E, row);
            const T sum = b13_row_ahead<T, MNT>(cur, jas, val, s, lane, E.x);
            const T v = row_result<T, MODE>(sum, opnd, d1, d2);
            row_store<T, MODE>(E, row, v);
        }
        cur = nxt;
    }
    store_partials<MODE>(d1, d2, partials);
}

// ---------------------------------------------------------------- launch

// Super-tile length (log2) of the 1x3 BCRS walks: the longest run, up to
// MFE_B13_SUPER tiles, that leaves no workgroup more tiles to walk than
// single tiles dealt round the XCDs would.  XCD 0 holds the most tiles, the
// full super-tiles' runs plus the first run of the ragged last one; on a
// matrix of few super-tiles long runs would load the first XCDs only (16^3:
// 20 tiles, with runs of 16 on 2 of the 8 XCDs, 6 tiles for some
// workgroups).  From 77^3 up the runs stay at 16.
int b13_super_log2(long ntiles, int grid) {
    const long per_xcd = grid >= kNumXcd ? grid / kNumXcd : 1;
    auto worst = [&](long S) {
        const long F = ntiles / (kNumXcd * S), R = ntiles % (kNumXcd * S);
        return (F * S + (R < S ? R : S) + per_xcd - 1) / per_xcd;
    };
    const long best = worst(1);
    int sl = 0;
    for (int l = 1; (1L << l) <= MFE_B13_SUPER; ++l)
        if (worst(1L << l) == best) sl = l;
    return sl;
}

template <typename K>
int grid_for(K kernel, long ntiles, int num_cu) {
    long per_cu = resident_per_cu((const void *)kernel);
    if (MFE_SPMV_WG_PER_CU > 0 && MFE_SPMV_WG_PER_CU < per_cu) per_cu = MFE_SPMV_WG_PER_CU;
    return resident_grid((long)num_cu * per_cu, ntiles);
}

// Bytes of a stored matrix, for the non-temporal choice (matrix_stream_nt).
template <typename T>
int64_t csr_bytes(const mfe_problem *P) {
    return P->nnz * (int64_t)(sizeof(T) + sizeof(int32_t)) + (P->m + 1) * (int64_t)sizeof(int32_t);
}
template <typename T>
int64_t b13_bytes(const mfe_problem *P) {
    return P->nslots * 64 * (int64_t)(3 * sizeof(T) + sizeof(int32_t));
}

// A launch whose grid would write more partials than `cap` (when cap > 0)
// is refused before it starts.
int check_cap(int grid, int cap) {
    if (cap > 0 && grid > cap) {
        set_error("the product's grid (" + std::to_string(grid) + " workgroups) exceeds its partials buffer (" +
                  std::to_string(cap) + ")");
        return MFE_EUNSUPPORTED;
    }
    return MFE_OK;
}

template <typename T, int MODE, bool MNT>
int launch_csr_as(const mfe_problem *P, const Epi<T> &E, CgState *st, double *partials, hipStream_t s,
                  int *grid_out, int cap) {
    const T *val = std::is_same<T, double>::value ? (const T *)P->val64.ptr : (const T *)P->val32.ptr;
    if (P->ncitems > 0) {
        auto kern = k_spmv_csrg<T, MODE, MNT>;
        const long ntiles = (P->ncitems + kBlock / 64 - 1) / (kBlock / 64);
        const int grid = grid_for(kern, ntiles, P->ctx->num_cu);
        MFE_TRY(check_cap(grid, cap));
        hipLaunchKernelGGL(kern, dim3(grid), dim3(kBlock), 0, s, (const int32_t *)P->ptr.ptr,
                           (const int32_t *)P->col.ptr, val, (const int2 *)P->citems.ptr, (long)P->ncitems,
                           (const int32_t *)P->crows.ptr, P->cruns, E, st, partials);
        MFE_HIP_TRY(hipGetLastError());
        if (grid_out) *grid_out = grid;
        return MFE_OK;
    }
#if MFE_CSR_STREAM
    auto kern = k_spmv_csrs<T, MODE, MNT>;
    const long ntiles = (P->m + (kBlock / 64) * kCsrsRows - 1) / ((kBlock / 64) * kCsrsRows);
#else
    // L lanes per row: with 32, a row of the 27-point matrix (one contiguous
    // 216-byte run of values) is read by one half-wavefront.
    constexpr int L = MFE_CSR_LANES;
    auto kern = k_spmv_csr<T, L, MODE, MNT>;
    const long ntiles = (P->m + kBlock / L - 1) / (kBlock / L);
#endif
    const int grid = grid_for(kern, ntiles, P->ctx->num_cu);
    MFE_TRY(check_cap(grid, cap));
#if MFE_CSR_STREAM
    hipLaunchKernelGGL(kern, dim3(grid), dim3(kBlock), 0, s, P->m, (const int32_t *)P->ptr.ptr,
                       (const int32_t *)P->col.ptr, (const CsrDesc *)P->cdesc.ptr, val, E, st, partials);
#else
    hipLaunchKernelGGL(kern, dim3(grid), dim3(kBlock), 0, s, P->m, (const int32_t *)P->ptr.ptr,
                       (const int32_t *)P->col.ptr, val, E, st, partials);
#endif
    MFE_HIP_TRY(hipGetLastError());
    if (grid_out) *grid_out = grid;
    return MFE_OK;
}

template <typename T, int MODE>
int launch_csr(const mfe_problem *P, const Epi<T> &E, CgState *st, double *partials, hipStream_t s, int *grid_out,
               int cap) {
    return matrix_stream_nt(csr_bytes<T>(P)) ? launch_csr_as<T, MODE, true>(P, E, st, partials, s, grid_out, cap)
                                             : launch_csr_as<T, MODE, false>(P, E, st, partials, s, grid_out, cap);
}

template <typename T, int MODE, bool MNT>
int launch_b13_as(const mfe_problem *P, const Epi<T> &E, CgState *st, double *partials, hipStream_t s,
                  int *grid_out, int cap) {
    const T *val = std::is_same<T, double>::value ? (const T *)P->bval64.ptr : (const T *)P->bval32.ptr;
    const long ntiles = (P->m + kBlock - 1) / kBlock;
    // the scalar read-ahead walk measured faster in FP64 (256^3: 0.794 against
    // 0.803 ms for the index read-ahead; 64^3 with runs of 16 tiles: 18.7
    // against 21.2 us for the plain walk; one exception below), the index
    // read-ahead in FP32 once each workgroup takes several tiles (256^3:
    // 0.404 against 0.414 ms), and the plain walk in FP32 below that
    constexpr bool scalar_walk = MFE_B13_WALK == 1 || (MFE_B13_WALK == 2 && std::is_same<T, double>::value);
    auto kern = scalar_walk ? k_spmv_b13s<T, MODE, MNT> : k_spmv_b13p<T, MODE, MNT>;
    int grid = grid_for(kern, ntiles, P->ctx->num_cu);
    if (!scalar_walk && ntiles < (long)MFE_B13_PIPE_TILES * grid) {
        kern = k_spmv_b13<T, MODE, MNT>;
        grid = grid_for(kern, ntiles, P->ctx->num_cu);
    }
    // Where the scalar walk's resident grid would leave some workgroups a
    // second tile and the plain walk's larger one (fewer registers, more
    // resident workgroups) takes every tile in one pass, there is no next
    // tile to read ahead and the plain walk is faster (64^3 FP64 CG: 37.7
    // against 36.5 k it/s; from 48^3 down and from 96^3 up it is 1-3 %
    // slower).
    if (scalar_walk && ntiles > grid) {
        const int gp = grid_for(k_spmv_b13<T, MODE, MNT>, ntiles, P->ctx->num_cu);
        if (ntiles <= gp) {
            kern = k_spmv_b13<T, MODE, MNT>;
            grid = gp;
        }
    }
    MFE_TRY(check_cap(grid, cap));
    hipLaunchKernelGGL(kern, dim3(grid), dim3(kBlock), 0, s, P->m, (const int32_t *)P->slot_base.ptr,
                       (const int32_t *)P->jas.ptr, (const B13Desc *)P->bdesc.ptr, val, E, st, partials,
                       b13_super_log2(ntiles, grid));
    MFE_HIP_TRY(hipGetLastError());
    if (grid_out) *grid_out = grid;
    return MFE_OK;
}

template <typename T, int MODE>
int launch_b13(const mfe_problem *P, const Epi<T> &E, CgState *st, double *partials, hipStream_t s, int *grid_out,
               int cap) {
    return matrix_stream_nt(b13_bytes<T>(P)) ? launch_b13_as<T, MODE, true>(P, E, st, partials, s, grid_out, cap)
                                             : launch_b13_as<T, MODE, false>(P, E, st, partials, s, grid_out, cap);
}

template <typename T, int MODE>
int launch_mode(const mfe_problem *P, int format, const SpmvArgs &a, hipStream_t s, int *grid) {
    Epi<T> E{(const T *)a.x, (T *)a.y, (T *)a.p_out, a.b, vectors_stream_nt(P->m)};
    if (format == MFE_CSR) return launch_csr<T, MODE>(P, E, a.st, a.partials, s, grid, a.max_partials);
    return launch_b13<T, MODE>(P, E, a.st, a.partials, s, grid, a.max_partials);
}

}  // namespace

int launch_spmv(const mfe_problem *P, int format, bool f32, SpmvMode mode, const SpmvArgs &a,
                hipStream_t s, int *grid) {
    if (f32) {
        switch (mode) {
            case kSpmvPlain: return launch_mode<float, kSpmvPlain>(P, format, a, s, grid);
            case kSpmvDot: return launch_mode<float, kSpmvDot>(P, format, a, s, grid);
            default: break;  // residuals are always evaluated in FP64
        }
        set_error("internal: FP32 residual SpMV requested");
        return MFE_EINVAL;
    }
    switch (mode) {
        case kSpmvPlain: return launch_mode<double, kSpmvPlain>(P, format, a, s, grid);
        case kSpmvDot: return launch_mode<double, kSpmvDot>(P, format, a, s, grid);
        case kSpmvResid: return launch_mode<double, kSpmvResid>(P, format, a, s, grid);
        case kSpmvTrue: return launch_mode<double, kSpmvTrue>(P, format, a, s, grid);
        case kSpmvDot2: return launch_mode<double, kSpmvDot2>(P, format, a, s, grid);
    }
    return MFE_EINVAL;
}

}  // namespace mfe
