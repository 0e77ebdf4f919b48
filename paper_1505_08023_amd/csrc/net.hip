// Learned initial guess for CG: a 3-D convolutional encoder-decoder on the
// node grid of a box mesh, trained on solutions of the plain method and run
// in BF16 on the matrix cores (v_mfma_f32_16x16x32_bf16, FP32 accumulation).
//
// Layout: activations channels-last, act[n][voxel][c] (bf16), voxel index
// x + G (y + G z) like the mesh's node ids; channel counts are multiples of 8
// so that 8 consecutive reduction indices k = d Cin + c (d the tap) are 8
// contiguous channels of one source voxel: one 16-byte load per MFMA lane.
//
// Convolution (one kernel for every use): out[n][p][o] = sum_{d,c}
// W[o][d Cin + c] in[n][src(p, d)][c] with three tap patterns per axis
//   s1: src = p + d - 1      s2: src = 2p + d - 1
//   t2: src = (p + 1 - d)/2  where p + 1 - d is even (transposed stride 2)
// and zero outside the grid.  The input gradient of an s1 layer is an s1
// convolution with the taps mirrored, that of s2 is t2 and that of t2 is s2
// (same taps), each with the weights transposed in (o, c): the backward pass
// reuses the forward kernel on a re-laid-out weight copy.  Weight gradients
// are an MFMA GEMM over voxels through LDS-transposed tiles, reduced in a
// fixed order over voxel splits (deterministic).  Master weights and Adam
// state are FP32.
#include <hip/hip_runtime.h>

#include <cmath>
#include <cstring>
#include <new>
#include <string>
#include <utility>
#include <vector>

#include "common.hpp"
#include "device_util.hpp"

typedef __bf16 bf16;
typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef float f32x4 __attribute__((ext_vector_type(4)));
typedef unsigned int u32x4 __attribute__((ext_vector_type(4)));

namespace mfe {
namespace {

enum ConvMode : int { kS1 = 0, kS2 = 1, kT2 = 2 };

__device__ __forceinline__ bf16x8 zero8() { return __builtin_bit_cast(bf16x8, (u32x4)(0u)); }

__device__ __forceinline__ bf16x8 load8(const bf16 *p) {
    return __builtin_bit_cast(bf16x8, *(const u32x4 *)p);
}

// Source index along one axis, or -1.
template <int MODE>
__device__ __forceinline__ int src_axis(int p, int d, int Gi) {
    int i;
    if (MODE == kS1) {
        i = p + d - 1;
    } else if (MODE == kS2) {
        i = 2 * p + d - 1;
    } else {
        const int t = p + 1 - d;
        if (t & 1) return -1;
        i = t >> 1;
    }
    return (i >= 0 && i < Gi) ? i : -1;
}

// Flat source voxel of output voxel (pz, py, px) for tap d, or -1.
template <int MODE>
__device__ __forceinline__ int64_t src_voxel(int pz, int py, int px, int d, int Gi) {
    const int iz = src_axis<MODE>(pz, d / 9, Gi);
    const int iy = src_axis<MODE>(py, (d / 3) % 3, Gi);
    const int ix = src_axis<MODE>(px, d % 3, Gi);
    if ((iz | iy | ix) < 0) return -1;
    return ((int64_t)iz * Gi + iy) * Gi + ix;
}

// ------------------------------------------------------------------ convolution (forward and input gradient)

// One wavefront computes MT tiles of 16 output voxels x 16 NT output
// channels (channel group blockIdx.y) over the reduction steps of split
// blockIdx.z.  W is [16 nt][Kpad] with zero rows beyond Cout and zero columns
// beyond Kreal = 27 Cin.  The operands of step i + 1 are requested before the
// matrix-core products of step i, so one step's loads overlap the previous
// step's products.  With part == nullptr the epilogue runs here: + bias[o],
// + add[v][o] (a skip connection or an accumulating gradient, may alias out),
// ReLU, store bf16 (and FP32).  Otherwise the split's FP32 sums go to
// part[split][v][o] and k_conv_reduce finishes.
template <int MODE, int NT, int MT>
__global__ __launch_bounds__(256) void k_conv(const bf16 *__restrict__ in, int Gi, int cin_log2,
                                              const bf16 *__restrict__ W, int Kpad, int Kreal, int Cout, int Go,
                                              int64_t total, int steps_per_split, const float *__restrict__ bias,
                                              const bf16 *add, int relu, bf16 *out, float *__restrict__ out32,
                                              float *__restrict__ part) {
    const int lane = threadIdx.x & 63;
    const int64_t wave = (int64_t)blockIdx.x * 4 + (threadIdx.x >> 6);
    const int64_t base = wave * 16 * MT;
    if (base >= total) return;
    const int o0 = blockIdx.y * 16 * NT;
    const int s0 = blockIdx.z * steps_per_split;
    const int s1 = min(s0 + steps_per_split, Kpad >> 5);
    const int row = lane & 15, kg = lane >> 4;
    const int64_t Vi = (int64_t)Gi * Gi * Gi;
    // Voxel coordinates by 32-bit division (the launchers keep total below
    // 2^31): 64-bit division has no hardware path and cost more issue time
    // than the products at batch 1.
    const uint32_t uGo = (uint32_t)Go, uVo = uGo * uGo * uGo;
    int pz[MT], py[MT], px[MT];
    int64_t nb[MT];
    bool rv[MT];
#pragma unroll
    for (int mt = 0; mt < MT; ++mt) {
        const int64_t v = base + mt * 16 + row;
        rv[mt] = v < total;
        const uint32_t vv = rv[mt] ? (uint32_t)v : 0u;
        const uint32_t n = vv / uVo, p = vv - n * uVo, q = p / uGo, z = q / uGo;
        px[mt] = (int)(p - q * uGo);
        py[mt] = (int)(q - z * uGo);
        pz[mt] = (int)z;
        nb[mt] = (int64_t)n * Vi;
    }
    f32x4 acc[MT][NT];
#pragma unroll
    for (int mt = 0; mt < MT; ++mt)
#pragma unroll
        for (int nt = 0; nt < NT; ++nt) acc[mt][nt] = (f32x4)(0.0f);
    const int cmask = (1 << cin_log2) - 1;
    const bf16 *Wrow = W + (int64_t)(o0 + row) * Kpad;
    auto load_step = [&](int st, bf16x8(&a)[MT], bf16x8(&b)[NT]) {
        const int k = st * 32 + 8 * kg;
        const int d = k >> cin_log2, c0 = k & cmask;
#pragma unroll
        for (int mt = 0; mt < MT; ++mt) {
            int64_t sv = -1;
            if (rv[mt] && k < Kreal) sv = src_voxel<MODE>(pz[mt], py[mt], px[mt], d, Gi);
            a[mt] = sv >= 0 ? load8(in + ((nb[mt] + sv) << cin_log2) + c0) : zero8();
        }
#pragma unroll
        for (int nt = 0; nt < NT; ++nt) b[nt] = load8(Wrow + (int64_t)nt * 16 * Kpad + k);
    };
    bf16x8 a0[MT], b0[NT];
    if (s0 < s1) load_step(s0, a0, b0);
    for (int st = s0; st < s1; ++st) {
        const bool more = st + 1 < s1;
        bf16x8 a1[MT], b1[NT];
        if (more) load_step(st + 1, a1, b1);
#pragma unroll
        for (int nt = 0; nt < NT; ++nt)
#pragma unroll
            for (int mt = 0; mt < MT; ++mt)
                acc[mt][nt] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a0[mt], b0[nt], acc[mt][nt], 0, 0, 0);
        if (more) {
#pragma unroll
            for (int mt = 0; mt < MT; ++mt) a0[mt] = a1[mt];
#pragma unroll
            for (int nt = 0; nt < NT; ++nt) b0[nt] = b1[nt];
        }
    }
#pragma unroll
    for (int mt = 0; mt < MT; ++mt)
#pragma unroll
        for (int nt = 0; nt < NT; ++nt)
#pragma unroll
            for (int j = 0; j < 4; ++j) {
                const int64_t v = base + mt * 16 + 4 * kg + j;
                const int o = o0 + nt * 16 + row;
                if (v >= total || o >= Cout) continue;
                float val = acc[mt][nt][j];
                const int64_t idx = v * Cout + o;
                if (part) {
                    part[(int64_t)blockIdx.z * total * Cout + idx] = val;
                    continue;
                }
                if (bias) val += bias[o];
                if (add) val += (float)add[idx];
                if (relu) val = fmaxf(val, 0.0f);
                out[idx] = (bf16)val;
                if (out32) out32[idx] = val;
            }
}

// Sum of the reduction splits in split order, then the epilogue of k_conv.
__global__ __launch_bounds__(256) void k_conv_reduce(const float *__restrict__ part, int nsplit, int64_t n,
                                                     int Cout, const float *__restrict__ bias, const bf16 *add,
                                                     int relu, bf16 *out, float *__restrict__ out32) {
    const int64_t stride = (int64_t)gridDim.x * 256;
    for (int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x; i < n; i += stride) {
        float val = 0.0f;
        for (int z = 0; z < nsplit; ++z) val += part[(int64_t)z * n + i];
        if (bias) val += bias[i & (Cout - 1)];  // Cout is a power of two
        if (add) val += (float)add[i];
        if (relu) val = fmaxf(val, 0.0f);
        out[i] = (bf16)val;
        if (out32) out32[i] = val;
    }
}

// ------------------------------------------------------------------ stride 1 through LDS

// Stride-1 convolution for few input channels (the full-resolution levels):
// a workgroup computes an output brick of kBx x kBy x kBz voxels and first
// stages the input brick with its one-voxel halo, (kBx+2)(kBy+2)(kBz+2)
// voxels x CIN channels, in LDS, zero outside the grid.  Every A operand of
// the implicit GEMM is then a 16-byte LDS read instead of a global gather
// (each input voxel is read from memory about (1 + 2/16)(1 + 2/4)^2 times
// instead of 27).  M fragment = one x-row of 16 voxels; wave w owns rows
// 4w .. 4w+3 of the 16 (y, z) rows.  W and the epilogue as in k_conv.
constexpr int kBx = 16, kBy = 4, kBz = 4;
constexpr int kHx = kBx + 2, kHy = kBy + 2, kHz = kBz + 2;

template <int CIN, int NT>
__global__ __launch_bounds__(256) void k_conv_s1_lds(const bf16 *__restrict__ in, int G, int batch,
                                                     const bf16 *__restrict__ W, int Kpad, int Cout,
                                                     const float *__restrict__ bias, const bf16 *add, int relu,
                                                     bf16 *out, float *__restrict__ out32) {
    constexpr int KP = (27 * CIN + 63) / 64 * 64;  // = Kpad
    constexpr int WS = KP + 8;                      // LDS row stride of W (16-byte pad against bank conflicts)
    __shared__ __attribute__((aligned(16))) bf16 tile[kHx * kHy * kHz * CIN];
    __shared__ __attribute__((aligned(16))) bf16 wt[16 * NT * WS];
    const int nbx = (G + kBx - 1) / kBx, nby = (G + kBy - 1) / kBy, nbz = (G + kBz - 1) / kBz;
    int b = blockIdx.x;
    const int bx = b % nbx;
    b /= nbx;
    const int by = b % nby;
    b /= nby;
    const int bz = b % nbz;
    const int n = b / nbz;
    const int x0 = bx * kBx, y0 = by * kBy, z0 = bz * kBz;
    const int64_t V = (int64_t)G * G * G;
    // stage the input brick with halo: 16-byte chunks of 8 channels; every
    // load of a thread is issued before its first LDS store
    constexpr int kChunks = kHx * kHy * kHz * (CIN / 8);
    constexpr int kIters = (kChunks + 255) / 256;
    bf16x8 v[kIters];
#pragma unroll
    for (int i = 0; i < kIters; ++i) {
        const int q = threadIdx.x + 256 * i;
        const int hv = q / (CIN / 8), part = q % (CIN / 8);
        const int hx = hv % kHx, hy = (hv / kHx) % kHy, hz = hv / (kHx * kHy);
        const int gx = x0 - 1 + hx, gy = y0 - 1 + hy, gz = z0 - 1 + hz;
        v[i] = zero8();
        if (q < kChunks && gx >= 0 && gx < G && gy >= 0 && gy < G && gz >= 0 && gz < G)
            v[i] = load8(in + ((int64_t)n * V + ((int64_t)gz * G + gy) * G + gx) * CIN + part * 8);
    }
    // the layer's weight rows, 16 NT x KP, also once per workgroup
    constexpr int kWChunks = 16 * NT * (KP / 8);
    constexpr int kWIters = (kWChunks + 255) / 256;
    bf16x8 wv[kWIters];
#pragma unroll
    for (int i = 0; i < kWIters; ++i) {
        const int q = threadIdx.x + 256 * i;
        wv[i] = q < kWChunks ? load8(W + (int64_t)(q / (KP / 8)) * Kpad + (q % (KP / 8)) * 8) : zero8();
    }
#pragma unroll
    for (int i = 0; i < kIters; ++i) {
        const int q = threadIdx.x + 256 * i;
        if (q < kChunks) *(bf16x8 *)(tile + q * 8) = v[i];  // q * 8 = hv * CIN + part * 8
    }
#pragma unroll
    for (int i = 0; i < kWIters; ++i) {
        const int q = threadIdx.x + 256 * i;
        if (q < kWChunks) *(bf16x8 *)(wt + (q / (KP / 8)) * WS + (q % (KP / 8)) * 8) = wv[i];
    }
    __syncthreads();
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const int row = lane & 15, kg = lane >> 4;
    constexpr int Kreal = 27 * CIN;
    f32x4 acc[4][NT];
#pragma unroll
    for (int mt = 0; mt < 4; ++mt)
#pragma unroll
        for (int nt = 0; nt < NT; ++nt) acc[mt][nt] = (f32x4)(0.0f);
    const bf16 *Wrow = wt + row * WS;
    constexpr int nsteps = KP >> 5;
    for (int st = 0; st < nsteps; ++st) {
        const int k = st * 32 + 8 * kg;
        bf16x8 b0[NT];
#pragma unroll
        for (int nt = 0; nt < NT; ++nt) b0[nt] = *(const bf16x8 *)(Wrow + nt * 16 * WS + k);
        const int d = k / CIN, c0 = k % CIN;
        const int dx = d % 3, dy = (d / 3) % 3, dz = d / 9;
        bf16x8 a[4];
#pragma unroll
        for (int mt = 0; mt < 4; ++mt) {
            const int f = wave * 4 + mt;  // x-row (vy, vz) of the brick
            const int vy = f % kBy, vz = f / kBy;
            const int hv = ((vz + dz) * kHy + (vy + dy)) * kHx + (row + dx);
            a[mt] = k < Kreal ? *(const bf16x8 *)(tile + hv * CIN + c0) : zero8();
        }
#pragma unroll
        for (int nt = 0; nt < NT; ++nt)
#pragma unroll
            for (int mt = 0; mt < 4; ++mt)
                acc[mt][nt] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a[mt], b0[nt], acc[mt][nt], 0, 0, 0);
    }
#pragma unroll
    for (int mt = 0; mt < 4; ++mt) {
        const int f = wave * 4 + mt;
        const int gy = y0 + f % kBy, gz = z0 + f / kBy;
        if (gy >= G || gz >= G) continue;
#pragma unroll
        for (int j = 0; j < 4; ++j) {
            const int gx = x0 + 4 * kg + j;
            if (gx >= G) continue;
            const int64_t v = (int64_t)n * V + ((int64_t)gz * G + gy) * G + gx;
#pragma unroll
            for (int nt = 0; nt < NT; ++nt) {
                const int o = nt * 16 + row;
                if (o >= Cout) continue;
                float val = acc[mt][nt][j];
                const int64_t idx = v * Cout + o;
                if (bias) val += bias[o];
                if (add) val += (float)add[idx];
                if (relu) val = fmaxf(val, 0.0f);
                out[idx] = (bf16)val;
                if (out32) out32[idx] = val;
            }
        }
    }
}

// ------------------------------------------------------------------ transposed stride 2 by parity class

// Along one axis an output p = 2j + q of the t2 pattern receives tap d = 1
// from source j when q = 0, and taps d = 0 (source j + 1) and d = 2 (source
// j) when q = 1; every source is inside the grid.  Splitting the outputs
// into the 8 parity classes (qx, qy, qz) leaves each class a dense
// convolution over its (1 + qx)(1 + qy)(1 + qz) live taps: a class tap t
// enumerates (tx, ty, tz), tx in {0, qx} fastest, and the reduction index is
// t Cin + c.  Class c = qx + 2 qy + 4 qz has (Gi - qx)(Gi - qy)(Gi - qz)
// output voxels per sample.
__host__ __device__ __forceinline__ int t2_ntaps(int c) { return (1 + (c & 1)) * (1 + ((c >> 1) & 1)) * (1 + (c >> 2)); }

__host__ __device__ __forceinline__ void t2_tap(int c, int t, int &tx, int &ty, int &tz) {
    const int qx = c & 1, qy = (c >> 1) & 1, qz = c >> 2;
    tx = qx ? (t & 1) : 0;
    t = qx ? t >> 1 : t;
    ty = qy ? (t & 1) : 0;
    tz = qy ? t >> 1 : t;
    if (!qz) tz = 0;
}

// class weights: per class c, [rows][kcpad[c]] at element offset woff[c]
struct T2Layout {
    int64_t woff[9];
    int kcpad[8];
};

__host__ __device__ inline T2Layout t2_layout(int Cin, int rows) {
    T2Layout L;
    L.woff[0] = 0;
    for (int c = 0; c < 8; ++c) {
        L.kcpad[c] = (t2_ntaps(c) * Cin + 31) / 32 * 32;
        L.woff[c + 1] = L.woff[c] + (int64_t)rows * L.kcpad[c];
    }
    return L;
}

// Class matrices out of a full [rows][Kpad] matrix (reduction index d Cin + c).
__global__ __launch_bounds__(256) void k_t2_class_weights(const bf16 *__restrict__ M, int rows, int Kpad, int Cin,
                                                          T2Layout L, bf16 *__restrict__ MC) {
    const int64_t n = L.woff[8];
    for (int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x; i < n; i += (int64_t)gridDim.x * 256) {
        int c = 0;
        while (i >= L.woff[c + 1]) ++c;
        const int64_t j = i - L.woff[c];
        const int r = (int)(j / L.kcpad[c]), kk = (int)(j % L.kcpad[c]);
        const int t = kk / Cin, ch = kk % Cin;
        bf16 v = (bf16)0.0f;
        if (t < t2_ntaps(c)) {
            int tx, ty, tz;
            t2_tap(c, t, tx, ty, tz);
            const int dx = (c & 1) ? 2 * tx : 1, dy = ((c >> 1) & 1) ? 2 * ty : 1, dz = (c >> 2) ? 2 * tz : 1;
            v = M[(int64_t)r * Kpad + (dx + 3 * dy + 9 * dz) * Cin + ch];
        }
        MC[i] = v;
    }
}

// wave-tile prefix over the classes
struct T2Tiles {
    int64_t tile0[9];
};

// The t2 convolution over all parity classes in one launch: wave tiles are
// numbered class by class; otherwise as k_conv (no reduction split: a class
// has at most 8 Cin reduction indices).
template <int NT, int MT>
__global__ __launch_bounds__(256) void k_conv_t2(const bf16 *__restrict__ in, int Gi, int cin_log2,
                                                 const bf16 *__restrict__ WC, T2Layout L, T2Tiles T, int Cout,
                                                 int batch, const float *__restrict__ bias, const bf16 *add, int relu,
                                                 bf16 *out, float *__restrict__ out32) {
    const int lane = threadIdx.x & 63;
    const int64_t wave = (int64_t)blockIdx.x * 4 + (threadIdx.x >> 6);
    if (wave >= T.tile0[8]) return;
    int c = 0;
    while (wave >= T.tile0[c + 1]) ++c;
    const int qx = c & 1, qy = (c >> 1) & 1, qz = c >> 2;
    const int ex = Gi - qx, ey = Gi - qy, ez = Gi - qz;
    const int64_t cvox = (int64_t)ex * ey * ez, count = (int64_t)batch * cvox;
    const int64_t base = (wave - T.tile0[c]) * 16 * MT;
    const int Go = 2 * Gi - 1;
    const int64_t Vi = (int64_t)Gi * Gi * Gi;
    const int o0 = blockIdx.y * 16 * NT;
    const int row = lane & 15, kg = lane >> 4;
    const int Kc = t2_ntaps(c) << cin_log2, Kcpad = L.kcpad[c];
    const int cmask = (1 << cin_log2) - 1;
    // Class coordinates by 32-bit division (the launcher keeps the output
    // voxel count below 2^31), and the flat output voxel of row `row` of each
    // tile, which the epilogue fetches from that row's lane instead of
    // dividing again.
    const uint32_t uex = (uint32_t)ex, uey = (uint32_t)ey, ucv = (uint32_t)cvox;
    const uint32_t uGo = (uint32_t)Go, uVo = uGo * uGo * uGo;
    int jx[MT], jy[MT], jz[MT], ovr[MT];
    int64_t nb[MT];
    bool rv[MT];
#pragma unroll
    for (int mt = 0; mt < MT; ++mt) {
        const int64_t v = base + mt * 16 + row;
        rv[mt] = v < count;
        const uint32_t vv = rv[mt] ? (uint32_t)v : 0u;
        const uint32_t n = vv / ucv, r = vv - n * ucv, q = r / uex, z = q / uey;
        jx[mt] = (int)(r - q * uex);
        jy[mt] = (int)(q - z * uey);
        jz[mt] = (int)z;
        nb[mt] = (int64_t)n * Vi;
        ovr[mt] = (int)(n * uVo + ((2 * z + qz) * uGo + 2 * (uint32_t)jy[mt] + qy) * uGo + 2 * (uint32_t)jx[mt] + qx);
    }
    f32x4 acc[MT][NT];
#pragma unroll
    for (int mt = 0; mt < MT; ++mt)
#pragma unroll
        for (int nt = 0; nt < NT; ++nt) acc[mt][nt] = (f32x4)(0.0f);
    const bf16 *Wrow = WC + L.woff[c] + (int64_t)(o0 + row) * Kcpad;
    auto load_step = [&](int st, bf16x8(&a)[MT], bf16x8(&b)[NT]) {
        const int k = st * 32 + 8 * kg;
        const int t = k >> cin_log2, ch = k & cmask;
        int tx, ty, tz;
        t2_tap(c, t, tx, ty, tz);
        const int ox = (qx && tx == 0) ? 1 : 0, oy = (qy && ty == 0) ? 1 : 0, oz = (qz && tz == 0) ? 1 : 0;
#pragma unroll
        for (int mt = 0; mt < MT; ++mt) {
            const int64_t sv = ((int64_t)(jz[mt] + oz) * Gi + (jy[mt] + oy)) * Gi + (jx[mt] + ox);
            a[mt] = (rv[mt] && k < Kc) ? load8(in + ((nb[mt] + sv) << cin_log2) + ch) : zero8();
        }
#pragma unroll
        for (int nt = 0; nt < NT; ++nt) b[nt] = load8(Wrow + (int64_t)nt * 16 * Kcpad + k);
    };
    const int nsteps = Kcpad >> 5;
    bf16x8 a0[MT], b0[NT];
    load_step(0, a0, b0);
    for (int st = 0; st < nsteps; ++st) {
        const bool more = st + 1 < nsteps;
        bf16x8 a1[MT], b1[NT];
        if (more) load_step(st + 1, a1, b1);
#pragma unroll
        for (int nt = 0; nt < NT; ++nt)
#pragma unroll
            for (int mt = 0; mt < MT; ++mt)
                acc[mt][nt] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a0[mt], b0[nt], acc[mt][nt], 0, 0, 0);
        if (more) {
#pragma unroll
            for (int mt = 0; mt < MT; ++mt) a0[mt] = a1[mt];
#pragma unroll
            for (int nt = 0; nt < NT; ++nt) b0[nt] = b1[nt];
        }
    }
    // accumulator element j of lane (row, kg) is tile row 4 kg + j
    int ovs[MT][4];
#pragma unroll
    for (int mt = 0; mt < MT; ++mt)
#pragma unroll
        for (int j = 0; j < 4; ++j) ovs[mt][j] = __shfl(ovr[mt], 4 * kg + j, 64);
#pragma unroll
    for (int mt = 0; mt < MT; ++mt)
#pragma unroll
        for (int j = 0; j < 4; ++j) {
            const int64_t v = base + mt * 16 + 4 * kg + j;
            if (v >= count) continue;
            const int64_t ov = ovs[mt][j];
#pragma unroll
            for (int nt = 0; nt < NT; ++nt) {
                const int o = o0 + nt * 16 + row;
                if (o >= Cout) continue;
                float val = acc[mt][nt][j];
                const int64_t idx = ov * Cout + o;
                if (bias) val += bias[o];
                if (add) val += (float)add[idx];
                if (relu) val = fmaxf(val, 0.0f);
                out[idx] = (bf16)val;
                if (out32) out32[idx] = val;
            }
        }
}

// ------------------------------------------------------------------ weight gradient

// part[split][o][k] = sum over this split's voxels of gy[v][o] * X[src(v, d)][c],
// k = d Cin + c, for k in this workgroup's 64-wide block.  Tiles of 32 voxels
// are staged transposed in LDS; wave w owns k-fragment w of the block and all
// NT o-fragments.
template <int MODE, int NT>
__global__ __launch_bounds__(256) void k_wgrad(const bf16 *__restrict__ gy, int Go, int Cout,
                                               const bf16 *__restrict__ X, int Gi, int cin_log2, int Kreal,
                                               int Kpad, int64_t total, int64_t per_split,
                                               float *__restrict__ part) {
    __shared__ __attribute__((aligned(16))) bf16 gyT[16 * NT][40];
    __shared__ __attribute__((aligned(16))) bf16 xT[64][40];
    const int kb = blockIdx.x, split = blockIdx.y;
    const int64_t v_lo = (int64_t)split * per_split;
    const int64_t v_hi = v_lo + per_split < total ? v_lo + per_split : total;
    const int t = threadIdx.x, lane = t & 63, wave = t >> 6, row = lane & 15, kg = lane >> 4;
    const int64_t Vi = (int64_t)Gi * Gi * Gi;
    // voxel coordinates by 32-bit division, as in k_conv (total < 2^31)
    const uint32_t uGo = (uint32_t)Go, uVo = uGo * uGo * uGo;
    const int cmask = (1 << cin_log2) - 1;
    f32x4 acc[NT];
#pragma unroll
    for (int i = 0; i < NT; ++i) acc[i] = (f32x4)(0.0f);
    for (int64_t v0 = v_lo; v0 < v_hi; v0 += 32) {
        const int vv = t & 31, grp = t >> 5;
        const int64_t v = v0 + vv;
        // gy tile, transposed: gyT[o][voxel]
        if (grp < NT) {
#pragma unroll
            for (int q = 0; q < 16; ++q) {
                const int o = grp * 16 + q;
                gyT[o][vv] = (v < v_hi && o < Cout) ? gy[v * Cout + o] : (bf16)0.0f;
            }
        }
        // gathered input tile, transposed: xT[k][voxel]
        {
            const int k = kb * 64 + grp * 8;
            bf16x8 val = zero8();
            if (v < v_hi && k < Kreal) {
                const uint32_t uv = (uint32_t)v, n = uv / uVo, p = uv - n * uVo, q = p / uGo, z = q / uGo;
                const int px = (int)(p - q * uGo), py = (int)(q - z * uGo), pz = (int)z;
                const int64_t s = src_voxel<MODE>(pz, py, px, k >> cin_log2, Gi);
                if (s >= 0) val = load8(X + (((int64_t)n * Vi + s) << cin_log2) + (k & cmask));
            }
#pragma unroll
            for (int j = 0; j < 8; ++j) xT[grp * 8 + j][vv] = val[j];
        }
        __syncthreads();
        const bf16x8 b = *(const bf16x8 *)&xT[wave * 16 + row][8 * kg];
#pragma unroll
        for (int i = 0; i < NT; ++i) {
            const bf16x8 a = *(const bf16x8 *)&gyT[i * 16 + row][8 * kg];
            acc[i] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a, b, acc[i], 0, 0, 0);
        }
        __syncthreads();
    }
    const int k = kb * 64 + wave * 16 + row;
#pragma unroll
    for (int i = 0; i < NT; ++i)
#pragma unroll
        for (int j = 0; j < 4; ++j) {
            const int o = i * 16 + 4 * kg + j;
            part[((int64_t)split * 16 * NT + o) * Kpad + k] = acc[i][j];
        }
}

// out[i] = sum_s part[s][i], fixed order
__global__ __launch_bounds__(256) void k_sum_splits(const float *__restrict__ part, int nsplit, int64_t n,
                                                    float *__restrict__ out) {
    for (int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x; i < n; i += (int64_t)gridDim.x * 256) {
        float s = 0.0f;
        for (int q = 0; q < nsplit; ++q) s += part[(int64_t)q * n + i];
        out[i] = s;
    }
}

// bias gradient partials: part[split][o] = sum over the split's voxels of gy[v][o]
__global__ __launch_bounds__(256) void k_bias_part(const bf16 *__restrict__ gy, int Cout, int64_t total,
                                                   int64_t per_split, float *__restrict__ part) {
    __shared__ float red[256];
    const int t = threadIdx.x;
    const int o = t % Cout, r = t / Cout, R = 256 / Cout;
    const int64_t lo = (int64_t)blockIdx.x * per_split;
    const int64_t hi = lo + per_split < total ? lo + per_split : total;
    float s = 0.0f;
    if (r < R)
        for (int64_t v = lo + r; v < hi; v += R) s += (float)gy[v * Cout + o];
    red[t] = s;
    __syncthreads();
    if (t < Cout) {
        float a = 0.0f;
        for (int q = 0; q < R; ++q) a += red[q * Cout + t];
        part[(int64_t)blockIdx.x * Cout + t] = a;
    }
}

// ------------------------------------------------------------------ elementwise

__global__ __launch_bounds__(256) void k_relu_bwd(int64_t n, const bf16 *__restrict__ gy, const bf16 *__restrict__ y,
                                                  bf16 *__restrict__ g) {
    for (int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x; i < n; i += (int64_t)gridDim.x * 256)
        g[i] = (float)y[i] > 0.0f ? gy[i] : (bf16)0.0f;
}

__global__ __launch_bounds__(256) void k_add_bf16(int64_t n, bf16 *__restrict__ a, const bf16 *__restrict__ b) {
    for (int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x; i < n; i += (int64_t)gridDim.x * 256)
        a[i] = (bf16)((float)a[i] + (float)b[i]);
}

__global__ __launch_bounds__(256) void k_fill_bf16(int64_t n, bf16 *__restrict__ a) {
    for (int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x; i < n; i += (int64_t)gridDim.x * 256) a[i] = (bf16)0.0f;
}

__device__ __forceinline__ bool on_boundary(int64_t p, int G) {
    const int x = (int)(p % G), y = (int)((p / G) % G), z = (int)(p / ((int64_t)G * G));
    return x == 0 || y == 0 || z == 0 || x == G - 1 || y == G - 1 || z == G - 1;
}

// input channels: 0 boundary value (0 inside), 1 boundary mask, 2..7 zero
__global__ __launch_bounds__(256) void k_net_input(int64_t total, int G, const double *__restrict__ g,
                                                   bf16 *__restrict__ in) {
    const int64_t V = (int64_t)G * G * G;
    for (int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x; i < total; i += (int64_t)gridDim.x * 256) {
        const bool bd = on_boundary(i % V, G);
        bf16 *q = in + i * 8;
        q[0] = (bf16)(bd ? (float)g[i] : 0.0f);
        q[1] = (bf16)(bd ? 1.0f : 0.0f);
        for (int c = 2; c < 8; ++c) q[c] = (bf16)0.0f;
    }
}

// MSE over interior nodes: gradient into channel 0 of g (stride 8), partials of the squared error
__global__ __launch_bounds__(256) void k_mse(int64_t total, int G, const float *__restrict__ pred,
                                             const double *__restrict__ target, double inv_count,
                                             bf16 *__restrict__ g, double *__restrict__ part) {
    const int64_t V = (int64_t)G * G * G;
    double acc = 0.0;
    for (int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x; i < total; i += (int64_t)gridDim.x * 256) {
        double e = 0.0;
        if (!on_boundary(i % V, G)) e = (double)pred[i * 8] - target[i];
        acc += e * e;
        g[i * 8] = (bf16)(2.0 * e * inv_count);
        for (int c = 1; c < 8; ++c) g[i * 8 + c] = (bf16)0.0f;
    }
    acc = block_sum(acc);
    if (threadIdx.x == 0) part[blockIdx.x] = acc;
}

// e = prediction - target on interior nodes, 0 on boundary nodes (FP64)
__global__ __launch_bounds__(256) void k_err(int64_t total, int G, const float *__restrict__ pred,
                                             const double *__restrict__ target, double *__restrict__ e) {
    const int64_t V = (int64_t)G * G * G;
    for (int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x; i < total; i += (int64_t)gridDim.x * 256)
        e[i] = on_boundary(i % V, G) ? 0.0 : (double)pred[i * 8] - target[i];
}

// energy norm of the error: partials of e.Ae, and the output gradient 2 (Ae) / count on interior nodes
__global__ __launch_bounds__(256) void k_energy(int64_t total, int G, const double *__restrict__ e,
                                                const double *__restrict__ ae, double inv_count, bf16 *__restrict__ g,
                                                double *__restrict__ part) {
    const int64_t V = (int64_t)G * G * G;
    double acc = 0.0;
    for (int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x; i < total; i += (int64_t)gridDim.x * 256) {
        const double q = on_boundary(i % V, G) ? 0.0 : ae[i];
        acc += e[i] * q;
        g[i * 8] = (bf16)(2.0 * q * inv_count);
        for (int c = 1; c < 8; ++c) g[i * 8 + c] = (bf16)0.0f;
    }
    acc = block_sum(acc);
    if (threadIdx.x == 0) part[blockIdx.x] = acc;
}

// prediction (channel 0) out of the stride-8 output, FP32
__global__ __launch_bounds__(256) void k_pred(int64_t total, const float *__restrict__ out32, float *__restrict__ pred) {
    for (int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x; i < total; i += (int64_t)gridDim.x * 256)
        pred[i] = out32[i * 8];
}

// x0 = g on boundary nodes (exact), the prediction inside
__global__ __launch_bounds__(256) void k_net_x0(int G, const double *__restrict__ g, const float *__restrict__ out32,
                                                double *__restrict__ x0) {
    const int64_t V = (int64_t)G * G * G;
    for (int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x; i < V; i += (int64_t)gridDim.x * 256)
        x0[i] = on_boundary(i, G) ? g[i] : (double)out32[i * 8];
}

__global__ __launch_bounds__(256) void k_adam(int64_t n, float *__restrict__ p, float *__restrict__ m,
                                              float *__restrict__ v, const float *__restrict__ g, float lr, float b1,
                                              float b2, float eps, float bc1, float bc2) {
    for (int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x; i < n; i += (int64_t)gridDim.x * 256) {
        const float gi = g[i];
        const float mi = b1 * m[i] + (1.0f - b1) * gi;
        const float vi = b2 * v[i] + (1.0f - b2) * gi * gi;
        m[i] = mi;
        v[i] = vi;
        p[i] -= lr * (mi / bc1) / (sqrtf(vi / bc2) + eps);
    }
}

// bf16 copies of one layer's weights: W[o][k] (forward) and the transposed,
// tap-permuted Wa[c][d' Cout + o] = W[o][d Cin + c] (input gradient), with
// d' = 26 - d for s1 (mirrored taps) and d' = d for s2 / t2.
__global__ __launch_bounds__(256) void k_layer_weights(const float *__restrict__ W32, int Cin, int Cout, int Kpad,
                                                       int KpadA, int rowsA, int mirror, bf16 *__restrict__ W,
                                                       bf16 *__restrict__ Wa) {
    const int64_t n = (int64_t)((Cout + 15) / 16 * 16) * Kpad;
    for (int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x; i < n; i += (int64_t)gridDim.x * 256) W[i] = (bf16)W32[i];
    const int64_t na = (int64_t)rowsA * KpadA;
    for (int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x; i < na; i += (int64_t)gridDim.x * 256) {
        const int c = (int)(i / KpadA), kk = (int)(i % KpadA);
        float val = 0.0f;
        if (c < Cin && kk < 27 * Cout) {
            const int dp = kk / Cout, o = kk % Cout;
            const int d = mirror ? 26 - dp : dp;
            val = W32[(int64_t)o * Kpad + d * Cin + c];
        }
        Wa[i] = (bf16)val;
    }
}

int ilog2(int v) {
    int l = 0;
    while ((1 << l) < v) ++l;
    return l;
}

int pad64(int v) { return (v + 63) / 64 * 64; }

}  // namespace

// ------------------------------------------------------------------ host-side launchers

namespace {

int grid_of(int64_t n) {
    int64_t g = (n + 255) / 256;
    return (int)(g < 8192 ? (g < 1 ? 1 : g) : 8192);
}

// Launch shape of one convolution: wave tile (NT channel fragments, MT voxel
// fragments) and reduction splits.  Larger tiles reuse each loaded operand
// for more products; they are taken while the grid still has kConvWaves
// wavefronts, and below that the reduction is split (small grids: the deep
// levels, and batch-1 inference).
constexpr int64_t kConvWaves = 4096;
constexpr int64_t kConvWsFloats = 4 << 20;  // split workspace, floats

struct ConvPlan {
    int NT, MT, nsplit, steps;  // steps per split
};

ConvPlan conv_plan(int64_t total, int Cout, int Kpad, int64_t ws_floats) {
    const int nt = (Cout + 15) / 16;
    static const int cand[4][4][2] = {
        {{1, 4}, {1, 2}, {1, 1}, {1, 1}},  // nt = 1
        {{2, 4}, {2, 2}, {2, 1}, {1, 1}},  // nt = 2
        {{4, 2}, {2, 2}, {2, 1}, {1, 1}},  // nt = 4
        {{4, 2}, {4, 1}, {2, 1}, {1, 1}},  // nt = 8
    };
    const int row = nt == 1 ? 0 : nt == 2 ? 1 : nt == 4 ? 2 : 3;
    const int nsteps = Kpad / 32;
    ConvPlan p{1, 1, 1, nsteps};
    int64_t waves = 0;
    for (int c = 0; c < 4; ++c) {
        p.NT = cand[row][c][0];
        p.MT = cand[row][c][1];
        waves = (total + 16 * p.MT - 1) / (16 * p.MT) * (nt / p.NT);
        if (waves >= kConvWaves) return p;
    }
    // split the reduction: at least 4 steps per split, workspace permitting
    int64_t ns = (kConvWaves + waves - 1) / waves;
    ns = std::min<int64_t>(ns, std::max(1, nsteps / 4));
    const int64_t per = total * Cout;
    ns = std::min<int64_t>(ns, per > 0 ? ws_floats / per : 1);
    if (ns <= 1) return p;
    p.steps = (int)((nsteps + ns - 1) / ns);
    p.nsplit = (nsteps + p.steps - 1) / p.steps;  // every split non-empty
    return p;
}

// Channel counts the convolution kernels take (powers of two: the tiles are
// 16 channels wide, 8 for the last layer).
bool conv_channels_ok(int c) { return c == 8 || c == 16 || c == 32 || c == 64 || c == 128; }

template <int MODE>
int conv_mode(hipStream_t s, const bf16 *in, int Gi, int Cin, const bf16 *W, int Kpad, int Cout, int Go,
              int batch, const float *bias, const bf16 *add, int relu, bf16 *out, float *out32, float *ws,
              int64_t ws_floats) {
    const int64_t total = (int64_t)batch * Go * Go * Go;
    const int nt = (Cout + 15) / 16;
    if (!conv_channels_ok(Cout)) {  // k_conv_reduce takes the bias channel as i & (Cout - 1)
        set_error("conv3d: output channels must be 8, 16, 32, 64 or 128");
        return MFE_EUNSUPPORTED;
    }
    if (total >= ((int64_t)1 << 31)) {
        set_error("conv3d: 2^31 or more output voxels in one call");
        return MFE_EUNSUPPORTED;
    }
    const int cl = ilog2(Cin), Kreal = 27 * Cin;
    const ConvPlan pl = conv_plan(total, Cout, Kpad, ws ? ws_floats : 0);
    float *part = pl.nsplit > 1 ? ws : nullptr;
#define MFE_CONV_CASE(NT_, MT_)                                                                                 \
    if (pl.NT == NT_ && pl.MT == MT_) {                                                                       \
        const int64_t waves = (total + 16 * MT_ - 1) / (16 * MT_);                                            \
        const dim3 grid((unsigned)((waves + 3) / 4), (unsigned)(nt / NT_), (unsigned)pl.nsplit);              \
        hipLaunchKernelGGL((k_conv<MODE, NT_, MT_>), grid, dim3(256), 0, s, in, Gi, cl, W, Kpad, Kreal, Cout, \
                           Go, total, pl.steps, bias, add, relu, out, out32, part);                           \
    }
    MFE_CONV_CASE(1, 1)
    MFE_CONV_CASE(1, 2)
    MFE_CONV_CASE(1, 4)
    MFE_CONV_CASE(2, 1)
    MFE_CONV_CASE(2, 2)
    MFE_CONV_CASE(2, 4)
    MFE_CONV_CASE(4, 1)
    MFE_CONV_CASE(4, 2)
#undef MFE_CONV_CASE
    MFE_HIP_TRY(hipGetLastError());
    if (part) {
        const int64_t n = total * Cout;
        hipLaunchKernelGGL(k_conv_reduce, dim3(grid_of(n)), dim3(256), 0, s, part, pl.nsplit, n, Cout, bias, add,
                           relu, out, out32);
        MFE_HIP_TRY(hipGetLastError());
    }
    return MFE_OK;
}

// t2 over its parity classes (WC: class weights of t2_layout(Cin, rows))
int conv_t2(hipStream_t s, const bf16 *in, int Gi, int Cin, const bf16 *WC, int Cout, int batch,
            const float *bias, const bf16 *add, int relu, bf16 *out, float *out32) {
    const int nt = (Cout + 15) / 16;
    if (!conv_channels_ok(Cout)) {
        set_error("conv3d: output channels must be 8, 16, 32, 64 or 128");
        return MFE_EUNSUPPORTED;
    }
    const T2Layout L = t2_layout(Cin, nt * 16);
    const int64_t total = (int64_t)batch * (2 * Gi - 1) * (2 * Gi - 1) * (2 * Gi - 1);
    if (total >= ((int64_t)1 << 31)) {
        set_error("conv3d: 2^31 or more output voxels in one call");
        return MFE_EUNSUPPORTED;
    }
    const ConvPlan pl = conv_plan(total, Cout, 64, 0);  // tile shape only
    T2Tiles T;
    T.tile0[0] = 0;
    for (int c = 0; c < 8; ++c) {
        const int64_t cnt = (int64_t)batch * (Gi - (c & 1)) * (Gi - ((c >> 1) & 1)) * (Gi - (c >> 2));
        T.tile0[c + 1] = T.tile0[c] + (cnt + 16 * pl.MT - 1) / (16 * pl.MT);
    }
    const int cl = ilog2(Cin);
#define MFE_T2_CASE(NT_, MT_)                                                                                  \
    if (pl.NT == NT_ && pl.MT == MT_) {                                                                        \
        const dim3 grid((unsigned)((T.tile0[8] + 3) / 4), (unsigned)(nt / NT_));                               \
        hipLaunchKernelGGL((k_conv_t2<NT_, MT_>), grid, dim3(256), 0, s, in, Gi, cl, WC, L, T, Cout, batch, bias, \
                           add, relu, out, out32);                                                             \
    }
    MFE_T2_CASE(1, 1)
    MFE_T2_CASE(1, 2)
    MFE_T2_CASE(1, 4)
    MFE_T2_CASE(2, 1)
    MFE_T2_CASE(2, 2)
    MFE_T2_CASE(2, 4)
    MFE_T2_CASE(4, 1)
    MFE_T2_CASE(4, 2)
#undef MFE_T2_CASE
    MFE_HIP_TRY(hipGetLastError());
    return MFE_OK;
}

int build_t2_classes(hipStream_t s, const bf16 *M, int rows, int Kpad, int Cin, bf16 *MC) {
    const T2Layout L = t2_layout(Cin, rows);
    hipLaunchKernelGGL(k_t2_class_weights, dim3(grid_of(L.woff[8])), dim3(256), 0, s, M, rows, Kpad, Cin, L, MC);
    MFE_HIP_TRY(hipGetLastError());
    return MFE_OK;
}

int64_t t2_class_elems(int Cin, int rows) { return t2_layout(Cin, rows).woff[8]; }

// W: [rows][Kpad] weights; WC: their class matrices, needed for t2
// stride 1 through LDS for Cin <= 32 and Cout <= 32
int conv_s1_lds(hipStream_t s, const bf16 *in, int G, int Cin, const bf16 *W, int Kpad, int Cout, int batch,
                const float *bias, const bf16 *add, int relu, bf16 *out, float *out32) {
    const int64_t nbrick = (int64_t)batch * ((G + kBx - 1) / kBx) * ((G + kBy - 1) / kBy) * ((G + kBz - 1) / kBz);
    const dim3 grid((unsigned)nbrick);
    if (Kpad != pad64(27 * Cin)) {
        set_error("internal: weight padding does not match the LDS stride-1 convolution");
        return MFE_EINVAL;
    }
#define MFE_S1L_CASE(CI, NT_)                                                                               \
    if (Cin == CI && (Cout + 15) / 16 == NT_) {                                                            \
        hipLaunchKernelGGL((k_conv_s1_lds<CI, NT_>), grid, dim3(256), 0, s, in, G, batch, W, Kpad, Cout, bias, \
                           add, relu, out, out32);                                                        \
        MFE_HIP_TRY(hipGetLastError());                                                                    \
        return MFE_OK;                                                                                     \
    }
    MFE_S1L_CASE(8, 1)
    MFE_S1L_CASE(8, 2)
    MFE_S1L_CASE(16, 1)
    MFE_S1L_CASE(16, 2)
    MFE_S1L_CASE(32, 1)
    MFE_S1L_CASE(32, 2)
#undef MFE_S1L_CASE
    set_error("internal: no LDS stride-1 convolution for these channels");
    return MFE_EINVAL;
}

#ifndef MFE_CONV_LDS
#define MFE_CONV_LDS 1  // stride-1 convolutions with Cin, Cout <= 32 through LDS bricks
#endif

int conv(hipStream_t s, int mode, const bf16 *in, int Gi, int Cin, const bf16 *W, const bf16 *WC, int Kpad,
         int Cout, int Go, int batch, const float *bias, const bf16 *add, int relu, bf16 *out, float *out32,
         float *ws, int64_t ws_floats) {
    if (MFE_CONV_LDS && mode == kS1 && Cin <= 32 && Cout <= 32)
        return conv_s1_lds(s, in, Gi, Cin, W, Kpad, Cout, batch, bias, add, relu, out, out32);
    if (mode == kS1)
        return conv_mode<kS1>(s, in, Gi, Cin, W, Kpad, Cout, Go, batch, bias, add, relu, out, out32, ws, ws_floats);
    if (mode == kS2)
        return conv_mode<kS2>(s, in, Gi, Cin, W, Kpad, Cout, Go, batch, bias, add, relu, out, out32, ws, ws_floats);
    if (!WC) {
        set_error("internal: t2 convolution without class weights");
        return MFE_EINVAL;
    }
    return conv_t2(s, in, Gi, Cin, WC, Cout, batch, bias, add, relu, out, out32);
}

// number of voxel splits of a weight-gradient launch
int wgrad_splits(int64_t total, int kblocks) {
    int64_t s = 2048 / (kblocks > 0 ? kblocks : 1);
    const int64_t max_by_work = (total + 255) / 256;  // at least 256 voxels per split
    if (s > max_by_work) s = max_by_work;
    return (int)(s < 1 ? 1 : s);
}

template <int MODE>
int wgrad_mode(hipStream_t s, const bf16 *gy, int Go, int Cout, const bf16 *X, int Gi, int Cin, int Kpad, int batch,
               float *part, int nsplit) {
    const int64_t total = (int64_t)batch * Go * Go * Go;
    if (total >= ((int64_t)1 << 31)) {
        set_error("conv3d weight gradient: 2^31 or more output voxels in one call");
        return MFE_EUNSUPPORTED;
    }
    const int64_t per = ((total + nsplit - 1) / nsplit + 31) / 32 * 32;
    const int nt = (Cout + 15) / 16, cl = ilog2(Cin);
    const dim3 grid(Kpad / 64, nsplit);
#define MFE_WG_CASE(NT_)                                                                                      \
    hipLaunchKernelGGL((k_wgrad<MODE, NT_>), grid, dim3(256), 0, s, gy, Go, Cout, X, Gi, cl, 27 * Cin, Kpad, \
                       total, per, part);
    if (nt == 1) MFE_WG_CASE(1)
    else if (nt == 2) MFE_WG_CASE(2)
    else if (nt == 4) MFE_WG_CASE(4)
    else if (nt == 8) MFE_WG_CASE(8)
    else {
        set_error("conv3d weight gradient: output channels must be 8, 16, 32, 64 or 128");
        return MFE_EUNSUPPORTED;
    }
#undef MFE_WG_CASE
    MFE_HIP_TRY(hipGetLastError());
    return MFE_OK;
}

int wgrad(hipStream_t s, int mode, const bf16 *gy, int Go, int Cout, const bf16 *X, int Gi, int Cin, int Kpad,
          int batch, float *part, int nsplit) {
    if (mode == kS1) return wgrad_mode<kS1>(s, gy, Go, Cout, X, Gi, Cin, Kpad, batch, part, nsplit);
    if (mode == kS2) return wgrad_mode<kS2>(s, gy, Go, Cout, X, Gi, Cin, Kpad, batch, part, nsplit);
    return wgrad_mode<kT2>(s, gy, Go, Cout, X, Gi, Cin, Kpad, batch, part, nsplit);
}

int out_size(int G, int mode) { return mode == kS1 ? G : mode == kS2 ? (G - 1) / 2 + 1 : 2 * (G - 1) + 1; }
int adjoint_mode(int mode) { return mode == kS1 ? kS1 : mode == kS2 ? kT2 : kS2; }

bool valid_channels(int c) { return c == 8 || c == 16 || c == 32 || c == 64 || c == 128; }

}  // namespace
}  // namespace mfe

using namespace mfe;

// ------------------------------------------------------------------ the network object

namespace {

struct LayerDef {
    int cin, cout, mode, relu, skip;
};
// encoder 8 -> 16 -> 32 -> 64 -> 128 (three stride-2 levels), decoder by
// transposed stride-2 convolutions with skip connections added before the ReLU
const LayerDef kLayers[] = {
    {8, 16, kS1, 1, -1},    {16, 16, kS1, 1, -1},  {16, 32, kS2, 1, -1}, {32, 32, kS1, 1, -1},
    {32, 64, kS2, 1, -1},   {64, 64, kS1, 1, -1},  {64, 128, kS2, 1, -1}, {128, 128, kS1, 1, -1},
    {128, 64, kT2, 1, 5},   {64, 64, kS1, 1, -1},  {64, 32, kT2, 1, 3},  {32, 32, kS1, 1, -1},
    {32, 16, kT2, 1, 1},    {16, 8, kS1, 0, -1},
};
constexpr int kNumLayers = sizeof(kLayers) / sizeof(kLayers[0]);

struct Layer {
    LayerDef def;
    int Gi, Go;
    int Kpad, rows;     // forward weights [rows][Kpad]
    int KpadA, rowsA;   // input-gradient weights [rowsA][KpadA]
    int64_t woff, boff; // offsets (floats) of W and b in the master parameter buffer
    Buffer act, gact, w, wa;
    Buffer wc;          // class matrices of W (t2 layers) or of Wa (s2 layers, whose adjoint is t2)
};

}  // namespace

struct mfe_net {
    mfe_ctx *ctx = nullptr;
    int G = 0, bmax = 0;
    Layer L[kNumLayers];
    int64_t nparam_dev = 0;  // padded device layout
    int64_t nparam = 0;      // natural layout [o][27][c] + b per layer
    Buffer p32, g32, m32, v32, in, out32, gpre, part, bpart, lpart;
    Buffer err, aerr;  // energy-norm loss: e and A e, FP64 [batch_max][G^3] (allocated on first use)
    int64_t part_floats = 0, bpart_floats = 0;
    int64_t step = 0;
    std::vector<std::pair<int, hipGraphExec_t>> fwd_graphs, bwd_graphs;  // per batch size
};

namespace {

int64_t voxels(int G) { return (int64_t)G * G * G; }

int upload_weights(mfe_net *N) {
    hipStream_t s = N->ctx->stream;
    for (auto &l : N->L) {
        const int64_t n = std::max((int64_t)l.rows * l.Kpad, (int64_t)l.rowsA * l.KpadA);
        hipLaunchKernelGGL(k_layer_weights, dim3(grid_of(n)), dim3(256), 0, s, (const float *)N->p32.ptr + l.woff,
                           l.def.cin, l.def.cout, l.Kpad, l.KpadA, l.rowsA, l.def.mode == kS1 ? 1 : 0,
                           (bf16 *)l.w.ptr, (bf16 *)l.wa.ptr);
        MFE_HIP_TRY(hipGetLastError());
        if (l.def.mode == kT2)
            MFE_TRY(build_t2_classes(s, (const bf16 *)l.w.ptr, l.rows, l.Kpad, l.def.cin, (bf16 *)l.wc.ptr));
        else if (l.def.mode == kS2)
            MFE_TRY(build_t2_classes(s, (const bf16 *)l.wa.ptr, l.rowsA, l.KpadA, l.def.cout, (bf16 *)l.wc.ptr));
    }
    return MFE_OK;
}

// The layer stack, from the staged input to out32.
int forward_layers(mfe_net *N, int batch, hipStream_t s) {
    for (int li = 0; li < kNumLayers; ++li) {
        Layer &l = N->L[li];
        const bf16 *x = li == 0 ? (const bf16 *)N->in.ptr : (const bf16 *)N->L[li - 1].act.ptr;
        const bf16 *add = l.def.skip >= 0 ? (const bf16 *)N->L[l.def.skip].act.ptr : nullptr;
        MFE_TRY(conv(s, l.def.mode, x, l.Gi, l.def.cin, (const bf16 *)l.w.ptr, (const bf16 *)l.wc.ptr, l.Kpad,
                     l.def.cout, l.Go, batch,
                     (const float *)N->p32.ptr + l.boff, add, l.def.relu, (bf16 *)l.act.ptr,
                     li == kNumLayers - 1 ? (float *)N->out32.ptr : nullptr, (float *)N->part.ptr,
                     N->part_floats));
    }
    return MFE_OK;
}

// Backward pass into g32 (padded device layout).  gact of the last layer holds dL/dout.
int backward(mfe_net *N, int batch, hipStream_t s) {
    for (int li = 0; li < kNumLayers - 1; ++li) {
        const int64_t n = (int64_t)batch * voxels(N->L[li].Go) * N->L[li].def.cout;
        hipLaunchKernelGGL(k_fill_bf16, dim3(grid_of(n)), dim3(256), 0, s, n, (bf16 *)N->L[li].gact.ptr);
    }
    for (int li = kNumLayers - 1; li >= 0; --li) {
        Layer &l = N->L[li];
        const int64_t total = (int64_t)batch * voxels(l.Go);
        const int64_t n = total * l.def.cout;
        const bf16 *gp = (const bf16 *)l.gact.ptr;
        if (l.def.relu) {
            hipLaunchKernelGGL(k_relu_bwd, dim3(grid_of(n)), dim3(256), 0, s, n, (const bf16 *)l.gact.ptr,
                               (const bf16 *)l.act.ptr, (bf16 *)N->gpre.ptr);
            MFE_HIP_TRY(hipGetLastError());
            gp = (const bf16 *)N->gpre.ptr;
        }
        const bf16 *x = li == 0 ? (const bf16 *)N->in.ptr : (const bf16 *)N->L[li - 1].act.ptr;
        // weight gradient
        const int nsplit = wgrad_splits(total, l.Kpad / 64);
        MFE_TRY(wgrad(s, l.def.mode, gp, l.Go, l.def.cout, x, l.Gi, l.def.cin, l.Kpad, batch, (float *)N->part.ptr,
                      nsplit));
        const int64_t nw = (int64_t)l.rows * l.Kpad;
        hipLaunchKernelGGL(k_sum_splits, dim3(grid_of(nw)), dim3(256), 0, s, (const float *)N->part.ptr, nsplit, nw,
                           (float *)N->g32.ptr + l.woff);
        // bias gradient
        const int bs = (int)std::min<int64_t>(1024, (total + 255) / 256);
        const int64_t per = (total + bs - 1) / bs;
        hipLaunchKernelGGL(k_bias_part, dim3(bs), dim3(256), 0, s, gp, l.def.cout, total, per,
                           (float *)N->bpart.ptr);
        hipLaunchKernelGGL(k_sum_splits, dim3(1), dim3(256), 0, s, (const float *)N->bpart.ptr, bs,
                           (int64_t)l.def.cout, (float *)N->g32.ptr + l.boff);
        MFE_HIP_TRY(hipGetLastError());
        // gradient into the skip source
        if (l.def.skip >= 0) {
            hipLaunchKernelGGL(k_add_bf16, dim3(grid_of(n)), dim3(256), 0, s, n, (bf16 *)N->L[l.def.skip].gact.ptr,
                               gp);
            MFE_HIP_TRY(hipGetLastError());
        }
        // input gradient, accumulated into the previous layer's output gradient
        if (li > 0) {
            bf16 *gx = (bf16 *)N->L[li - 1].gact.ptr;
            MFE_TRY(conv(s, adjoint_mode(l.def.mode), gp, l.Go, l.def.cout, (const bf16 *)l.wa.ptr,
                         (const bf16 *)l.wc.ptr, l.KpadA,
                         l.def.cin, l.Gi, batch, nullptr, gx, 0, gx, nullptr, (float *)N->part.ptr,
                         N->part_floats));
        }
    }
    return MFE_OK;
}

// The forward layer stack and the backward pass launch a few dozen kernels
// each; per batch size they are captured once into HIP graphs and replayed
// (every buffer they touch is owned by the net, so the graphs stay valid for
// its lifetime; weights are read at replay).
int net_graph(mfe_net *N, bool bwd, int batch, hipGraphExec_t *out) {
    auto &cache = bwd ? N->bwd_graphs : N->fwd_graphs;
    for (auto &e : cache)
        if (e.first == batch) {
            *out = e.second;
            return MFE_OK;
        }
    hipStream_t cs = N->ctx->cap_stream;
    MFE_HIP_TRY(hipStreamBeginCapture(cs, hipStreamCaptureModeThreadLocal));
    const int rc = bwd ? backward(N, batch, cs) : forward_layers(N, batch, cs);
    hipGraph_t g = nullptr;
    const hipError_t e = hipStreamEndCapture(cs, &g);
    if (rc != MFE_OK || e != hipSuccess) {
        if (g) (void)hipGraphDestroy(g);
        if (rc != MFE_OK) return rc;
        set_error(std::string("hipStreamEndCapture failed: ") + hipGetErrorString(e));
        return MFE_EHIP;
    }
    hipGraphExec_t ex = nullptr;
    const hipError_t e2 = hipGraphInstantiate(&ex, g, nullptr, nullptr, 0);
    (void)hipGraphDestroy(g);
    if (e2 != hipSuccess) {
        set_error(std::string("hipGraphInstantiate failed: ") + hipGetErrorString(e2));
        return MFE_EHIP;
    }
    cache.push_back({batch, ex});
    *out = ex;
    return MFE_OK;
}

int run_net_graph(mfe_net *N, bool bwd, int batch) {
    hipGraphExec_t ex = nullptr;
    MFE_TRY(net_graph(N, bwd, batch, &ex));
    MFE_HIP_TRY(hipGraphLaunch(ex, N->ctx->stream));
    return MFE_OK;
}

// Stage the boundary data as the network input, then run the layer stack.
int forward(mfe_net *N, int batch, const double *g) {
    hipStream_t s = N->ctx->stream;
    const int64_t total = (int64_t)batch * voxels(N->G);
    hipLaunchKernelGGL(k_net_input, dim3(grid_of(total)), dim3(256), 0, s, total, N->G, g, (bf16 *)N->in.ptr);
    MFE_HIP_TRY(hipGetLastError());
    return run_net_graph(N, false, batch);
}

int check_net(const mfe_net *N, int batch) {
    if (!N || batch < 1 || batch > N->bmax) {
        set_error("net is NULL or batch outside 1..batch_max");
        return MFE_EINVAL;
    }
    return MFE_OK;
}

// natural layout <-> padded device layout (host side)
void natural_to_dev(const mfe_net *N, const float *nat, std::vector<float> &dev) {
    dev.assign(N->nparam_dev, 0.0f);
    int64_t q = 0;
    for (const auto &l : N->L) {
        const int ci = l.def.cin, co = l.def.cout;
        for (int o = 0; o < co; ++o)
            for (int d = 0; d < 27; ++d)
                for (int c = 0; c < ci; ++c) dev[l.woff + (int64_t)o * l.Kpad + d * ci + c] = nat[q++];
        for (int o = 0; o < co; ++o) dev[l.boff + o] = nat[q++];
    }
}

void dev_to_natural(const mfe_net *N, const std::vector<float> &dev, float *nat) {
    int64_t q = 0;
    for (const auto &l : N->L) {
        const int ci = l.def.cin, co = l.def.cout;
        for (int o = 0; o < co; ++o)
            for (int d = 0; d < 27; ++d)
                for (int c = 0; c < ci; ++c) nat[q++] = dev[l.woff + (int64_t)o * l.Kpad + d * ci + c];
        for (int o = 0; o < co; ++o) nat[q++] = dev[l.boff + o];
    }
}

}  // namespace

extern "C" {

int mfe_net_create(mfe_ctx *ctx, int G, int batch_max, mfe_net **out) {
    clear_error();
    if (!ctx || !out || G < 9 || (G - 1) % 8 != 0 || batch_max < 1) {
        set_error("need ctx, out, G >= 9 with G - 1 divisible by 8, batch_max >= 1");
        return MFE_EINVAL;
    }
    *out = nullptr;
    if (hipSetDevice(ctx->device) != hipSuccess) return MFE_EHIP;
    mfe_net *N = new (std::nothrow) mfe_net();
    if (!N) return MFE_ENOMEM;
    N->ctx = ctx;
    N->G = G;
    N->bmax = batch_max;
    int Gc = G;
    int64_t off = 0, nat = 0, max_part = 0, max_act = 0;
    for (int li = 0; li < kNumLayers; ++li) {
        Layer &l = N->L[li];
        l.def = kLayers[li];
        l.Gi = Gc;
        l.Go = out_size(Gc, l.def.mode);
        Gc = l.Go;
        l.Kpad = pad64(27 * l.def.cin);
        l.rows = (l.def.cout + 15) / 16 * 16;
        l.KpadA = pad64(27 * l.def.cout);
        l.rowsA = (l.def.cin + 15) / 16 * 16;
        l.woff = off;
        off += (int64_t)l.rows * l.Kpad;
        l.boff = off;
        off += (l.def.cout + 3) / 4 * 4;
        nat += (int64_t)l.def.cout * 27 * l.def.cin + l.def.cout;
        const int nsplit = wgrad_splits((int64_t)batch_max * voxels(l.Go), l.Kpad / 64);
        max_part = std::max(max_part, (int64_t)nsplit * l.rows * l.Kpad);
        max_act = std::max(max_act, (int64_t)batch_max * voxels(l.Go) * l.def.cout);
    }
    N->nparam_dev = off;
    N->nparam = nat;
    int rc = MFE_OK;
    auto A = [&](Buffer *b, size_t bytes) {
        if (rc == MFE_OK) rc = dev_alloc(ctx, b, bytes);
    };
    for (auto &l : N->L) {
        const int64_t n = (int64_t)batch_max * voxels(l.Go) * l.def.cout;
        A(&l.act, n * sizeof(bf16));
        A(&l.gact, n * sizeof(bf16));
        A(&l.w, (size_t)l.rows * l.Kpad * sizeof(bf16));
        A(&l.wa, (size_t)l.rowsA * l.KpadA * sizeof(bf16));
        if (l.def.mode == kT2) A(&l.wc, (size_t)t2_class_elems(l.def.cin, l.rows) * sizeof(bf16));
        if (l.def.mode == kS2) A(&l.wc, (size_t)t2_class_elems(l.def.cout, l.rowsA) * sizeof(bf16));
    }
    A(&N->p32, off * sizeof(float));
    A(&N->g32, off * sizeof(float));
    A(&N->m32, off * sizeof(float));
    A(&N->v32, off * sizeof(float));
    A(&N->in, (size_t)batch_max * voxels(G) * 8 * sizeof(bf16));
    A(&N->out32, (size_t)batch_max * voxels(G) * 8 * sizeof(float));
    A(&N->gpre, max_act * sizeof(bf16));
    max_part = std::max<int64_t>(max_part, kConvWsFloats);
    N->part_floats = max_part;
    A(&N->part, max_part * sizeof(float));
    A(&N->bpart, 1024 * 128 * sizeof(float));
    A(&N->lpart, 8192 * sizeof(double));
    if (rc == MFE_OK) {
        hipStream_t s = ctx->stream;
        for (Buffer *b : {&N->p32, &N->g32, &N->m32, &N->v32})
            if (hipMemsetAsync(b->ptr, 0, b->bytes, s) != hipSuccess) rc = MFE_EHIP;
        if (rc == MFE_OK && upload_weights(N) != MFE_OK) rc = MFE_EHIP;
        if (rc == MFE_OK && hipStreamSynchronize(s) != hipSuccess) rc = MFE_EHIP;
    }
    if (rc != MFE_OK) {
        mfe_net_destroy(N);
        return rc;
    }
    ctx->nets.push_back(N);
    *out = N;
    return MFE_OK;
}

int mfe_net_destroy(mfe_net *N) {
    if (!N) return MFE_OK;
    mfe_ctx *ctx = N->ctx;
    (void)hipSetDevice(ctx->device);
    (void)hipStreamSynchronize(ctx->stream);
    for (auto *c : {&N->fwd_graphs, &N->bwd_graphs})
        for (auto &e : *c) (void)hipGraphExecDestroy(e.second);
    for (auto &l : N->L)
        for (Buffer *b : {&l.act, &l.gact, &l.w, &l.wa, &l.wc}) dev_free(ctx, b);
    for (Buffer *b : {&N->p32, &N->g32, &N->m32, &N->v32, &N->in, &N->out32, &N->gpre, &N->part, &N->bpart, &N->lpart,
                      &N->err, &N->aerr})
        dev_free(ctx, b);
    unregister(ctx->nets, N);
    delete N;
    return MFE_OK;
}

int mfe_net_num_params(const mfe_net *N, int64_t *n) {
    clear_error();
    if (!N || !n) {
        set_error("net and n must be non-NULL");
        return MFE_EINVAL;
    }
    *n = N->nparam;
    return MFE_OK;
}

int mfe_net_set_params(mfe_net *N, const float *params_host) {
    clear_error();
    if (!N || !params_host) {
        set_error("net and params must be non-NULL");
        return MFE_EINVAL;
    }
    if (hipSetDevice(N->ctx->device) != hipSuccess) return MFE_EHIP;
    std::vector<float> dev;
    natural_to_dev(N, params_host, dev);
    hipStream_t s = N->ctx->stream;
    MFE_HIP_TRY(hipMemcpyAsync(N->p32.ptr, dev.data(), dev.size() * sizeof(float), hipMemcpyHostToDevice, s));
    MFE_HIP_TRY(hipMemsetAsync(N->m32.ptr, 0, N->m32.bytes, s));
    MFE_HIP_TRY(hipMemsetAsync(N->v32.ptr, 0, N->v32.bytes, s));
    N->step = 0;
    MFE_TRY(upload_weights(N));
    MFE_HIP_TRY(hipStreamSynchronize(s));
    return MFE_OK;
}

int mfe_net_get_params(const mfe_net *N, float *params_host) {
    clear_error();
    if (!N || !params_host) {
        set_error("net and params must be non-NULL");
        return MFE_EINVAL;
    }
    std::vector<float> dev(N->nparam_dev);
    MFE_HIP_TRY(hipMemcpyAsync(dev.data(), N->p32.ptr, dev.size() * sizeof(float), hipMemcpyDeviceToHost,
                               N->ctx->stream));
    MFE_HIP_TRY(hipStreamSynchronize(N->ctx->stream));
    dev_to_natural(N, dev, params_host);
    return MFE_OK;
}

int mfe_net_forward(mfe_net *N, int batch, const double *g_dev, float *pred_dev) {
    clear_error();
    MFE_TRY(check_net(N, batch));
    if (!g_dev) {
        set_error("g must be non-NULL");
        return MFE_EINVAL;
    }
    if (hipSetDevice(N->ctx->device) != hipSuccess) return MFE_EHIP;
    MFE_TRY(forward(N, batch, g_dev));
    if (pred_dev) {
        const int64_t total = (int64_t)batch * voxels(N->G);
        hipLaunchKernelGGL(k_pred, dim3(grid_of(total)), dim3(256), 0, N->ctx->stream, total,
                           (const float *)N->out32.ptr, pred_dev);
        MFE_HIP_TRY(hipGetLastError());
    }
    return MFE_OK;
}

namespace {

// Backward pass from the output gradient the loss kernel left in the last layer's gact, then the loss
// (sum of lg block partials / count) and the parameter gradient back to the host when asked for.
int finish_loss_grad(mfe_net *N, int batch, int lg, double count, double *loss_host, float *grad_host) {
    hipStream_t s = N->ctx->stream;
    MFE_TRY(run_net_graph(N, true, batch));
    if (loss_host) {
        std::vector<double> lp(lg);
        MFE_HIP_TRY(hipMemcpyAsync(lp.data(), N->lpart.ptr, lg * sizeof(double), hipMemcpyDeviceToHost, s));
        MFE_HIP_TRY(hipStreamSynchronize(s));
        double acc = 0.0;
        for (double v : lp) acc += v;
        *loss_host = acc / count;
    }
    if (grad_host) {
        std::vector<float> dev(N->nparam_dev);
        MFE_HIP_TRY(hipMemcpyAsync(dev.data(), N->g32.ptr, dev.size() * sizeof(float), hipMemcpyDeviceToHost, s));
        MFE_HIP_TRY(hipStreamSynchronize(s));
        dev_to_natural(N, dev, grad_host);
    }
    return MFE_OK;
}

}  // namespace

int mfe_net_loss_grad(mfe_net *N, int batch, const double *g_dev, const double *target_dev, double *loss_host,
                      float *grad_host) {
    clear_error();
    MFE_TRY(check_net(N, batch));
    if (!g_dev || !target_dev) {
        set_error("g and target must be non-NULL");
        return MFE_EINVAL;
    }
    if (hipSetDevice(N->ctx->device) != hipSuccess) return MFE_EHIP;
    hipStream_t s = N->ctx->stream;
    MFE_TRY(forward(N, batch, g_dev));
    const int64_t total = (int64_t)batch * voxels(N->G);
    const int64_t inner = (int64_t)(N->G - 2) * (N->G - 2) * (N->G - 2);
    const int lg = std::min(1024, grid_of(total));
    hipLaunchKernelGGL(k_mse, dim3(lg), dim3(256), 0, s, total, N->G, (const float *)N->out32.ptr, target_dev,
                       1.0 / ((double)batch * inner), (bf16 *)N->L[kNumLayers - 1].gact.ptr, (double *)N->lpart.ptr);
    MFE_HIP_TRY(hipGetLastError());
    return finish_loss_grad(N, batch, lg, (double)batch * inner, loss_host, grad_host);
}

int mfe_net_loss_grad_energy(mfe_net *N, const mfe_problem *A, int format, int batch, const double *g_dev,
                             const double *target_dev, double *loss_host, float *grad_host) {
    clear_error();
    MFE_TRY(check_net(N, batch));
    if (!A || !g_dev || !target_dev) {
        set_error("problem, g and target must be non-NULL");
        return MFE_EINVAL;
    }
    if (A->ctx != N->ctx || !A->is_mesh || A->Nx != N->G - 1 || A->Ny != N->G - 1 || A->Nz != N->G - 1) {
        set_error("the problem must be the (G-1)^3 element box mesh of the network's grid, on its context");
        return MFE_EINVAL;
    }
    if ((format != MFE_CSR && format != MFE_BCRS13) || !(A->formats & format)) {
        set_error("format must be MFE_CSR or MFE_BCRS13 and built for the problem");
        return MFE_EINVAL;
    }
    if (hipSetDevice(N->ctx->device) != hipSuccess) return MFE_EHIP;
    hipStream_t s = N->ctx->stream;
    const int64_t V = voxels(N->G);
    const size_t bytes = (size_t)N->bmax * V * sizeof(double);
    if (!N->err.ptr) MFE_TRY(dev_alloc(N->ctx, &N->err, bytes));
    if (!N->aerr.ptr) MFE_TRY(dev_alloc(N->ctx, &N->aerr, bytes));
    MFE_TRY(forward(N, batch, g_dev));
    const int64_t total = (int64_t)batch * V;
    const int64_t inner = (int64_t)(N->G - 2) * (N->G - 2) * (N->G - 2);
    double *e = (double *)N->err.ptr, *ae = (double *)N->aerr.ptr;
    hipLaunchKernelGGL(k_err, dim3(grid_of(total)), dim3(256), 0, s, total, N->G, (const float *)N->out32.ptr,
                       target_dev, e);
    MFE_HIP_TRY(hipGetLastError());
    for (int b = 0; b < batch; ++b) {
        SpmvArgs a{e + (int64_t)b * V, ae + (int64_t)b * V, nullptr, nullptr, nullptr, nullptr};
        MFE_TRY(launch_spmv(A, format, false, kSpmvPlain, a, s));
    }
    const int lg = std::min(1024, grid_of(total));
    hipLaunchKernelGGL(k_energy, dim3(lg), dim3(256), 0, s, total, N->G, (const double *)e, (const double *)ae,
                       1.0 / ((double)batch * inner), (bf16 *)N->L[kNumLayers - 1].gact.ptr, (double *)N->lpart.ptr);
    MFE_HIP_TRY(hipGetLastError());
    return finish_loss_grad(N, batch, lg, (double)batch * inner, loss_host, grad_host);
}

int mfe_net_set_grad(mfe_net *N, const float *grad_host) {
    clear_error();
    if (!N || !grad_host) {
        set_error("net and grad must be non-NULL");
        return MFE_EINVAL;
    }
    if (hipSetDevice(N->ctx->device) != hipSuccess) return MFE_EHIP;
    std::vector<float> dev;
    natural_to_dev(N, grad_host, dev);
    hipStream_t s = N->ctx->stream;
    MFE_HIP_TRY(hipMemcpyAsync(N->g32.ptr, dev.data(), dev.size() * sizeof(float), hipMemcpyHostToDevice, s));
    MFE_HIP_TRY(hipStreamSynchronize(s));
    return MFE_OK;
}

int mfe_net_adam_step(mfe_net *N, float lr, float beta1, float beta2, float eps) {
    clear_error();
    if (!N || !(lr >= 0.0f) || !(beta1 >= 0.0f && beta1 < 1.0f) || !(beta2 >= 0.0f && beta2 < 1.0f) || !(eps > 0.0f)) {
        set_error("need net, lr >= 0, 0 <= beta1, beta2 < 1, eps > 0");
        return MFE_EINVAL;
    }
    if (hipSetDevice(N->ctx->device) != hipSuccess) return MFE_EHIP;
    N->step += 1;
    const float bc1 = 1.0f - std::pow(beta1, (float)N->step), bc2 = 1.0f - std::pow(beta2, (float)N->step);
    hipLaunchKernelGGL(k_adam, dim3(grid_of(N->nparam_dev)), dim3(256), 0, N->ctx->stream, N->nparam_dev,
                       (float *)N->p32.ptr, (float *)N->m32.ptr, (float *)N->v32.ptr, (const float *)N->g32.ptr, lr,
                       beta1, beta2, eps, bc1, bc2);
    MFE_HIP_TRY(hipGetLastError());
    return upload_weights(N);
}

int mfe_net_predict_x0(mfe_net *N, const double *g_dev, double *x0_dev) {
    clear_error();
    MFE_TRY(check_net(N, 1));
    if (!g_dev || !x0_dev) {
        set_error("g and x0 must be non-NULL");
        return MFE_EINVAL;
    }
    if (hipSetDevice(N->ctx->device) != hipSuccess) return MFE_EHIP;
    MFE_TRY(forward(N, 1, g_dev));
    hipLaunchKernelGGL(k_net_x0, dim3(grid_of(voxels(N->G))), dim3(256), 0, N->ctx->stream, N->G, g_dev,
                       (const float *)N->out32.ptr, x0_dev);
    MFE_HIP_TRY(hipGetLastError());
    return MFE_OK;
}

int mfe_conv3d_bf16(mfe_ctx *ctx, int mode, int batch, int Gi, int cin, const void *in_dev, int cout,
                    const float *w_host, const float *bias_host, int relu, void *out_dev, float *out32_dev) {
    clear_error();
    if (!ctx || !in_dev || !w_host || !out_dev || batch < 1 || Gi < 2 || mode < 0 || mode > 2 ||
        !valid_channels(cin) || !valid_channels(cout)) {
        set_error("need ctx, in, w, out, batch >= 1, Gi >= 2, mode 0..2, channels in {8, 16, 32, 64, 128}");
        return MFE_EINVAL;
    }
    if (hipSetDevice(ctx->device) != hipSuccess) return MFE_EHIP;
    const int Kpad = pad64(27 * cin), rows = (cout + 15) / 16 * 16;
    std::vector<bf16> w((size_t)rows * Kpad, (bf16)0.0f);
    for (int o = 0; o < cout; ++o)
        for (int k = 0; k < 27 * cin; ++k) w[(size_t)o * Kpad + k] = (bf16)w_host[(size_t)o * 27 * cin + k];
    Buffer wb, bb, ws, wc;
    int rc = dev_alloc(ctx, &wb, w.size() * sizeof(bf16));
    if (rc == MFE_OK) rc = dev_alloc(ctx, &bb, cout * sizeof(float));
    if (rc == MFE_OK) rc = dev_alloc(ctx, &ws, kConvWsFloats * sizeof(float));
    if (rc == MFE_OK && mode == kT2) rc = dev_alloc(ctx, &wc, t2_class_elems(cin, rows) * sizeof(bf16));
    hipStream_t s = ctx->stream;
    if (rc == MFE_OK &&
        (hipMemcpyAsync(wb.ptr, w.data(), w.size() * sizeof(bf16), hipMemcpyHostToDevice, s) != hipSuccess ||
         (bias_host && hipMemcpyAsync(bb.ptr, bias_host, cout * sizeof(float), hipMemcpyHostToDevice, s) != hipSuccess)))
        rc = MFE_EHIP;
    if (rc == MFE_OK && mode == kT2) rc = build_t2_classes(s, (const bf16 *)wb.ptr, rows, Kpad, cin, (bf16 *)wc.ptr);
    if (rc == MFE_OK)
        rc = conv(s, mode, (const bf16 *)in_dev, Gi, cin, (const bf16 *)wb.ptr, (const bf16 *)wc.ptr, Kpad, cout,
                  out_size(Gi, mode), batch,
                  bias_host ? (const float *)bb.ptr : nullptr, nullptr, relu, (bf16 *)out_dev, out32_dev,
                  (float *)ws.ptr, kConvWsFloats);
    if (hipStreamSynchronize(s) != hipSuccess && rc == MFE_OK) rc = MFE_EHIP;
    dev_free(ctx, &wb);
    dev_free(ctx, &bb);
    dev_free(ctx, &ws);
    dev_free(ctx, &wc);
    return rc;
}

int mfe_conv3d_dgrad_bf16(mfe_ctx *ctx, int mode, int batch, int Gi, int cin, const void *gy_dev, int cout,
                          const float *w_host, int accumulate, void *gx_dev, float *gx32_dev) {
    clear_error();
    if (!ctx || !gy_dev || !w_host || !gx_dev || batch < 1 || Gi < 2 || mode < 0 || mode > 2 ||
        !valid_channels(cin) || !valid_channels(cout) || (accumulate != 0 && accumulate != 1)) {
        set_error("need ctx, gy, w, gx, batch >= 1, Gi >= 2, mode 0..2, channels in {8, 16, 32, 64, 128}, "
                  "accumulate 0 or 1");
        return MFE_EINVAL;
    }
    const int Go = out_size(Gi, mode);
    if (out_size(Go, adjoint_mode(mode)) != Gi) {
        set_error("the adjoint of a stride-2 convolution maps back onto the input grid only for odd Gi");
        return MFE_EINVAL;
    }
    if (hipSetDevice(ctx->device) != hipSuccess) return MFE_EHIP;
    // the network's own weight preparation: FP32 master [rows][Kpad] -> bf16
    // W and the (o, c)-transposed, tap-permuted Wa, and for s2 the class
    // matrices of Wa (its adjoint is a transposed stride-2 convolution)
    const int Kpad = pad64(27 * cin), rows = (cout + 15) / 16 * 16;
    const int KpadA = pad64(27 * cout), rowsA = (cin + 15) / 16 * 16;
    std::vector<float> w32((size_t)rows * Kpad, 0.0f);
    for (int o = 0; o < cout; ++o)
        for (int k = 0; k < 27 * cin; ++k) w32[(size_t)o * Kpad + k] = w_host[(size_t)o * 27 * cin + k];
    Buffer wm, wb, wab, ws, wc;
    int rc = dev_alloc(ctx, &wm, w32.size() * sizeof(float));
    if (rc == MFE_OK) rc = dev_alloc(ctx, &wb, (size_t)rows * Kpad * sizeof(bf16));
    if (rc == MFE_OK) rc = dev_alloc(ctx, &wab, (size_t)rowsA * KpadA * sizeof(bf16));
    if (rc == MFE_OK) rc = dev_alloc(ctx, &ws, kConvWsFloats * sizeof(float));
    if (rc == MFE_OK && mode == kS2) rc = dev_alloc(ctx, &wc, t2_class_elems(cout, rowsA) * sizeof(bf16));
    hipStream_t s = ctx->stream;
    if (rc == MFE_OK && hipMemcpyAsync(wm.ptr, w32.data(), w32.size() * sizeof(float), hipMemcpyHostToDevice, s) !=
                            hipSuccess)
        rc = MFE_EHIP;
    if (rc == MFE_OK) {
        const int64_t n = std::max((int64_t)rows * Kpad, (int64_t)rowsA * KpadA);
        hipLaunchKernelGGL(k_layer_weights, dim3(grid_of(n)), dim3(256), 0, s, (const float *)wm.ptr, cin, cout, Kpad,
                           KpadA, rowsA, mode == kS1 ? 1 : 0, (bf16 *)wb.ptr, (bf16 *)wab.ptr);
        if (hipGetLastError() != hipSuccess) rc = MFE_EHIP;
    }
    if (rc == MFE_OK && mode == kS2) rc = build_t2_classes(s, (const bf16 *)wab.ptr, rowsA, KpadA, cout, (bf16 *)wc.ptr);
    if (rc == MFE_OK)
        rc = conv(s, adjoint_mode(mode), (const bf16 *)gy_dev, Go, cout, (const bf16 *)wab.ptr, (const bf16 *)wc.ptr,
                  KpadA, cin, Gi, batch, nullptr, accumulate ? (const bf16 *)gx_dev : nullptr, 0, (bf16 *)gx_dev,
                  gx32_dev, (float *)ws.ptr, kConvWsFloats);
    if (hipStreamSynchronize(s) != hipSuccess && rc == MFE_OK) rc = MFE_EHIP;
    for (Buffer *b : {&wm, &wb, &wab, &ws, &wc}) dev_free(ctx, b);
    return rc;
}

int mfe_conv3d_wgrad_bf16(mfe_ctx *ctx, int mode, int batch, int Gi, int cin, const void *x_dev, int cout,
                          const void *gy_dev, float *dw_host) {
    clear_error();
    if (!ctx || !x_dev || !gy_dev || !dw_host || batch < 1 || Gi < 2 || mode < 0 || mode > 2 ||
        !valid_channels(cin) || !valid_channels(cout)) {
        set_error("need ctx, x, gy, dw, batch >= 1, Gi >= 2, mode 0..2, channels in {8, 16, 32, 64, 128}");
        return MFE_EINVAL;
    }
    if (hipSetDevice(ctx->device) != hipSuccess) return MFE_EHIP;
    const int Go = out_size(Gi, mode);
    const int Kpad = pad64(27 * cin), rows = (cout + 15) / 16 * 16;
    const int64_t total = (int64_t)batch * voxels(Go);
    const int nsplit = wgrad_splits(total, Kpad / 64);
    TempBuffer part(ctx), sum(ctx);
    MFE_TRY(part.alloc((size_t)nsplit * rows * Kpad * sizeof(float)));
    MFE_TRY(sum.alloc((size_t)rows * Kpad * sizeof(float)));
    hipStream_t s = ctx->stream;
    int rc = wgrad(s, mode, (const bf16 *)gy_dev, Go, cout, (const bf16 *)x_dev, Gi, cin, Kpad, batch,
                   (float *)part.ptr(), nsplit);
    std::vector<float> h((size_t)rows * Kpad);
    if (rc == MFE_OK) {
        const int64_t n = (int64_t)rows * Kpad;
        hipLaunchKernelGGL(k_sum_splits, dim3(grid_of(n)), dim3(256), 0, s, (const float *)part.ptr(), nsplit, n,
                           (float *)sum.ptr());
        if (hipGetLastError() != hipSuccess ||
            hipMemcpyAsync(h.data(), sum.ptr(), h.size() * sizeof(float), hipMemcpyDeviceToHost, s) != hipSuccess)
            rc = MFE_EHIP;
    }
    if (hipStreamSynchronize(s) != hipSuccess && rc == MFE_OK) rc = MFE_EHIP;
    if (rc == MFE_OK)
        for (int o = 0; o < cout; ++o)
            for (int k = 0; k < 27 * cin; ++k) dw_host[(size_t)o * 27 * cin + k] = h[(size_t)o * Kpad + k];
    return rc;
}

}  // extern "C"
