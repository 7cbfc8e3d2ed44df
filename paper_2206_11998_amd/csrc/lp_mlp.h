// lp_mlp.h -- device code of the learned state estimator (a 16 -> 64 -> 64 -> 1
// network, ReLU hidden layers, sigmoid output) shared by the network kernels
// (lp_mlp.hip) and the fused fit-and-update kernel (lp_solve.hip).  The
// network may stand in for the quotient estimator of the blended update
// (Sec. 2.1, state estimator); it is not part of the paper's method.
//
// BF16 matrix cores with FP32 accumulation, FP32 master weights.  One wave
// handles a tile of 16 samples.  Every layer is computed transposed,
// Y^T = W X^T, so that the accumulator fragment of one layer (lane l: sample
// l % 16, units 4 (l / 16) .. +3) is the B-operand fragment of the next.
//
// Layer 1 (K = 16 inputs) uses v_mfma_f32_16x16x16_bf16, lane l, v = 0..3:
//   A[i][k]: i = l % 16, k = 4 (l / 16) + v;  B[k][j]: j = l % 16, k = 4 (l / 16) + v
// Layer 2 (K = 64) uses gfx950's v_mfma_f32_16x16x32_bf16 twice, lane l, v = 0..7:
//   A[i][k]: i = l % 16, k = 8 (l / 16) + v;  B[k][j]: j = l % 16, k = 8 (l / 16) + v
// with the contraction order permuted so that B is two layer-1 accumulator
// fragments side by side: position 8 g + v of the pair (2 kk, 2 kk + 1) is
// hidden unit 16 (2 kk) + 4 g + v for v < 4 and 16 (2 kk + 1) + 4 g + v - 4
// for v >= 4, and the W2 fragment is loaded in the same order.
// Accumulators of both: D[i][j]: j = l % 16, i = 4 (l / 16) + v.
#ifndef LP_MLP_H
#define LP_MLP_H
#include "lp_internal.h"

typedef short bf16x4 __attribute__((ext_vector_type(4)));
typedef short s16x8 __attribute__((ext_vector_type(8)));
typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef float f32x4 __attribute__((ext_vector_type(4)));

#define MLP_IN 16
#define MLP_H 64
#define OFF_W1 0
#define OFF_B1 (OFF_W1 + MLP_H * MLP_IN)
#define OFF_W2 (OFF_B1 + MLP_H)
#define OFF_B2 (OFF_W2 + MLP_H * MLP_H)
#define OFF_W3 (OFF_B2 + MLP_H)
#define OFF_B3 (OFF_W3 + MLP_H)
static_assert(OFF_B3 + 1 == LP_MLP_NPARAM, "parameter layout");

// FP32 -> BF16, round to nearest even (NaN stays NaN)
__device__ __forceinline__ short f2bf(float f) {
    unsigned u = __float_as_uint(f);
    if ((u & 0x7f800000u) == 0x7f800000u) return (short)((u >> 16) | ((u & 0xffffu) ? 0x40u : 0u));
    u += 0x7fffu + ((u >> 16) & 1u);
    return (short)(u >> 16);
}

__device__ __forceinline__ f32x4 mfma16(bf16x4 a, bf16x4 b, f32x4 c) {
    return __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(a, b, c, 0, 0, 0);
}

__device__ __forceinline__ f32x4 mfma32(s16x8 a, s16x8 b, f32x4 c) {
    return __builtin_amdgcn_mfma_f32_16x16x32_bf16(__builtin_bit_cast(bf16x8, a), __builtin_bit_cast(bf16x8, b), c,
                                                   0, 0, 0);
}

__device__ __forceinline__ s16x8 cat8(bf16x4 lo, bf16x4 hi) {
    s16x8 r;
#pragma unroll
    for (int v = 0; v < 4; ++v) {
        r[v] = lo[v];
        r[4 + v] = hi[v];
    }
    return r;
}

__device__ __forceinline__ f32x4 zero4() {
    f32x4 z = {0.f, 0.f, 0.f, 0.f};
    return z;
}

__device__ __forceinline__ float sigmoidf(float z) { return 1.f / (1.f + __expf(-z)); }

// Weights of one wave in fragment order (network kernels).
struct MlpRegs {
    bf16x4 a1[4];     // W1 tiles (unit block ob): W1[16 ob + l%16][4 (l/16) + v]
    s16x8 a2[4][2];   // W2 tiles [ob][kk] in the permuted contraction order
    float b1[4][4];   // b1[16 ob + 4 (l/16) + v]
    float b2[4][4];
    float w3[4][4];
    float b3;
};

__device__ __forceinline__ void load_regs(const float *th, MlpRegs &R) {
    const int l = threadIdx.x & 63, r = l & 15, c = 4 * (l >> 4);
#pragma unroll
    for (int ob = 0; ob < 4; ++ob) {
#pragma unroll
        for (int v = 0; v < 4; ++v) {
            R.a1[ob][v] = f2bf(th[OFF_W1 + (16 * ob + r) * MLP_IN + c + v]);
            R.b1[ob][v] = th[OFF_B1 + 16 * ob + c + v];
            R.b2[ob][v] = th[OFF_B2 + 16 * ob + c + v];
            R.w3[ob][v] = th[OFF_W3 + 16 * ob + c + v];
        }
#pragma unroll
        for (int kk = 0; kk < 2; ++kk)
#pragma unroll
            for (int v = 0; v < 8; ++v)
                R.a2[ob][kk][v] =
                    f2bf(th[OFF_W2 + (16 * ob + r) * MLP_H + 16 * (2 * kk + (v >> 2)) + c + (v & 3)]);
    }
    R.b3 = th[OFF_B3];
}

// The same weights in LDS (fused kernel): BF16 W1 and W2 row-major, FP32
// biases and output weights.  Filled by a whole block (mlp_shared_load, then
// a barrier); fragments are read where they are used.
struct MlpShared {
    short w1[MLP_H * MLP_IN];
    short w2[MLP_H * MLP_H];
    float b1[MLP_H], b2[MLP_H], w3[MLP_H];
    float b3;
};

__device__ __forceinline__ void mlp_shared_load(const float *th, MlpShared &w) {
    for (int q = threadIdx.x; q < MLP_H * MLP_IN; q += blockDim.x) w.w1[q] = f2bf(th[OFF_W1 + q]);
    for (int q = threadIdx.x; q < MLP_H * MLP_H; q += blockDim.x) w.w2[q] = f2bf(th[OFF_W2 + q]);
    for (int q = threadIdx.x; q < MLP_H; q += blockDim.x) {
        w.b1[q] = th[OFF_B1 + q];
        w.b2[q] = th[OFF_B2 + q];
        w.w3[q] = th[OFF_W3 + q];
    }
    if (threadIdx.x == 0) w.b3 = th[OFF_B3];
}

// Weight sources of forward(): registers or LDS, the same values.
struct RegWeights {
    const MlpRegs &R;
    __device__ __forceinline__ bf16x4 a1(int ob) const { return R.a1[ob]; }
    __device__ __forceinline__ s16x8 a2(int ob, int kk) const { return R.a2[ob][kk]; }
    __device__ __forceinline__ float b1(int ob, int v) const { return R.b1[ob][v]; }
    __device__ __forceinline__ float b2(int ob, int v) const { return R.b2[ob][v]; }
    __device__ __forceinline__ float w3(int ob, int v) const { return R.w3[ob][v]; }
    __device__ __forceinline__ float b3() const { return R.b3; }
};

struct SharedWeights {
    const MlpShared &w;
    __device__ __forceinline__ bf16x4 ld4(const short *p) const { return *reinterpret_cast<const bf16x4 *>(p); }
    __device__ __forceinline__ bf16x4 a1(int ob) const {
        const int l = threadIdx.x & 63;
        return ld4(&w.w1[(16 * ob + (l & 15)) * MLP_IN + 4 * (l >> 4)]);
    }
    __device__ __forceinline__ s16x8 a2(int ob, int kk) const {
        const int l = threadIdx.x & 63;
        const short *row = &w.w2[(16 * ob + (l & 15)) * MLP_H + 4 * (l >> 4)];
        return cat8(ld4(row + 16 * (2 * kk)), ld4(row + 16 * (2 * kk + 1)));
    }
    __device__ __forceinline__ float b1(int ob, int v) const { return w.b1[16 * ob + 4 * ((threadIdx.x & 63) >> 4) + v]; }
    __device__ __forceinline__ float b2(int ob, int v) const { return w.b2[16 * ob + 4 * ((threadIdx.x & 63) >> 4) + v]; }
    __device__ __forceinline__ float w3(int ob, int v) const { return w.w3[16 * ob + 4 * ((threadIdx.x & 63) >> 4) + v]; }
    __device__ __forceinline__ float b3() const { return w.b3; }
};

// Input fragment: features 4 (l/16) .. +3 of sample l % 16 (zero when absent)
// from a row-major [sample][MLP_IN] array with stride `stride` floats.
__device__ __forceinline__ bf16x4 load_x(const float *feat, int64_t idx, bool ok, int stride = MLP_IN) {
    const int c = 4 * ((threadIdx.x & 63) >> 4);
    bf16x4 x;
#pragma unroll
    for (int v = 0; v < 4; ++v) x[v] = ok ? f2bf(feat[idx * stride + c + v]) : (short)0;
    return x;
}

// Forward pass of the tile: pre-activations d1, d2 (FP32, bias added), the
// BF16 hidden fragment h1 and the output z of sample l % 16 (in every lane).
template <class W>
__device__ __forceinline__ float forward(const W &w, bf16x4 x, f32x4 d1[4], bf16x4 h1[4], f32x4 d2[4]) {
#pragma unroll
    for (int ob = 0; ob < 4; ++ob) {
        d1[ob] = mfma16(w.a1(ob), x, zero4());
#pragma unroll
        for (int v = 0; v < 4; ++v) {
            d1[ob][v] += w.b1(ob, v);
            h1[ob][v] = f2bf(d1[ob][v] > 0.f ? d1[ob][v] : 0.f);
        }
    }
    float zp = 0.f;
#pragma unroll
    for (int ob = 0; ob < 4; ++ob) {
        f32x4 acc = zero4();
#pragma unroll
        for (int kk = 0; kk < 2; ++kk) acc = mfma32(w.a2(ob, kk), cat8(h1[2 * kk], h1[2 * kk + 1]), acc);
#pragma unroll
        for (int v = 0; v < 4; ++v) {
            acc[v] += w.b2(ob, v);
            zp += w.w3(ob, v) * (acc[v] > 0.f ? acc[v] : 0.f);
        }
        d2[ob] = acc;
    }
    // the four lanes of a sample (l, l+16, l+32, l+48) hold a quarter each
    zp += __shfl_xor(zp, 16);
    zp += __shfl_xor(zp, 32);
    return zp + w.b3();
}

// The network's phi for one particle -- 1.25 sigmoid(z) capped at 1 where
// every input is within range and the estimate is away from 1/2, else the
// quotient estimator's phi (phi = 0 where the update forces it) -- then the
// blended update and the mover, as the update kernel does them.  Counts the
// particle into used / plain / lim.
template <int D>
__device__ __forceinline__ void mlp_blend_update(const DevCfg &cfg, const Soa &p, DevScalars *sc, int i, double dt,
                                                 float z, bool in_range, const double st[D + 2],
                                                 const double lw[D + 2], const double uw[D + 2],
                                                 const double xs[D], double phi_plain, uint8_t mf,
                                                 unsigned long long &used, unsigned long long &plain,
                                                 unsigned long long &lim) {
    constexpr int NF = D + 2, FP = D + 1;
    double phi;
    if (mf & LP_MLP_FORCE0) {
        phi = 0.0;
    } else {
        const float y = fminf(1.25f * sigmoidf(z), 1.0f);
        if (in_range && fabsf(y - 0.5f) >= cfg.mlp_band) {
            phi = (double)y;
            ++used;
        } else {
            phi = phi_plain;
            ++plain;
        }
    }
    double ns[NF];
#pragma unroll
    for (int f = 0; f < NF; ++f) ns[f] = st[f] + dt * (uw[f] - phi * (uw[f] - lw[f]));
#pragma unroll
    for (int a = 0; a < D; ++a) {
        double xn = xs[a] + 0.5 * dt * (st[1 + a] + ns[1 + a]);
        if (cfg.periodic[a]) {
            if (xn >= cfg.hi[a]) xn -= cfg.L[a];
            else if (xn < cfg.lo[a]) xn += cfg.L[a];
        }
        p.x[a][i] = xn;
        p.u[a][i] = ns[1 + a];
    }
    p.V[i] = ns[0];
    p.P[i] = ns[FP];
    uint8_t flags = mf & (uint8_t)~LP_MLP_FORCE0;
    if (phi < 1.0) {
        flags |= LP_FLAG_LIMITED;
        ++lim;
    }
    if (!(ns[0] > 0.0) || !(ns[FP] > 0.0)) {
        flags |= LP_FLAG_NUMERIC;
        atomicOr(&sc->error_bits, 2u);
    }
    if (p.flags) p.flags[i] = flags;
    if (p.phi) p.phi[i] = (float)phi;
}

// The three network counters of a block added once each (all threads of the
// block call it; same-address atomics serialise in L2).
__device__ __forceinline__ void mlp_block_counts(DevScalars *sc, unsigned long long used, unsigned long long plain,
                                                 unsigned long long lim) {
    for (int o = 32; o > 0; o >>= 1) {
        used += __shfl_xor(used, o);
        plain += __shfl_xor(plain, o);
        lim += __shfl_xor(lim, o);
    }
    __shared__ unsigned long long part[LP_BLOCK / 64][3];
    const int wv = threadIdx.x >> 6;
    if ((threadIdx.x & 63) == 0) {
        part[wv][0] = used;
        part[wv][1] = plain;
        part[wv][2] = lim;
    }
    __syncthreads();
    if (threadIdx.x < 3) {
        unsigned long long v = 0;
        for (int q = 0; q < (int)(blockDim.x >> 6); ++q) v += part[q][threadIdx.x];
        unsigned long long *dst = threadIdx.x == 0 ? &sc->n_mlp : threadIdx.x == 1 ? &sc->n_mlp_plain : &sc->n_limited;
        if (v) atomicAdd(dst, v);
    }
}

#endif
