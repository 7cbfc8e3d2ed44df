// lp_mlp.hip -- the learned state estimator's kernels on gfx950: inference
// over a batch, the estimator stage of a step whose update was staged, and
// training (forward and backward of the mean binary cross-entropy, Adam).
// The network and its fragment layouts are in lp_mlp.h.
#include "lp_mlp.h"

// ---------------------------------------------------------------------------
// Network output z (and sigmoid) for n samples: one wave per tile of 16.
// ---------------------------------------------------------------------------
__global__ __launch_bounds__(64) void k_mlp_forward(const float *th, int64_t n, const float *feat, float *z_out,
                                                    float *y_out) {
    MlpRegs R;
    load_regs(th, R);
    const int l = threadIdx.x & 63;
    const int64_t ntile = (n + 15) / 16;
    for (int64_t tile = blockIdx.x; tile < ntile; tile += gridDim.x) {
        const int64_t idx = tile * 16 + (l & 15);
        const bool ok = idx < n;
        f32x4 d1[4], d2[4];
        bf16x4 h1[4];
        const float z = forward(RegWeights{R}, load_x(feat, idx, ok), d1, h1, d2);
        if (ok && l < 16) {
            if (z_out) z_out[idx] = z;
            if (y_out) y_out[idx] = sigmoidf(z);
        }
    }
}

void launch_mlp_forward(const float *th, int64_t n, const float *feat, float *z, float *y, hipStream_t st) {
    int64_t nt = (n + 15) / 16;
    unsigned g = (unsigned)(nt < 4096 ? (nt > 0 ? nt : 1) : 4096);
    hipLaunchKernelGGL(k_mlp_forward, dim3(g), dim3(64), 0, st, th, n, feat, z, y);
    (void)hipGetLastError();
}

// ---------------------------------------------------------------------------
// Estimator stage of a step with the network: phi = min(1, 1.25 sigmoid(z))
// where the network is trusted, the quotient estimator's phi elsewhere, then
// the blended update and the mover -- the same arithmetic as the update kernel.
// Items: every cell-order particle (queued == 0), or (queued != 0) only the
// particles staged by the FP64 fallback (its queue) and by the refinement
// (its queue, pairs), when the fused kernel applied the network to the rest.
// ---------------------------------------------------------------------------
template <int D>
__global__ __launch_bounds__(256) void k_mlp_apply(const float *th, Sorted srt, Soa p, DevCfg cfg, DevScalars *sc,
                                                  int n_real, MlpStage ms, int queued, const int *fq, const int *rq) {
    constexpr int NF = D + 2, FP = D + 1;
    MlpRegs R;
    load_regs(th, R);
    const int l = threadIdx.x & 63;
    const int wv = threadIdx.x >> 6;
    const int n_fb = queued ? sc->n_fallback : 0;
    const int n_items = queued ? n_fb + sc->n_refine : sc->n_total;
    const int n_total = sc->n_total;
    const double dt = sc->dt;
    // the cell-order particle of item w (-1: none)
    auto item = [&](int64_t w) -> int {
        if (w >= n_items) return -1;
        if (!queued) return (int)w;
        return w < n_fb ? fq[w] : rq[2 * (w - n_fb)];
    };
    // groups of 64 items, one wave each: four 16-item tiles through the
    // network, then every lane finishes its own item of the group
    const int64_t ngroup = ((int64_t)n_items + 63) / 64;
    unsigned long long used = 0, plain = 0, lim = 0;
    for (int64_t grp = (int64_t)blockIdx.x * 4 + wv; grp < ngroup; grp += (int64_t)gridDim.x * 4) {
        const int s = item(grp * 64 + l);
        const bool ok = s >= 0 && s < n_total;
        const int i = ok ? srt.id[s] : n_real;
        const bool mine = ok && i < n_real && srt.h[s] > 0.0;  // not a deleted particle's slot
        // the update's operands are loaded before the network runs, so their
        // latency overlaps the matrix instructions
        double st[NF], lw[NF], uw[NF], xs[D];
        double phi_plain = 0.0;
        uint8_t mf = 0;
        if (mine) {
            st[0] = srt.V[s];
#pragma unroll
            for (int a = 0; a < D; ++a) {
                st[1 + a] = srt.u[a][s];
                xs[a] = srt.x[a][s];
            }
            st[FP] = srt.P[s];
#pragma unroll
            for (int f = 0; f < NF; ++f) {
                lw[f] = ms.rates[(int64_t)f * ms.ld + s];
                uw[f] = ms.rates[(int64_t)(NF + f) * ms.ld + s];
            }
            phi_plain = ms.phi_plain[s];
            mf = ms.mflag[s];
        }
        // tile t covers items 64 grp + 16 t .. + 15; after its pass, lane l
        // of quarter t holds the output of item 64 grp + l (a column of the
        // products depends on its own sample only, so unstaged rows of ghosts
        // affect nothing else)
        float z = 0.f;
#pragma unroll
        for (int t = 0; t < 4; ++t) {
            const int st_ = item(grp * 64 + 16 * t + (l & 15));
            const bf16x4 x = load_x(ms.feat, st_ >= 0 ? st_ : 0, st_ >= 0 && st_ < n_total);
            f32x4 d1[4], d2[4];
            bf16x4 h1[4];
            const float zt = forward(RegWeights{R}, x, d1, h1, d2);
            if ((l >> 4) == t) z = zt;
        }
        if (!mine) continue;
        bool in_range = true;
#pragma unroll
        for (int q = 0; q < MLP_IN; ++q) in_range = in_range && fabsf(ms.feat[(int64_t)s * MLP_IN + q]) <= cfg.mlp_feat_max;
        mlp_blend_update<D>(cfg, p, sc, i, dt, z, in_range, st, lw, uw, xs, phi_plain, mf, used, plain, lim);
    }
    mlp_block_counts(sc, used, plain, lim);
}

void launch_mlp_apply(const float *th, const Sorted &s, const Soa &p, const DevCfg &cfg, DevScalars *sc,
                      int64_t n_total_cap, int n_real, const MlpStage &ms, int queued, const int *fq, const int *rq,
                      hipStream_t st) {
    // four waves per block, at most 8192 waves: each wave loads the weights
    // once (the queued particles are few: at most 256 blocks)
    int64_t nb = ((n_total_cap + 63) / 64 + 3) / 4;
    const int64_t cap = queued ? 256 : 2048;
    unsigned g = (unsigned)(nb < cap ? (nb > 0 ? nb : 1) : cap);
    if (cfg.D == 3)
        hipLaunchKernelGGL(k_mlp_apply<3>, dim3(g), dim3(256), 0, st, th, s, p, cfg, sc, n_real, ms, queued, fq, rq);
    else
        hipLaunchKernelGGL(k_mlp_apply<2>, dim3(g), dim3(256), 0, st, th, s, p, cfg, sc, n_real, ms, queued, fq, rq);
    (void)hipGetLastError();
}

// ---------------------------------------------------------------------------
// Training: forward and backward of the mean binary cross-entropy over a
// batch.  Every block (one wave) accumulates its tiles' gradient in registers
// and writes it, complete, to its row of part[]; k_mlp_reduce sums the rows in
// a fixed order.  Weight gradients sum over samples, so their products take
// the sample index as the contraction dimension: the fragments are turned
// around through LDS.
// ---------------------------------------------------------------------------
__global__ __launch_bounds__(64) void k_mlp_grad(const float *th, int64_t b0, int64_t nb, const float *feat,
                                                 const float *target, float inv_batch, float *part,
                                                 float *loss_part) {
    __shared__ short sA[MLP_H * 16];   // [unit][sample], BF16
    __shared__ short sB[MLP_H * 16];   // [unit][sample], BF16
    __shared__ short sX[MLP_IN * 16];  // [feature][sample], BF16
    MlpRegs R;
    load_regs(th, R);
    const int l = threadIdx.x & 63, r = l & 15, c = 4 * (l >> 4);
    // W2 transposed tiles [ib][kb]: W2[16 kb + 4 (l/16) + v][16 ib + l%16]
    bf16x4 a2t[4][4];
#pragma unroll
    for (int ib = 0; ib < 4; ++ib)
#pragma unroll
        for (int kb = 0; kb < 4; ++kb)
#pragma unroll
            for (int v = 0; v < 4; ++v) a2t[ib][kb][v] = f2bf(th[OFF_W2 + (16 * kb + c + v) * MLP_H + 16 * ib + r]);
    f32x4 g1[4], g2[4][4];
#pragma unroll
    for (int q = 0; q < 4; ++q) {
        g1[q] = zero4();
#pragma unroll
        for (int w = 0; w < 4; ++w) g2[q][w] = zero4();
    }
    float gb1[4][4], gb2[4][4], gw3[4][4], gb3 = 0.f, loss = 0.f;
#pragma unroll
    for (int q = 0; q < 4; ++q)
#pragma unroll
        for (int v = 0; v < 4; ++v) { gb1[q][v] = 0.f; gb2[q][v] = 0.f; gw3[q][v] = 0.f; }

    const int64_t ntile = (nb + 15) / 16;
    for (int64_t tile = blockIdx.x; tile < ntile; tile += gridDim.x) {
        const int64_t j = tile * 16 + r;  // sample of this lane, within the batch
        const bool ok = j < nb;
        const int64_t idx = b0 + j;
        const bf16x4 x = load_x(feat, idx, ok);
        f32x4 d1[4], d2[4];
        bf16x4 h1[4];
        const float z = forward(RegWeights{R}, x, d1, h1, d2);
        const float t = ok ? target[idx] : 0.f;
        const float y = sigmoidf(z);
        const float dz = ok ? (y - t) * inv_batch : 0.f;
        if (ok && l < 16) {
            loss += (z > 0.f ? z : 0.f) + log1pf(__expf(-fabsf(z))) - t * z;
            gb3 += dz;
        }
        // output layer and second hidden layer
        bf16x4 da2[4];
#pragma unroll
        for (int ob = 0; ob < 4; ++ob)
#pragma unroll
            for (int v = 0; v < 4; ++v) {
                const float a2 = d2[ob][v];
                gw3[ob][v] += dz * (a2 > 0.f ? a2 : 0.f);
                const float g = a2 > 0.f ? dz * R.w3[ob][v] : 0.f;
                gb2[ob][v] += g;
                da2[ob][v] = f2bf(g);
            }
        // dW2 = dA2 H1^T over the tile's samples
#pragma unroll
        for (int ob = 0; ob < 4; ++ob)
#pragma unroll
            for (int v = 0; v < 4; ++v) {
                sA[(16 * ob + c + v) * 16 + r] = da2[ob][v];
                sB[(16 * ob + c + v) * 16 + r] = h1[ob][v];
            }
#pragma unroll
        for (int v = 0; v < 4; ++v) sX[(c + v) * 16 + r] = x[v];
        __syncthreads();
        bf16x4 fa[4], fb[4];
#pragma unroll
        for (int q = 0; q < 4; ++q)
#pragma unroll
            for (int v = 0; v < 4; ++v) {
                fa[q][v] = sA[(16 * q + r) * 16 + c + v];
                fb[q][v] = sB[(16 * q + r) * 16 + c + v];
            }
#pragma unroll
        for (int ob = 0; ob < 4; ++ob)
#pragma unroll
            for (int ib = 0; ib < 4; ++ib) g2[ob][ib] = mfma16(fa[ob], fb[ib], g2[ob][ib]);
        // dH1 = W2^T dA2, through the first hidden layer's ReLU
        bf16x4 da1[4];
#pragma unroll
        for (int ib = 0; ib < 4; ++ib) {
            f32x4 acc = zero4();
#pragma unroll
            for (int kb = 0; kb < 4; ++kb) acc = mfma16(a2t[ib][kb], da2[kb], acc);
#pragma unroll
            for (int v = 0; v < 4; ++v) {
                const float g = d1[ib][v] > 0.f ? acc[v] : 0.f;
                gb1[ib][v] += g;
                da1[ib][v] = f2bf(g);
            }
        }
        __syncthreads();  // sA is reused
#pragma unroll
        for (int ob = 0; ob < 4; ++ob)
#pragma unroll
            for (int v = 0; v < 4; ++v) sA[(16 * ob + c + v) * 16 + r] = da1[ob][v];
        __syncthreads();
        // dW1 = dA1 X over the tile's samples
        bf16x4 fx;
#pragma unroll
        for (int v = 0; v < 4; ++v) fx[v] = sX[r * 16 + c + v];
#pragma unroll
        for (int ob = 0; ob < 4; ++ob) {
            bf16x4 f;
#pragma unroll
            for (int v = 0; v < 4; ++v) f[v] = sA[(16 * ob + r) * 16 + c + v];
            g1[ob] = mfma16(f, fx, g1[ob]);
        }
        __syncthreads();  // before the next tile overwrites sA, sB, sX
    }
    // this block's complete gradient, parameter layout order
    float *out = part + (int64_t)blockIdx.x * LP_MLP_NPARAM;
#pragma unroll
    for (int ob = 0; ob < 4; ++ob)
#pragma unroll
        for (int v = 0; v < 4; ++v) {
            out[OFF_W1 + (16 * ob + c + v) * MLP_IN + r] = g1[ob][v];
#pragma unroll
            for (int ib = 0; ib < 4; ++ib) out[OFF_W2 + (16 * ob + c + v) * MLP_H + 16 * ib + r] = g2[ob][ib][v];
        }
    // per-unit sums over the 16 lanes (samples) that share a unit set
#pragma unroll
    for (int ob = 0; ob < 4; ++ob)
#pragma unroll
        for (int v = 0; v < 4; ++v) {
            float a = gb1[ob][v], b = gb2[ob][v], w = gw3[ob][v];
#pragma unroll
            for (int o = 1; o < 16; o <<= 1) {
                a += __shfl_xor(a, o);
                b += __shfl_xor(b, o);
                w += __shfl_xor(w, o);
            }
            if (r == 0) {
                out[OFF_B1 + 16 * ob + c + v] = a;
                out[OFF_B2 + 16 * ob + c + v] = b;
                out[OFF_W3 + 16 * ob + c + v] = w;
            }
        }
    for (int o = 1; o < 64; o <<= 1) {
        gb3 += __shfl_xor(gb3, o);
        loss += __shfl_xor(loss, o);
    }
    if (l == 0) {
        out[OFF_B3] = gb3;
        loss_part[blockIdx.x] = loss;
    }
}

// grad[q] = sum of the blocks' rows in block order; *loss likewise (mean over the batch)
__global__ void k_mlp_reduce(const float *part, const float *loss_part, int nblk, float inv_batch, float *grad,
                             float *loss) {
    const int q = blockIdx.x * blockDim.x + threadIdx.x;
    if (q < LP_MLP_NPARAM) {
        float s = 0.f;
        for (int b = 0; b < nblk; ++b) s += part[(int64_t)b * LP_MLP_NPARAM + q];
        grad[q] = s;
    }
    if (q == 0 && loss) {
        float s = 0.f;
        for (int b = 0; b < nblk; ++b) s += loss_part[b];
        *loss = s * inv_batch;
    }
}

// Adam step t (1-based) on the FP32 master weights; the batch loss is added
// to *loss_acc.
__global__ void k_mlp_adam(float *th, float *m, float *v, const float *grad, float lr, float b1, float b2,
                           float eps, int t, const float *loss, float *loss_acc) {
    const int q = blockIdx.x * blockDim.x + threadIdx.x;
    if (q < LP_MLP_NPARAM) {
        const float g = grad[q];
        const float mq = b1 * m[q] + (1.f - b1) * g;
        const float vq = b2 * v[q] + (1.f - b2) * g * g;
        m[q] = mq;
        v[q] = vq;
        const float mh = mq / (1.f - powf(b1, (float)t));
        const float vh = vq / (1.f - powf(b2, (float)t));
        th[q] -= lr * mh / (sqrtf(vh) + eps);
    }
    if (q == 0 && loss_acc) *loss_acc += *loss;
}

// Blocks of a gradient launch: every block covers several tiles, so that the
// fixed-order reduction over the blocks' rows stays short.
int mlp_grad_blocks(int64_t nb) {
    int64_t nt = (nb + 15) / 16;
    return (int)(nt < 128 ? (nt > 0 ? nt : 1) : 128);
}

void launch_mlp_grad(const float *th, int64_t b0, int64_t nb, const float *feat, const float *target, float *part,
                     float *loss_part, float *grad, float *loss, hipStream_t st) {
    const int blk = mlp_grad_blocks(nb);
    const float inv = 1.f / (float)nb;
    hipLaunchKernelGGL(k_mlp_grad, dim3(blk), dim3(64), 0, st, th, b0, nb, feat, target, inv, part, loss_part);
    hipLaunchKernelGGL(k_mlp_reduce, dim3((LP_MLP_NPARAM + 255) / 256), dim3(256), 0, st, part, loss_part, blk, inv,
                       grad, loss);
    (void)hipGetLastError();
}

void launch_mlp_adam(float *th, float *m, float *v, const float *grad, float lr, float b1, float b2, float eps,
                     int t, const float *loss, float *loss_acc, hipStream_t st) {
    hipLaunchKernelGGL(k_mlp_adam, dim3((LP_MLP_NPARAM + 255) / 256), dim3(256), 0, st, th, m, v, grad, lr, b1, b2,
                       eps, t, loss, loss_acc);
    (void)hipGetLastError();
}

// ---------------------------------------------------------------------------
// Staged inputs and quotient-estimator phi back to the caller's order.
// ---------------------------------------------------------------------------
__global__ void k_features_out(Sorted srt, MlpStage ms, const int *n_total_dev, int n_real, float *feat,
                               float *phi, uint8_t *valid) {
    const int s = blockIdx.x * blockDim.x + threadIdx.x;
    if (s >= *n_total_dev) return;
    const int i = srt.id[s];
    if (i >= n_real) return;
#pragma unroll
    for (int q = 0; q < MLP_IN; ++q) feat[(int64_t)i * MLP_IN + q] = ms.feat[(int64_t)s * MLP_IN + q];
    phi[i] = (float)ms.phi_plain[s];
    if (valid) valid[i] = (ms.mflag[s] & LP_MLP_FORCE0) ? 0 : 1;
}

void launch_features_out(const Sorted &s, const MlpStage &ms, const int *n_total_dev, int64_t n_total_cap,
                         int n_real, float *feat, float *phi, uint8_t *valid, hipStream_t st) {
    unsigned g = (unsigned)((n_total_cap + LP_BLOCK - 1) / LP_BLOCK);
    hipLaunchKernelGGL(k_features_out, dim3(g > 0 ? g : 1), dim3(LP_BLOCK), 0, st, s, ms, n_total_dev, n_real, feat,
                       phi, valid);
    (void)hipGetLastError();
}

__global__ void k_fill_f32(float *p, int n, float v) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) p[i] = v;
}

void launch_fill_f32(float *p, int n, float v, hipStream_t st) {
    hipLaunchKernelGGL(k_fill_f32, dim3((n + 255) / 256 > 0 ? (n + 255) / 256 : 1), dim3(256), 0, st, p, n, v);
    (void)hipGetLastError();
}
