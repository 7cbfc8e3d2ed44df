// lp_grid.hip -- per-step particle bookkeeping on gfx950:
//   smoothing lengths, radii and the CFL time step (Sec. 2.2 loop, dt rule),
//   mirror ghosts across solid walls (Sec. 2.2, step 1),
//   the cell-ordered particle layout that replaces the octree (Sec. 2.2,
//   step 2): a counting sort by Morton cell at the finest level, one exclusive
//   scan that doubles as the finest cell table, and coarser tables taken from it.
// All kernels are HBM-bound streaming kernels: coalesced SoA loads/stores,
// 256-thread blocks, one element per thread (grid-stride where noted).
#include "lp_internal.h"

#define CHECK_LAUNCH() (void)hipGetLastError()

static inline unsigned blocks_for(uint64_t n, int per = LP_BLOCK) {
    uint64_t b = (n + per - 1) / per;
    if (b < 1) b = 1;
    return (unsigned)b;
}

// ---------------------------------------------------------------------------
// Scalars
// ---------------------------------------------------------------------------
__global__ void k_reset_scalars(DevScalars *sc, double dt_in, int n_real, int clear_halt) {
    sc->n_total = n_real;
    sc->n_in = n_real;
    sc->n_dead = 0;
    sc->min_hc = 0x7ff0000000000000ull;  // +inf
    sc->rmax = 0ull;
    sc->rmin = 0x7ff0000000000000ull;
    sc->dt_in = dt_in;
    sc->n_ghost = 0;
    sc->prev_max_count = sc->max_count;
    sc->max_count = 0;
    sc->n_fallback = 0;
    sc->n_refine = 0;
    sc->n_overflow = 0;
    sc->n_fovf = 0;
    sc->n_limited = 0ull;
    sc->n_mlp = 0ull;
    sc->n_mlp_plain = 0ull;
    sc->done = 0u;  // recomputed by k_dt from t and t_end
    if (clear_halt) sc->halt = 0u;
    for (int a = 0; a < 3; ++a) { sc->xlo[a] = ~0ull; sc->xhi[a] = 0ull; }
    for (int q = 0; q < 8; ++q) { sc->head[0][q] = 0u; sc->head[1][q] = 0u; }
}

void launch_reset_scalars(DevScalars *sc, double dt_in, int n_real, int clear_halt, hipStream_t st) {
    hipLaunchKernelGGL(k_reset_scalars, dim3(1), dim3(1), 0, st, sc, dt_in, n_real, clear_halt);
    CHECK_LAUNCH();
}

// Admission of the particle work of a step.  n_total = real + ghost particles,
// or 0 with dt = 0 when the step is skipped: t_end reached, more ghosts than
// the workspace was sized for (then halt stays raised until the host re-plans
// the workspace; every later kernel of the step sees n_total = 0), or, with
// stop_on_error, an error reported by an earlier step and not yet collected.
__global__ void k_gate(DevScalars *sc, int n_real, long long cap_ghost, int stop_on_error) {
    if (sc->n_ghost > cap_ghost) sc->halt = 1u;
    if (sc->done || sc->halt || (stop_on_error && sc->error_bits)) {
        sc->n_total = 0;
        sc->n_in = 0;  // nothing sorted either (the ghost count may exceed the arrays)
        sc->dt = 0.0;
    } else {
        sc->n_in = n_real + sc->n_ghost;
        sc->n_total = n_real - sc->n_dead + sc->n_ghost;  // absent particles stay out of the cell order
    }
}

void launch_gate(DevScalars *sc, int n_real, int64_t cap_ghost, int stop_on_error, hipStream_t st) {
    hipLaunchKernelGGL(k_gate, dim3(1), dim3(1), 0, st, sc, n_real, (long long)cap_ghost, stop_on_error);
    CHECK_LAUNCH();
}

__device__ __forceinline__ double wave_min(double v) {
    for (int o = 32; o > 0; o >>= 1) v = fmin(v, __shfl_xor(v, o));
    return v;
}
__device__ __forceinline__ double wave_max(double v) {
    for (int o = 32; o > 0; o >>= 1) v = fmax(v, __shfl_xor(v, o));
    return v;
}

// Per-block minima of (h/c, r, -r, x_a, -x_a) written to part[block * PREP_W + q],
// then the block's count of absent particles (zero mass: no radius, no part in
// the minima); k_prep_final folds the block results (order-free min and an
// integer count, so exact).  With the positions xb and enlarged radii Rb of
// the last list build (list reuse), the same pass also reduces the reuse
// check's a = max_i (r_i + d_i - R_i) and d = max_i d_i, d_i = |x_i - xb_i|
// (minimum image), as minima of their negatives.
#define PREP_Q 11
#define PREP_W (PREP_Q + 1)
#define PREP_PER 4  // particles per thread (the block reduction is paid once for them)
__global__ void k_prep(Soa p, DevCfg cfg, double *h_out, double *r_out, double *part, const double *xb0,
                       const double *xb1, const double *xb2, const double *Rb) {
    double v[PREP_Q];
    for (int q = 0; q < PREP_Q; ++q) v[q] = INFINITY;
    int dead = 0;
    const int base = blockIdx.x * blockDim.x * PREP_PER + threadIdx.x;
#pragma unroll
    for (int u = 0; u < PREP_PER; ++u) {
        const int i = base + u * (int)blockDim.x;
        if (i >= p.n) break;
        if (!(p.m[i] > 0.0)) {
            h_out[i] = 0.0;
            r_out[i] = 0.0;
            ++dead;
            continue;
        }
        double V = p.V[i], P = p.P[i], m = p.m[i];
        double mv = m * V;
        double h = cfg.D == 3 ? cbrt(mv) : sqrt(mv);
        double c = sqrt(cfg.gamma * P * V);
        double r = cfg.kappa * h;
        h_out[i] = h;
        r_out[i] = r;
        v[0] = fmin(v[0], h / c);
        v[1] = fmin(v[1], r);
        v[2] = fmin(v[2], -r);
        for (int a = 0; a < cfg.D; ++a) {
            double x = p.x[a][i];
            v[3 + a] = fmin(v[3 + a], x);
            v[6 + a] = fmin(v[6 + a], -x);
        }
        if (Rb) {
            const double *xb[3] = {xb0, xb1, xb2};
            double d2 = 0.0;
            for (int a = 0; a < cfg.D; ++a) {
                const double e = min_image(cfg, a, p.x[a][i] - xb[a][i]);
                d2 += e * e;
            }
            const double di = sqrt(d2);
            const double ai = r + di - Rb[i];
            const bool bad = !(ai == ai) || !(di == di);  // NaN positions: rebuild
            v[9] = fmin(v[9], bad ? -INFINITY : -ai);
            v[10] = fmin(v[10], bad ? -INFINITY : -di);
        }
    }
    __shared__ double red[PREP_Q][LP_BLOCK / 64];
    __shared__ int dred[LP_BLOCK / 64];
    for (int q = 0; q < PREP_Q; ++q) {
        double w = wave_min(v[q]);
        if ((threadIdx.x & 63) == 0) red[q][threadIdx.x >> 6] = w;
    }
    for (int o = 32; o > 0; o >>= 1) dead += __shfl_xor(dead, o);
    if ((threadIdx.x & 63) == 0) dred[threadIdx.x >> 6] = dead;
    __syncthreads();
    if (threadIdx.x < PREP_Q) {
        double w = red[threadIdx.x][0];
        for (int k = 1; k < LP_BLOCK / 64; ++k) w = fmin(w, red[threadIdx.x][k]);
        part[(int64_t)blockIdx.x * PREP_W + threadIdx.x] = w;
    } else if (threadIdx.x == PREP_Q) {
        int d = 0;
        for (int k = 0; k < LP_BLOCK / 64; ++k) d += dred[k];
        part[(int64_t)blockIdx.x * PREP_W + PREP_Q] = (double)d;
    }
}

__global__ void k_prep_final(const double *part, int nblocks, DevScalars *sc) {
    __shared__ double red[PREP_Q][1024 / 64];
    __shared__ double dred[1024 / 64];
    double v[PREP_Q];
    double dead = 0.0;  // integer-valued: exact in any order
    for (int q = 0; q < PREP_Q; ++q) v[q] = INFINITY;
    for (int b = threadIdx.x; b < nblocks; b += blockDim.x) {
        for (int q = 0; q < PREP_Q; ++q) v[q] = fmin(v[q], part[(int64_t)b * PREP_W + q]);
        dead += part[(int64_t)b * PREP_W + PREP_Q];
    }
    for (int q = 0; q < PREP_Q; ++q) {
        double w = wave_min(v[q]);
        if ((threadIdx.x & 63) == 0) red[q][threadIdx.x >> 6] = w;
    }
    for (int o = 32; o > 0; o >>= 1) dead += __shfl_xor(dead, o);
    if ((threadIdx.x & 63) == 0) dred[threadIdx.x >> 6] = dead;
    __syncthreads();
    if (threadIdx.x == 0) {
        double d = 0.0;
        for (int k = 0; k < (int)(blockDim.x / 64); ++k) d += dred[k];
        sc->n_dead = (int)d;
        double m[PREP_Q];
        for (int q = 0; q < PREP_Q; ++q) {
            m[q] = red[q][0];
            for (int k = 1; k < (int)(blockDim.x / 64); ++k) m[q] = fmin(m[q], red[q][k]);
        }
        if (m[0] < INFINITY) sc->min_hc = dbl_bits(m[0]);
        if (m[1] < INFINITY) sc->rmin = dbl_bits(m[1]);
        if (m[2] < INFINITY) sc->rmax = dbl_bits(-m[2]);
        for (int a = 0; a < 3; ++a)
            if (m[3 + a] < INFINITY) {
                sc->xlo[a] = dbl_key(m[3 + a]);
                sc->xhi[a] = dbl_key(-m[6 + a]);
            }
        if (m[9] < INFINITY) {  // the reuse check ran (and some particle is present)
            sc->reuse_a = dbl_key(-m[9]);
            sc->reuse_d = dbl_bits(-m[10]);
        }
    }
}

void launch_prep(const Soa &p, const DevCfg &cfg, DevScalars *sc, double *h, double *r, double *part,
                 hipStream_t st, double *const xb[3], const double *Rb) {
    unsigned nb = blocks_for(p.n, LP_BLOCK * PREP_PER);
    const double *x0 = xb ? xb[0] : nullptr, *x1 = xb ? xb[1] : nullptr;
    const double *x2 = xb ? (cfg.D == 3 ? xb[2] : xb[0]) : nullptr;
    hipLaunchKernelGGL(k_prep, dim3(nb), dim3(LP_BLOCK), 0, st, p, cfg, h, r, part, x0, x1, x2, xb ? Rb : nullptr);
    hipLaunchKernelGGL(k_prep_final, dim3(1), dim3(1024), 0, st, part, (int)nb, sc);
    CHECK_LAUNCH();
}

size_t prep_partial_words(int64_t n) { return (size_t)((n + LP_BLOCK - 1) / LP_BLOCK + 1) * PREP_W; }

// dt = cfl * min h/c unless given; with clip, the step is shortened so that t
// does not pass t_end (and set to zero once t_end is reached).
__global__ void k_dt(DevCfg cfg, DevScalars *sc, int clip) {
    double dt = sc->dt_in > 0.0 ? sc->dt_in : cfg.cfl * bits_dbl(sc->min_hc);
    sc->clipped = 0u;
    if (sc->n_dead >= sc->n_total) {  // every particle absent (n_total holds the real count here)
        sc->dt = 0.0;
        sc->done = 1u;
        return;
    }
    if (clip && sc->t_end > 0.0) {
        double rem = sc->t_end - sc->t;
        if (!(rem > 0.0)) { dt = 0.0; sc->done = 1u; }
        else if (dt >= rem) { dt = rem; sc->clipped = 1u; }
    }
    sc->dt = dt;
}

// min / max of given radii (for searches on caller-provided radii)
// Range of the radii and bounding box of the positions: a grid-stride pass per
// thread, then per wave and per block (LDS), then one atomic per block and
// quantity (min and max are order-free, so the result is exact).
__global__ __launch_bounds__(LP_BLOCK) void k_rminmax(const double *r, double *x0, double *x1, double *x2, int D,
                                                      int n, DevScalars *sc) {
    constexpr int NW = LP_BLOCK / 64;
    __shared__ double red[8][NW];
    const double *const xs[3] = {x0, x1, x2};
    // v[0] = min r, v[1] = max r, v[2 + a] = min x_a, v[5 + a] = max x_a
    double v[8] = {INFINITY, 0.0, INFINITY, INFINITY, INFINITY, -INFINITY, -INFINITY, -INFINITY};
    for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < n; i += gridDim.x * blockDim.x) {
        const double ri = r[i];
        v[0] = fmin(v[0], ri);
        v[1] = fmax(v[1], ri);
        for (int a = 0; a < D; ++a) {
            const double xa = xs[a][i];
            v[2 + a] = fmin(v[2 + a], xa);
            v[5 + a] = fmax(v[5 + a], xa);
        }
    }
    const int w = threadIdx.x >> 6;
    for (int q = 0; q < 8; ++q) {
        const bool is_min = q == 0 || (q >= 2 && q < 5);
        const double t = is_min ? wave_min(v[q]) : wave_max(v[q]);
        if ((threadIdx.x & 63) == 0) red[q][w] = t;
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        double b[8];
        for (int q = 0; q < 8; ++q) {
            const bool is_min = q == 0 || (q >= 2 && q < 5);
            b[q] = red[q][0];
            for (int k = 1; k < NW; ++k) b[q] = is_min ? fmin(b[q], red[q][k]) : fmax(b[q], red[q][k]);
        }
        if (b[0] < INFINITY) atomicMin(&sc->rmin, dbl_bits(b[0]));
        if (b[1] > 0.0) atomicMax(&sc->rmax, dbl_bits(b[1]));
        for (int a = 0; a < D; ++a)
            if (b[2 + a] <= b[5 + a]) {
                atomicMin(&sc->xlo[a], dbl_key(b[2 + a]));
                atomicMax(&sc->xhi[a], dbl_key(b[5 + a]));
            }
    }
}

void launch_rminmax(const double *r, const double *const x[3], int D, int n, DevScalars *sc, hipStream_t st) {
    unsigned blocks = blocks_for(n);
    if (blocks > 1024) blocks = 1024;
    hipLaunchKernelGGL(k_rminmax, dim3(blocks), dim3(LP_BLOCK), 0, st, r, (double *)x[0], (double *)x[1],
                       (double *)x[2], D, n, sc);
    CHECK_LAUNCH();
}

// t += dt after a step
__global__ void k_advance_time(DevScalars *sc) {
    if (sc->n_total > 0) {
        sc->t = sc->clipped ? sc->t_end : sc->t + sc->dt;  // a clipped step lands on t_end exactly
        sc->steps += 1ull;
    }
}

void launch_advance_time(DevScalars *sc, hipStream_t st) {
    hipLaunchKernelGGL(k_advance_time, dim3(1), dim3(1), 0, st, sc);
    CHECK_LAUNCH();
}

void launch_dt(const DevCfg &cfg, DevScalars *sc, int clip_t_end, hipStream_t st) {
    hipLaunchKernelGGL(k_dt, dim3(1), dim3(1), 0, st, cfg, sc, clip_t_end);
    CHECK_LAUNCH();
}

// ---------------------------------------------------------------------------
// Mirror ghosts: a particle closer than r_max to a wall plane w gets an image
// at 2w - x with the normal velocity reversed; ghost ids follow (source id,
// wall index) order through an exclusive scan of per-particle counts.
// ---------------------------------------------------------------------------
__device__ __forceinline__ int ghost_walls(const DevCfg &cfg, const Soa &p, int i, double rmax, int *which) {
    int k = 0;
    for (int a = 0; a < cfg.D; ++a) {
        double x = p.x[a][i];
        if (cfg.wall_lo[a] && x - cfg.lo[a] < rmax) { if (which) which[k] = 2 * a; ++k; }
        if (cfg.wall_hi[a] && cfg.hi[a] - x < rmax) { if (which) which[k] = 2 * a + 1; ++k; }
    }
    return k;
}

__global__ void k_ghost_count(Soa p, DevCfg cfg, DevScalars *sc, uint32_t *gcnt) {
    int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= p.n) return;
    double rmax = bits_dbl(sc->rmax);
    gcnt[i] = p.m[i] > 0.0 ? (uint32_t)ghost_walls(cfg, p, i, rmax, nullptr) : 0u;  // absent: no ghost
}

void launch_ghost_count(const Soa &p, const DevCfg &cfg, DevScalars *sc, uint32_t *gcnt, hipStream_t st) {
    hipLaunchKernelGGL(k_ghost_count, dim3(blocks_for(p.n)), dim3(LP_BLOCK), 0, st, p, cfg, sc, gcnt);
    CHECK_LAUNCH();
}

__global__ void k_ghost_write(Soa p, DevCfg cfg, DevScalars *sc, const uint32_t *goff, const double *h,
                              const double *r, Ghosts g, long long cap_ghost) {
    int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= p.n || sc->n_total == 0) return;  // step skipped by k_gate
    double rmax = bits_dbl(sc->rmax);
    int which[6];
    int k = ghost_walls(cfg, p, i, rmax, which);
    uint32_t o = goff[i];
    for (int q = 0; q < k; ++q) {
        int a = which[q] >> 1;
        double w = (which[q] & 1) ? cfg.hi[a] : cfg.lo[a];
        uint32_t gi = o + q;
        if ((long long)gi >= cap_ghost) return;  // k_gate has already raised halt
        for (int b = 0; b < cfg.D; ++b) {
            double xb = p.x[b][i], ub = p.u[b][i];
            if (b == a) { xb = 2.0 * w - xb; ub = -ub; }
            g.x[b][gi] = xb;
            g.u[b][gi] = ub;
        }
        g.V[gi] = p.V[i];
        g.P[gi] = p.P[i];
        g.h[gi] = h[i];
        g.r[gi] = r[i];
    }
}

void launch_ghost_write(const Soa &p, const DevCfg &cfg, DevScalars *sc, const uint32_t *goff, const double *h,
                        const double *r, Ghosts g, int64_t cap_ghost, hipStream_t st) {
    hipLaunchKernelGGL(k_ghost_write, dim3(blocks_for(p.n)), dim3(LP_BLOCK), 0, st, p, cfg, sc, goff, h, r, g,
                       (long long)cap_ghost);
    CHECK_LAUNCH();
}

// ---------------------------------------------------------------------------
// Fill (used instead of memset so the sequence stays graph-safe).
// ---------------------------------------------------------------------------
__global__ void k_fill_u32(uint32_t *p, uint64_t n, uint32_t v, const unsigned *gate) {
    if (gate && *gate == 0u) return;
    uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
    uint64_t stride = (uint64_t)gridDim.x * blockDim.x;
    for (; i < n; i += stride) p[i] = v;
}

void launch_fill_u32(uint32_t *p, uint64_t n, uint32_t v, hipStream_t st, const unsigned *gate) {
    uint64_t b = (n + LP_BLOCK - 1) / LP_BLOCK;
    if (b > 65536) b = 65536;
    if (b < 1) b = 1;
    hipLaunchKernelGGL(k_fill_u32, dim3((unsigned)b), dim3(LP_BLOCK), 0, st, p, n, v, gate);
    CHECK_LAUNCH();
}

// ---------------------------------------------------------------------------
// Cell keys at the finest level + per-cell slot (counting-sort histogram).
// ---------------------------------------------------------------------------
template <int D>
__global__ void k_keys(const double *x0, const double *x1, const double *x2, const double *g0, const double *g1,
                       const double *g2, int n_real, const int *n_total_dev, DevGrid g, uint32_t *key,
                       uint32_t *slot, uint32_t *cnt, const unsigned *gate, const double *m) {
    if (gate && *gate == 0u) return;
    int i = blockIdx.x * blockDim.x + threadIdx.x;
    int n_total = *n_total_dev;
    if (i >= n_total) return;
    if (m && i < n_real && !(m[i] > 0.0)) {
        // absent: no cell and no slot (k_scatter skips it); the cell order
        // holds the present particles only
        key[i] = LP_KEY_ABSENT;
        slot[i] = 0u;
        return;
    }
    double p[3];
    if (i < n_real) { p[0] = x0[i]; p[1] = x1[i]; p[2] = D == 3 ? x2[i] : 0.0; }
    else { int q = i - n_real; p[0] = g0[q]; p[1] = g1[q]; p[2] = D == 3 ? g2[q] : 0.0; }
    int c[3] = {0, 0, 0};
    for (int a = 0; a < D; ++a) c[a] = cell_coord(g, g.L_hi, a, p[a]);
    const uint32_t k = morton<D>(c);
    key[i] = k;
    slot[i] = atomicAdd(&cnt[k], 1u);
}

void launch_keys(const double *const x[3], const double *const gx[3], int n_real, const int *n_total_dev,
                 int n_total_cap, const DevGrid &g, int D, uint32_t *key, uint32_t *slot, uint32_t *cnt,
                 hipStream_t st, const unsigned *gate, const double *m) {
    dim3 grid(blocks_for(n_total_cap));
    if (D == 3)
        hipLaunchKernelGGL(k_keys<3>, grid, dim3(LP_BLOCK), 0, st, x[0], x[1], x[2], gx[0], gx[1], gx[2], n_real,
                           n_total_dev, g, key, slot, cnt, gate, m);
    else
        hipLaunchKernelGGL(k_keys<2>, grid, dim3(LP_BLOCK), 0, st, x[0], x[1], x[1], gx[0], gx[1], gx[1], n_real,
                           n_total_dev, g, key, slot, cnt, gate, m);
    CHECK_LAUNCH();
}

// ---------------------------------------------------------------------------
// Exclusive scan of u32 (three passes: tile sums, scan of sums, tile scan).
// Tiles of 256 threads x 8 items; wave64 shuffles inside, LDS across waves.
// ---------------------------------------------------------------------------
#define SCAN_ITEMS 8
#define SCAN_TILE (LP_BLOCK * SCAN_ITEMS)

__device__ __forceinline__ uint32_t wave_incl_scan(uint32_t v) {
    int lane = threadIdx.x & 63;
    for (int o = 1; o < 64; o <<= 1) {
        uint32_t t = __shfl_up(v, o);
        if (lane >= o) v += t;
    }
    return v;
}

// block exclusive scan of one value per thread; returns exclusive prefix, sets *total
__device__ __forceinline__ uint32_t block_excl_scan(uint32_t v, uint32_t *total) {
    __shared__ uint32_t wsum[LP_BLOCK / 64];
    int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
    uint32_t inc = wave_incl_scan(v);
    if (lane == 63) wsum[w] = inc;
    __syncthreads();
    uint32_t off = 0, tot = 0;
    for (int q = 0; q < LP_BLOCK / 64; ++q) {
        if (q < w) off += wsum[q];
        tot += wsum[q];
    }
    __syncthreads();
    *total = tot;
    return off + inc - v;
}

__global__ void k_scan_tiles(const uint32_t *data, uint64_t n, uint32_t *sums, const unsigned *gate) {
    if (gate && *gate == 0u) return;
    uint64_t base = (uint64_t)blockIdx.x * SCAN_TILE;
    uint32_t s = 0;
    for (int k = 0; k < SCAN_ITEMS; ++k) {
        uint64_t i = base + (uint64_t)k * LP_BLOCK + threadIdx.x;
        if (i < n) s += data[i];
    }
    // block reduce
    for (int o = 32; o > 0; o >>= 1) s += __shfl_xor(s, o);
    __shared__ uint32_t ws[LP_BLOCK / 64];
    if ((threadIdx.x & 63) == 0) ws[threadIdx.x >> 6] = s;
    __syncthreads();
    if (threadIdx.x == 0) {
        uint32_t t = 0;
        for (int q = 0; q < LP_BLOCK / 64; ++q) t += ws[q];
        sums[blockIdx.x] = t;
    }
}

// one block of 1024 threads: exclusive scan of the tile sums in place, total to
// sums[nt]; each thread scans a contiguous chunk sequentially.
__global__ __launch_bounds__(1024) void k_scan_sums(uint32_t *sums, uint64_t nt, const unsigned *gate) {
    if (gate && *gate == 0u) return;
    __shared__ uint32_t ws[16];
    uint64_t chunk = (nt + 1023) / 1024;
    uint64_t b = (uint64_t)threadIdx.x * chunk, e = b + chunk;
    if (e > nt) e = nt;
    uint32_t s = 0;
    for (uint64_t i = b; i < e; ++i) s += sums[i];
    int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
    uint32_t inc = wave_incl_scan(s);
    if (lane == 63) ws[w] = inc;
    __syncthreads();
    uint32_t off = 0, tot = 0;
    for (int q = 0; q < 16; ++q) {
        if (q < w) off += ws[q];
        tot += ws[q];
    }
    uint32_t run = off + inc - s;
    for (uint64_t i = b; i < e; ++i) {
        uint32_t v = sums[i];
        sums[i] = run;
        run += v;
    }
    if (threadIdx.x == 0) sums[nt] = tot;
}

__global__ void k_scan_apply(uint32_t *data, uint64_t n, const uint32_t *sums, int *total_dev,
                             const unsigned *gate) {
    if (gate && *gate == 0u) return;
    uint64_t base = (uint64_t)blockIdx.x * SCAN_TILE;
    // each thread owns SCAN_ITEMS consecutive items
    uint64_t first = base + (uint64_t)threadIdx.x * SCAN_ITEMS;
    uint32_t v[SCAN_ITEMS];
    uint32_t s = 0;
    for (int k = 0; k < SCAN_ITEMS; ++k) {
        uint64_t i = first + k;
        v[k] = i < n ? data[i] : 0u;
        s += v[k];
    }
    uint32_t tot;
    uint32_t ex = block_excl_scan(s, &tot) + sums[blockIdx.x];
    for (int k = 0; k < SCAN_ITEMS; ++k) {
        uint64_t i = first + k;
        if (i < n) data[i] = ex;
        ex += v[k];
    }
    if (blockIdx.x == gridDim.x - 1 && threadIdx.x == 0) {
        uint64_t nt = gridDim.x;
        data[n] = sums[nt];
        if (total_dev) *total_dev = (int)sums[nt];
    }
}

uint64_t scan_tmp_words(uint64_t n) { return (n + SCAN_TILE - 1) / SCAN_TILE + 2; }

void launch_scan_u32(uint32_t *data, uint64_t n, uint32_t *tmp, int *total_dev, hipStream_t st,
                     const unsigned *gate) {
    uint64_t nt = (n + SCAN_TILE - 1) / SCAN_TILE;
    if (nt < 1) nt = 1;
    hipLaunchKernelGGL(k_scan_tiles, dim3((unsigned)nt), dim3(LP_BLOCK), 0, st, data, n, tmp, gate);
    hipLaunchKernelGGL(k_scan_sums, dim3(1), dim3(1024), 0, st, tmp, nt, gate);
    hipLaunchKernelGGL(k_scan_apply, dim3((unsigned)nt), dim3(LP_BLOCK), 0, st, data, n, tmp, total_dev, gate);
    CHECK_LAUNCH();
}

// ---------------------------------------------------------------------------
// Scatter into cell order: pos = start[key] + slot.
// ---------------------------------------------------------------------------
__global__ void k_scatter(ScatterArgs a, int n_real, const int *n_total_dev, const uint32_t *key,
                          const uint32_t *slot, const uint32_t *start, int *sorted_id) {
    int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= *n_total_dev) return;
    const uint32_t ki = key[i];
    if (ki == LP_KEY_ABSENT) return;
    uint32_t pos = start[ki] + slot[i];
    sorted_id[pos] = i;
    bool real = i < n_real;
    // deleted since the cell order was built: it keeps its slot, out of every
    // distance test (infinite coordinates) and with no radius (k_prep)
    const bool gone = real && a.m && !(a.m[i] > 0.0);
    double vals[12];
    for (int d = 0; d < a.nd; ++d) {
        double v = real ? a.src[d][i] : (a.gsrc[d] ? a.gsrc[d][i - n_real] : 0.0);
        if (gone && d < 3) v = INFINITY;
        vals[d] = v;
        a.dst[d][pos] = v;
    }
    if (a.rec || a.recf) {
        double e[LP_REC];
#pragma unroll
        for (int q = 0; q < LP_REC; ++q) {
            e[q] = 0.0;
            for (int d = 0; d < 12; ++d)
                if (d == a.rec_src[q]) e[q] = vals[d];
        }
        if (a.rec) {
            // the particle's gather record: one 64-byte write
            double2 *r = reinterpret_cast<double2 *>(a.rec + (int64_t)LP_REC * pos);
#pragma unroll
            for (int q = 0; q < LP_REC / 2; ++q) r[q] = make_double2(e[2 * q], e[2 * q + 1]);
        }
        if (a.recf) {
            // the FP32-field record: positions, then the fields rounded to FP32
            uint4 *r = reinterpret_cast<uint4 *>(reinterpret_cast<char *>(a.recf) + (int64_t)LP_RECF_BYTES * pos);
            auto lo = [](double v) { return (unsigned)__double2loint(v); };
            auto hi = [](double v) { return (unsigned)__double2hiint(v); };
            auto fb = [](double v) { return __float_as_uint((float)v); };
            r[0] = make_uint4(lo(e[0]), hi(e[0]), lo(e[1]), hi(e[1]));
            if (a.dim == 3) {
                r[1] = make_uint4(lo(e[2]), hi(e[2]), fb(e[3]), fb(e[4]));
                r[2] = make_uint4(fb(e[5]), fb(e[6]), fb(e[7]), 0u);
            } else {
                r[1] = make_uint4(fb(e[2]), fb(e[3]), fb(e[4]), fb(e[5]));
                r[2] = make_uint4(0u, 0u, 0u, 0u);
            }
        }
    }
}

void launch_scatter(const ScatterArgs &a, int n_real, const int *n_total_dev, int n_total_cap, const uint32_t *key,
                    const uint32_t *slot, const uint32_t *start, int *sorted_id, hipStream_t st) {
    hipLaunchKernelGGL(k_scatter, dim3(blocks_for(n_total_cap)), dim3(LP_BLOCK), 0, st, a, n_real, n_total_dev,
                       key, slot, start, sorted_id);
    CHECK_LAUNCH();
}

// ---------------------------------------------------------------------------
// Coarser cell tables: the first particle of a cell is the first particle of
// its first child.
// ---------------------------------------------------------------------------
__global__ void k_coarsen(uint32_t *dst, const uint32_t *src, uint64_t ncell, int D, const int *n_total_dev,
                          const unsigned *gate) {
    if (gate && *gate == 0u) return;
    uint64_t c = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (c < ncell) dst[c] = src[c << D];
    else if (c == ncell) dst[c] = (uint32_t)*n_total_dev;
}

void launch_coarsen(uint32_t *tables, const DevGrid &g, int D, const int *n_total_dev, hipStream_t st,
                    const unsigned *gate) {
    for (int L = g.L_hi - 1; L >= g.L_lo; --L) {
        uint64_t ncell = 1ull << (D * L);
        hipLaunchKernelGGL(k_coarsen, dim3(blocks_for(ncell + 1)), dim3(LP_BLOCK), 0, st, tables + g.off[L],
                           tables + g.off[L + 1], ncell, D, n_total_dev, gate);
    }
    CHECK_LAUNCH();
}

// ---------------------------------------------------------------------------
// Neighbour-list reuse.  A rebuild step finds, for every particle, the
// candidates within R_i = rscale r_i; later steps filter them exactly.  That
// filter misses no neighbour while |x_j - x_i| < r_i now implies
// |x_j - x_i| < R_i at the rebuild, which the triangle inequality guarantees
// when r_i + d_i + d_j < R_i for all i, j (d: displacement since the rebuild):
// max_i (r_i + d_i - R_i) + max_j d_j < 0, checked with a margin of 1e-9 of
// the smallest radius against rounding (the two maxima are reduced by k_prep
// in the same pass as the radii).
// ---------------------------------------------------------------------------
__global__ void k_reuse_decide(DevScalars *sc, int force) {
    unsigned rb = 0u;
    if (sc->n_total > 0) {
        if (force || !sc->have_cand || sc->cand_short || sc->pop_changed) rb = 1u;
        else {
            const unsigned long long ka = sc->reuse_a;
            const double a = (ka >> 63) ? bits_dbl(ka & 0x7fffffffffffffffull) : bits_dbl(~ka);
            const double d = bits_dbl(sc->reuse_d);
            const double rmin = bits_dbl(sc->rmin);
            rb = (a + d < -1e-9 * rmin) ? 0u : 1u;
        }
    }
    sc->rebuild = rb;
    if (sc->n_total > 0) {
        sc->pop_changed = 0u;  // the cells of this step see the particles as they are
        // a rebuild orders the present particles; otherwise the order of the
        // last build stands, particles deleted since then included (they are
        // skipped by every kernel that takes a particle from it)
        if (rb) sc->n_sorted = sc->n_total;
        else sc->n_total = sc->n_sorted;
    }
    if (rb) {
        sc->have_cand = 1u;
        sc->n_builds += 1ull;
        sc->max_cand = 0;
        sc->cand_short = 0u;
    }
    sc->reuse_a = 0ull;
    sc->reuse_d = 0ull;
}

__global__ void k_reuse_commit(Soa p, DevCfg cfg, const double *r, double *xb0, double *xb1, double *xb2, double *Rb,
                               double rscale, const DevScalars *sc) {
    if (!sc->rebuild) return;
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= p.n) return;
    xb0[i] = p.x[0][i];
    xb1[i] = p.x[1][i];
    if (cfg.D == 3) xb2[i] = p.x[2][i];
    Rb[i] = r[i] * rscale;
}

void launch_reuse(const Soa &p, const DevCfg &cfg, const double *r, double *const xb[3], double *Rb, int n,
                  double rscale, int force, DevScalars *sc, hipStream_t st) {
    dim3 grid(blocks_for((uint64_t)n));
    double *x2 = cfg.D == 3 ? xb[2] : xb[0];
    // the check's maxima come from k_prep of the same step
    hipLaunchKernelGGL(k_reuse_decide, dim3(1), dim3(1), 0, st, sc, force);
    hipLaunchKernelGGL(k_reuse_commit, grid, dim3(LP_BLOCK), 0, st, p, cfg, r, xb[0], xb[1], x2, Rb, rscale, sc);
    CHECK_LAUNCH();
}

// ---------------------------------------------------------------------------
// Neighbour lists back to the caller's indexing.
// ---------------------------------------------------------------------------
__global__ void k_lists_out(const int *sorted_id, const int *nbr, int ldn, const int *count, int n, int max_nb,
                            int *count_out, int *idx_out) {
    int s = blockIdx.x * blockDim.x + threadIdx.x;
    if (s >= n) return;
    int i = sorted_id[s];
    int k = count[s];
    count_out[i] = k;
    int kk = k < max_nb ? k : max_nb;
    for (int c = 0; c < kk; ++c) idx_out[(int64_t)i * max_nb + c] = sorted_id[nb_at(nbr, ldn, s, c)];
}

void launch_lists_out(const int *sorted_id, const int *nbr, int ldn, const int *count, int n, int max_nb,
                      int *count_out, int *idx_out, hipStream_t st) {
    hipLaunchKernelGGL(k_lists_out, dim3(blocks_for(n)), dim3(LP_BLOCK), 0, st, sorted_id, nbr, ldn, count, n, max_nb,
                       count_out, idx_out);
    CHECK_LAUNCH();
}

// ---------------------------------------------------------------------------
// Conservation totals in FP64 with a fixed reduction order (deterministic):
// per-block tree sums over the caller's order, then one block sums the partials.
// ---------------------------------------------------------------------------
__global__ void k_cons_partial(Soa p, DevCfg cfg, double *partials) {
    __shared__ double sh[5][LP_BLOCK];
    double acc[5] = {0, 0, 0, 0, 0};
    int stride = gridDim.x * blockDim.x;
    for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < p.n; i += stride) {
        double m = p.m[i], V = p.V[i], P = p.P[i];
        double u0 = p.u[0][i], u1 = p.u[1][i], u2 = cfg.D == 3 ? p.u[2][i] : 0.0;
        double e = P * V / (cfg.gamma - 1.0);
        double ke = 0.5 * (u0 * u0 + u1 * u1 + u2 * u2);
        acc[0] += m;
        acc[1] += m * u0;
        acc[2] += m * u1;
        acc[3] += m * u2;
        acc[4] += m * (e + ke);
    }
    for (int q = 0; q < 5; ++q) sh[q][threadIdx.x] = acc[q];
    __syncthreads();
    for (int o = LP_BLOCK / 2; o > 0; o >>= 1) {
        if (threadIdx.x < o)
            for (int q = 0; q < 5; ++q) sh[q][threadIdx.x] += sh[q][threadIdx.x + o];
        __syncthreads();
    }
    if (threadIdx.x < 5) partials[blockIdx.x * 5 + threadIdx.x] = sh[threadIdx.x][0];
}

__global__ void k_cons_final(const double *partials, int nblocks, double *out) {
    if (threadIdx.x < 5) {
        double s = 0.0;
        for (int b = 0; b < nblocks; ++b) s += partials[b * 5 + threadIdx.x];
        out[threadIdx.x] = s;
    }
}

void launch_conservation(const Soa &p, const DevCfg &cfg, double *partials, int nblocks, double *out,
                         hipStream_t st) {
    hipLaunchKernelGGL(k_cons_partial, dim3(nblocks), dim3(LP_BLOCK), 0, st, p, cfg, partials);
    hipLaunchKernelGGL(k_cons_final, dim3(1), dim3(64), 0, st, partials, nblocks, out);
    CHECK_LAUNCH();
}

// ---------------------------------------------------------------------------
// Open boundaries (Sec. 2.2, step 1: outflow by deleting particles; Sec. 3.2:
// the state of particles entering from a reservoir).
// ---------------------------------------------------------------------------
// keep[i] = 1 for a particle inside every outflow face (x_a >= lo_a for a bit a
// of lo_mask, x_a < hi_a for a bit a of hi_mask), else 0
__global__ void k_out_keep(Soa p, DevCfg cfg, uint32_t lo_mask, uint32_t hi_mask, uint32_t *keep) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= p.n) return;
    bool gone = false;
    for (int a = 0; a < cfg.D; ++a) {
        const double xa = p.x[a][i];
        if (((lo_mask >> a) & 1u) && xa < cfg.lo[a]) gone = true;
        if (((hi_mask >> a) & 1u) && xa >= cfg.hi[a]) gone = true;
    }
    keep[i] = gone ? 0u : 1u;
}

// Outflow compaction through a staging area: slot k (n entries) holds array k
// of x[0..D-1], u[0..D-1], V, P, m, then n floats of phi and n bytes of flags.
// After the exclusive scan of keep (pos[n] = particles kept), every kept
// particle's entries go, in order, to the staging area ...
__global__ void k_out_gather_all(Soa p, int D, const uint32_t *pos, double *tmp) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= p.n) return;
    const uint32_t q = pos[i];
    if (pos[i + 1] == q) return;
    const size_t n = (size_t)p.n;
    double *t = tmp + q;
    for (int a = 0; a < D; ++a) t[a * n] = p.x[a][i];
    for (int a = 0; a < D; ++a) t[(D + a) * n] = p.u[a][i];
    t[2 * D * n] = p.V[i];
    t[(2 * D + 1) * n] = p.P[i];
    t[(2 * D + 2) * n] = p.m[i];
    if (p.phi) reinterpret_cast<float *>(tmp + (2 * D + 3) * n)[q] = p.phi[i];
    if (p.flags) reinterpret_cast<uint8_t *>(tmp + (2 * D + 3) * n + (n + 1) / 2)[q] = p.flags[i];
}

// ... and back to the front of the caller's arrays
__global__ void k_out_copy_back(Soa p, int D, uint32_t kept, const double *tmp) {
    const uint32_t q = blockIdx.x * blockDim.x + threadIdx.x;
    if (q >= kept) return;
    const size_t n = (size_t)p.n;
    const double *t = tmp + q;
    for (int a = 0; a < D; ++a) p.x[a][q] = t[a * n];
    for (int a = 0; a < D; ++a) p.u[a][q] = t[(D + a) * n];
    p.V[q] = t[2 * D * n];
    p.P[q] = t[(2 * D + 1) * n];
    const_cast<double *>(p.m)[q] = t[(2 * D + 2) * n];
    if (p.phi) p.phi[q] = reinterpret_cast<const float *>(tmp + (2 * D + 3) * n)[q];
    if (p.flags) p.flags[q] = reinterpret_cast<const uint8_t *>(tmp + (2 * D + 3) * n + (n + 1) / 2)[q];
}

void launch_out_keep(const Soa &p, const DevCfg &cfg, uint32_t lo_mask, uint32_t hi_mask, uint32_t *keep,
                     hipStream_t st) {
    hipLaunchKernelGGL(k_out_keep, dim3(blocks_for(p.n)), dim3(LP_BLOCK), 0, st, p, cfg, lo_mask, hi_mask, keep);
    CHECK_LAUNCH();
}

size_t out_stage_bytes(int D, int64_t n) {
    return sizeof(double) * ((size_t)(2 * D + 3) * n + (n + 1) / 2) + (size_t)n;
}

void launch_out_compact(const Soa &p, int D, const uint32_t *pos, uint32_t kept, double *tmp, hipStream_t st) {
    hipLaunchKernelGGL(k_out_gather_all, dim3(blocks_for(p.n)), dim3(LP_BLOCK), 0, st, p, D, pos, tmp);
    if (kept > 0)
        hipLaunchKernelGGL(k_out_copy_back, dim3(blocks_for((int)kept)), dim3(LP_BLOCK), 0, st, p, D, kept,
                           (const double *)tmp);
    CHECK_LAUNCH();
}

// Inflow layer: particle n + q sits at lattice point q (the first other axis
// fastest) of the face plane at depth `depth` inside the face.  Each position
// is one rounded product and one rounded sum: contraction into a fused
// multiply-add is off here, as it would change the last bit.
__global__ void k_inflow_layer(Soa p, DevCfg cfg, int64_t n0, int64_t count, int64_t cnt0, int axis, int o0, int o1,
                               double spacing, double xa, double un, double V, double P, double mass) {
#pragma clang fp contract(off)
    const int64_t q = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (q >= count) return;
    const int64_t i = n0 + q;
    const int64_t k[2] = {q % cnt0, q / cnt0};
    const int oth[2] = {o0, o1};
    for (int a = 0; a < cfg.D; ++a) p.u[a][i] = 0.0;
    p.x[axis][i] = xa;
    p.u[axis][i] = un;
    for (int t = 0; t < cfg.D - 1; ++t) {
        const double off = ((double)k[t] + 0.5) * spacing;
        p.x[oth[t]][i] = cfg.lo[oth[t]] + off;
    }
    p.V[i] = V;
    p.P[i] = P;
    const_cast<double *>(p.m)[i] = mass;
    if (p.phi) p.phi[i] = 1.0f;
    if (p.flags) p.flags[i] = 0;
}

void launch_inflow_layer(const Soa &p, const DevCfg &cfg, int64_t n0, int64_t count, int64_t cnt0, int axis, int o0,
                         int o1, double spacing, double xa, double un, double V, double P, double mass,
                         hipStream_t st) {
    const int64_t nb = (count + LP_BLOCK - 1) / LP_BLOCK;
    hipLaunchKernelGGL(k_inflow_layer, dim3((unsigned)nb), dim3(LP_BLOCK), 0, st, p, cfg, n0, count, cnt0, axis, o0,
                       o1, spacing, xa, un, V, P, mass);
    CHECK_LAUNCH();
}

// Inlet layer of the face (side 0: lo, 1: hi): per block the sum of P and the
// count of the particles at distance 0 <= d < width inside the face, in a
// fixed order (grid-stride per thread, then the wave, then the block's waves)
__global__ __launch_bounds__(LP_BLOCK) void k_res_partial(const double *xa, const double *P, int n, int side,
                                                         double face, double width, double *part,
                                                         const double *m, const unsigned *gate) {
    if (gate && *gate == 0u) return;
    __shared__ double red[2][LP_BLOCK / 64];
    double sum = 0.0, cnt = 0.0;
    for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < n; i += gridDim.x * blockDim.x) {
        const double d = side == 0 ? xa[i] - face : face - xa[i];
        if (d >= 0.0 && d < width && (!m || m[i] > 0.0)) {  // m: absent particles do not count
            sum += P[i];
            cnt += 1.0;
        }
    }
    for (int o = 32; o > 0; o >>= 1) {
        sum += __shfl_xor(sum, o);
        cnt += __shfl_xor(cnt, o);
    }
    const int w = threadIdx.x >> 6;
    if ((threadIdx.x & 63) == 0) {
        red[0][w] = sum;
        red[1][w] = cnt;
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        double a = 0.0, b = 0.0;
        for (int k = 0; k < LP_BLOCK / 64; ++k) {
            a += red[0][k];
            b += red[1][k];
        }
        part[2 * blockIdx.x] = a;
        part[2 * blockIdx.x + 1] = b;
    }
}

// the reservoir inflow state from the block sums: the layer's mean pressure
// (the reservoir's with an empty layer), the density of equal entropy and
// the speed of equal enthalpy with the reservoir at rest
__global__ void k_res_final(const double *part, int nblocks, double p_res, double rho_res, double gamma,
                            double *out, const unsigned *gate) {
    if (gate && *gate == 0u) return;
    double sum = 0.0, cnt = 0.0;
    for (int b = 0; b < nblocks; ++b) {
        sum += part[2 * b];
        cnt += part[2 * b + 1];
    }
    const double p_in = cnt > 0.0 ? sum / cnt : p_res;
    const double rho_in = rho_res * pow(p_in / p_res, 1.0 / gamma);
    const double c2_res = gamma * p_res / rho_res, c2_in = gamma * p_in / rho_in;
    const double u2 = 2.0 * (c2_res - c2_in) / (gamma - 1.0);
    out[0] = p_in;
    out[1] = rho_in;
    out[2] = u2 > 0.0 ? sqrt(u2) : 0.0;
    out[3] = cnt;
}

void launch_reservoir(const double *xa, const double *P, int n, int side, double face, double width, double p_res,
                      double rho_res, double gamma, double *part, int nblocks, double *out, hipStream_t st) {
    hipLaunchKernelGGL(k_res_partial, dim3(nblocks), dim3(LP_BLOCK), 0, st, xa, P, n, side, face, width, part,
                       (const double *)nullptr, (const unsigned *)nullptr);
    hipLaunchKernelGGL(k_res_final, dim3(1), dim3(1), 0, st, part, nblocks, p_res, rho_res, gamma, out,
                       (const unsigned *)nullptr);
    CHECK_LAUNCH();
}

// ---------------------------------------------------------------------------
// Open boundaries inside the steps of lp_run_open (Sec. 2.2, step 1).  A
// particle of zero mass is absent: no radius, no ghost, no place in the cell
// order, never updated.  At the end of a step that ran (n_total >
// 0): every present particle past an outflow face gets mass 0; the step is
// counted; after every in_every-th step one inflow layer is written at slot
// n_hw (the state fixed, or the reservoir state of the layer inside the face
// as lp_reservoir_inflow computes it) and n_hw advances.  Any deletion or
// layer raises pop_changed, which makes the next step rebuild its lists.
// ---------------------------------------------------------------------------
__global__ void k_open_outflow(Soa p, DevCfg cfg, OpenDev o, DevScalars *sc) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (sc->n_total > 0 && i < p.n && p.m[i] > 0.0) {
        bool gone = false;
        for (int a = 0; a < cfg.D; ++a) {
            const double xa = p.x[a][i];
            if (((o.lo_mask >> a) & 1u) && xa < cfg.lo[a]) gone = true;
            if (((o.hi_mask >> a) & 1u) && xa >= cfg.hi[a]) gone = true;
        }
        if (gone) const_cast<double *>(p.m)[i] = 0.0;
    }
}

__global__ void k_open_tick(DevScalars *sc, int every) {
    if (sc->n_total == 0) {  // skipped step: nothing ran, nothing to add
        sc->insert_now = 0u;
        return;
    }
    sc->open_k += 1ull;
    sc->insert_now = (every > 0 && sc->open_k % (unsigned long long)every == 0ull) ? 1u : 0u;
}

// lattice point q of the layer at slot n_hw + q, with the state given or from
// the reservoir outputs: the same rounding as k_inflow_layer and lp_inflow_layer
__global__ void k_open_inflow(Soa p, DevCfg cfg, OpenDev o, DevScalars *sc) {
#pragma clang fp contract(off)
    if (!sc->insert_now) return;
    const int64_t n0 = sc->n_hw;
    if (n0 + o.count > o.cap) {
        if (blockIdx.x == 0 && threadIdx.x == 0) atomicOr(&sc->error_bits, 4u);
        return;
    }
    const int64_t q = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (q >= o.count) return;
    double un = o.un, V = o.V, P = o.P, mass = o.mass;
    if (o.res_width > 0.0) {
        const double *out = o.res_part + 2 * o.res_blocks;
        const double rho = out[1];
        P = out[0];
        V = 1.0 / rho;
        un = o.side == 0 ? out[2] : -out[2];
        mass = rho;
        for (int a = 0; a < cfg.D; ++a) mass = mass * o.spacing;
    }
    const int64_t i = n0 + q;
    const int64_t k[2] = {q % o.cnt0, q / o.cnt0};
    const int oth[2] = {o.o0, o.o1};
    for (int a = 0; a < cfg.D; ++a) p.u[a][i] = 0.0;
    p.x[o.axis][i] = o.xa;
    p.u[o.axis][i] = un;
    for (int t = 0; t < cfg.D - 1; ++t) {
        const double off = ((double)k[t] + 0.5) * o.spacing;
        p.x[oth[t]][i] = cfg.lo[oth[t]] + off;
    }
    p.V[i] = V;
    p.P[i] = P;
    const_cast<double *>(p.m)[i] = mass;
    if (p.phi) p.phi[i] = 1.0f;
    if (p.flags) p.flags[i] = 0;
}

__global__ void k_open_commit(OpenDev o, DevScalars *sc) {
    if (sc->insert_now && sc->n_hw + o.count <= o.cap) {
        sc->n_hw += (int)o.count;
        if (o.count > 0) sc->pop_changed = 1u;
    }
}

void launch_open_end(const Soa &p, const DevCfg &cfg, const OpenDev &o, DevScalars *sc, hipStream_t st) {
    hipLaunchKernelGGL(k_open_outflow, dim3(blocks_for(p.n)), dim3(LP_BLOCK), 0, st, p, cfg, o, sc);
    hipLaunchKernelGGL(k_open_tick, dim3(1), dim3(1), 0, st, sc, o.in_every);
    if (o.in_every > 0 && o.count > 0) {
        if (o.res_width > 0.0) {
            const unsigned *gate = &sc->insert_now;
            hipLaunchKernelGGL(k_res_partial, dim3(o.res_blocks), dim3(LP_BLOCK), 0, st, (const double *)p.x[o.axis],
                               (const double *)p.P, p.n, o.side, o.res_face, o.res_width, o.res_part, p.m, gate);
            hipLaunchKernelGGL(k_res_final, dim3(1), dim3(1), 0, st, (const double *)o.res_part, o.res_blocks,
                               o.res_p, o.res_rho, o.gamma, o.res_part + 2 * o.res_blocks, gate);
        }
        const int64_t nb = (o.count + LP_BLOCK - 1) / LP_BLOCK;
        hipLaunchKernelGGL(k_open_inflow, dim3((unsigned)nb), dim3(LP_BLOCK), 0, st, p, cfg, o, sc);
        hipLaunchKernelGGL(k_open_commit, dim3(1), dim3(1), 0, st, o, sc);
    }
    CHECK_LAUNCH();
}

__global__ void k_alive_keep(Soa p, uint32_t *keep) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i < p.n) keep[i] = p.m[i] > 0.0 ? 1u : 0u;
}

void launch_alive_keep(const Soa &p, uint32_t *keep, hipStream_t st) {
    hipLaunchKernelGGL(k_alive_keep, dim3(blocks_for(p.n)), dim3(LP_BLOCK), 0, st, p, keep);
    CHECK_LAUNCH();
}
