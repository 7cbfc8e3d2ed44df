// lp_search.hip -- neighbour search (Sec. 2.2, step 3) on gfx950.
//
// A group of G lanes serves one particle of the cell-ordered array.  The
// particle picks the grid level whose cells are just below its radius, and the
// group walks the 3^D..5^D cells that cover its search box: lanes take cells
// round-robin, read each cell's contiguous run of particles (cell order keeps
// a group's candidates, and a wave's, inside a few cache lines), and test
// d2 < r^2 exactly in FP64.  Hits are appended to a per-particle buffer in LDS
// and then ranked in LDS by (d2, original id), so the list written out is the
// unique (d2, id) order whatever order the lanes found the hits in.
// Output: nbr[c * ldn + s] (column-major in the list position c, so the solver
// reads it coalesced) holds cell-order indices; count[s] is the true count.
#include "lp_internal.h"

// Entry c of the list of cell-order particle s: ldn > 0 column-major
// (c * ldn + s), ldn < 0 row-major (s * (-ldn) + c), ldn == 0 interleaved by
// eight particles, (s / 8) * 8 max_nb + 8 c + s % 8, the layout of the
// candidate lists: the eight lane groups of a wave reading entries c0 .. c0 + 7
// of their particles read 64 consecutive entries.
__device__ __forceinline__ int64_t list_at(int ldn, int s, int c, int max_nb) {
    if (ldn > 0) return (int64_t)c * ldn + s;
    if (ldn < 0) return (int64_t)s * (-ldn) + c;
    return (int64_t)(s >> 3) * (8 * max_nb) + 8 * c + (s & 7);
}

// Cells of level L that cover [x - r, x + r] per axis: first cell and count.
template <int D>
__device__ __forceinline__ void search_box(const DevGrid &g, const DevCfg &cfg, int L, const double xi[3], double ri,
                                           int clo[3], int cn[3]) {
    for (int a = 0; a < D; ++a) {
        int n = g.nc[L][a];
        // inv_s[L] = 2^L / S, an exact power-of-two scaling of the first level's
        const double inv = ldexp(g.inv_s[g.L_lo], L - g.L_lo);
        double tl = (xi[a] - ri - g.lo[a]) * inv;
        double th = (xi[a] + ri - g.lo[a]) * inv;
        int lo = floor_clamped(tl - 1e-9), hi = floor_clamped(th + 1e-9);
        if (cfg.periodic[a]) {
            if (hi - lo + 1 >= n || hi < lo) { lo = 0; hi = n - 1; }
        } else {
            // particles outside the grid sit in its edge cells, so the
            // clamped range still covers every candidate
            lo = lo < 0 ? 0 : (lo > n - 1 ? n - 1 : lo);
            hi = hi > n - 1 ? n - 1 : (hi < 0 ? 0 : hi);
        }
        clo[a] = lo;
        cn[a] = hi - lo + 1;
    }
}

// Morton code of the c-th cell of a search box (periodic axes wrapped).
template <int D>
__device__ __forceinline__ uint32_t cell_code(const DevGrid &g, const DevCfg &cfg, int L, const int clo[3],
                                              const int cn[3], int c) {
    int cc[3];
    cc[0] = clo[0] + c % cn[0];
    cc[1] = clo[1] + (c / cn[0]) % cn[1];
    cc[2] = D == 3 ? clo[2] + c / (cn[0] * cn[1]) : 0;
    for (int a = 0; a < D; ++a)
        if (cfg.periodic[a]) {
            int n = g.nc[L][a];
            cc[a] = ((cc[a] % n) + n) % n;
        }
    return morton<D>(cc);
}

template <int D, int G>
__global__ __launch_bounds__(LP_BLOCK) void k_search(Sorted srt, const int *n_total_dev, int n_real,
                                                     const uint32_t *tables, DevGrid g, DevCfg cfg, int *nbr, int ldn,
                                                     int *count, DevScalars *sc, int lcap, int *ovf_queue,
                                                     double rscale, const unsigned *gate, int *max_out) {
    if (gate && *gate == 0u) return;
    constexpr int PPB = LP_BLOCK / G;
    extern __shared__ unsigned char smem[];
    const int max_nb = cfg.max_nb;
    double *ld2 = reinterpret_cast<double *>(smem);
    int *lj = reinterpret_cast<int *>(ld2 + PPB * lcap);
    int *lcnt = lj + PPB * lcap;

    const int lane = threadIdx.x % G;
    const int grp = threadIdx.x / G;
    const int s = xcd_remap(blockIdx.x, gridDim.x) * PPB + grp;
    const int n_total = *n_total_dev;
    const bool active = s < n_total && srt.id[s] < n_real;
    double *gd2 = ld2 + grp * lcap;
    int *gj = lj + grp * lcap;
    if (lane == 0) lcnt[grp] = 0;
    __syncthreads();

    if (active) {
        double xi[3] = {srt.x[0][s], srt.x[1][s], D == 3 ? srt.x[2][s] : 0.0};
        double ri = srt.r[s] * rscale;
        double r2 = ri * ri;
        int L = level_for_radius(g, ri);
        const uint32_t *tab = tables + g.off[L];
        int clo[3] = {0, 0, 0}, cn[3] = {1, 1, 1};
        search_box<D>(g, cfg, L, xi, ri, clo, cn);
        const int ncells = cn[0] * cn[1] * (D == 3 ? cn[2] : 1);
        for (int c = lane; c < ncells; c += G) {
            uint32_t code = cell_code<D>(g, cfg, L, clo, cn, c);
            uint32_t b = tab[code], e = tab[code + 1];
            for (uint32_t j = b; j < e; ++j) {
                if ((int)j == s) continue;
                double dx[3];
                disp_to<D>(cfg, srt.x, j, xi, dx);
                double d2 = dist2_exact<D>(dx);
                if (d2 < r2) {
                    int slot = atomicAdd(&lcnt[grp], 1);
                    if (slot < lcap) {
                        gd2[slot] = d2;
                        gj[slot] = (int)j;
                    }
                }
            }
        }
    }
    __syncthreads();
    {
        int kmax = active ? lcnt[grp] : 0;
        for (int o = 32; o > 0; o >>= 1) kmax = max(kmax, __shfl_xor(kmax, o));
        // the atomic only when it can raise the maximum: same-address atomics
        // serialise in L2, and one per wave costs milliseconds at 2M particles
        if ((threadIdx.x & 63) == 0 && kmax > __hip_atomic_load(max_out, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT))
            atomicMax(max_out, kmax);
    }
    if (active) {
        int k = lcnt[grp];
        if (lane == 0) {
            count[s] = k;
            if (k > max_nb) atomicOr(&sc->error_bits, 1u);
            // the list does not fit the LDS buffer: one wave redoes it (and
            // for k > max_nb writes max_nb valid entries, so readers stay in bounds)
            if (k > lcap) ovf_queue[atomicAdd(&sc->n_overflow, 1)] = s;
        }
        if (k <= lcap) {
            for (int e = lane; e < k; e += G) {
                double de = gd2[e];
                int je = gj[e];
                int rank = 0;
                for (int f = 0; f < k; ++f) {
                    double df = gd2[f];
                    if (df < de) ++rank;
                    else if (df == de && f != e && srt.id[gj[f]] < srt.id[je]) ++rank;  // exact tie: id order
                }
                nbr[list_at(ldn, s, rank, cfg.max_nb)] = je;
            }
        }
    }
}

// Lists longer than the LDS buffer of k_search: one wave per particle, a
// buffer of max_nb entries.
template <int D>
__global__ __launch_bounds__(64) void k_search_overflow(Sorted srt, const uint32_t *tables, DevGrid g, DevCfg cfg,
                                                         int *nbr, int ldn, DevScalars *sc, const int *ovf_queue,
                                                         double rscale, const unsigned *gate) {
    if (gate && *gate == 0u) return;
    __shared__ double gd2[256];
    __shared__ int gj[256];
    __shared__ int lcnt;
    const int lane = threadIdx.x;
    const int nq = sc->n_overflow;
    for (int w = blockIdx.x; w < nq; w += gridDim.x) {
        const int s = ovf_queue[w];
        if (lane == 0) lcnt = 0;
        __syncthreads();
        double xi[3] = {srt.x[0][s], srt.x[1][s], D == 3 ? srt.x[2][s] : 0.0};
        double ri = srt.r[s] * rscale;
        double r2 = ri * ri;
        int L = level_for_radius(g, ri);
        const uint32_t *tab = tables + g.off[L];
        int clo[3] = {0, 0, 0}, cn[3] = {1, 1, 1};
        search_box<D>(g, cfg, L, xi, ri, clo, cn);
        const int ncells = cn[0] * cn[1] * (D == 3 ? cn[2] : 1);
        for (int c = lane; c < ncells; c += 64) {
            uint32_t code = cell_code<D>(g, cfg, L, clo, cn, c);
            uint32_t b = tab[code], e = tab[code + 1];
            for (uint32_t j = b; j < e; ++j) {
                if ((int)j == s) continue;
                double dx[3];
                disp_to<D>(cfg, srt.x, j, xi, dx);
                double d2 = dist2_exact<D>(dx);
                if (d2 < r2) {
                    int slot = atomicAdd(&lcnt, 1);
                    if (slot < cfg.max_nb) {
                        gd2[slot] = d2;
                        gj[slot] = (int)j;
                    }
                }
            }
        }
        __syncthreads();
        int k = lcnt < cfg.max_nb ? lcnt : cfg.max_nb;
        for (int e = lane; e < k; e += 64) {
            double de = gd2[e];
            int je = gj[e];
            int rank = 0;
            for (int f = 0; f < k; ++f) {
                double df = gd2[f];
                if (df < de) ++rank;
                else if (df == de && f != e && srt.id[gj[f]] < srt.id[je]) ++rank;
            }
            nbr[list_at(ldn, s, rank, cfg.max_nb)] = je;
        }
        __syncthreads();
    }
}

// Balanced variant: the group prunes the cells of the search box whose box
// lies provably outside the ball, prefix-sums the candidate counts of the rest
// (G cells at a time) and deals the candidates out so that in every round each
// lane tests exactly one -- consecutive lanes test consecutive particles of a
// cell, so the position loads coalesce.  Hits are compacted with a ballot and
// ranked by a counting sort on a monotone bucket of d2 followed by exact
// (d2, original id) comparisons inside each bucket, so the list is the same
// unique (d2, id) order as k_search's.  A hit is staged as the FP32 rounding
// of its d2 (round to nearest is monotone, so a smaller key means a smaller
// d2); only hits whose keys tie recompute their exact FP64 d2 for the order.
#define SB_NB 32  // rank buckets per particle
// 16-bit counters per group in LDS: SB_NB plus one padding word, so that the
// groups of a wave start on different banks
#define SB_GSTRIDE (SB_NB + 2)

// c = q * n + rem for 0 <= c < 2^24 without an integer division (the FP32
// quotient is off by at most one either way; corrected without branches)
__device__ __forceinline__ int div_small(int c, int n, float rcp, int &rem) {
    int q = (int)((float)c * rcp);
    int r = c - q * n;
    const int lo = r < 0 ? 1 : 0, hi = r >= n ? 1 : 0;
    q += hi - lo;
    rem = r + (lo - hi) * n;
    return q;
}

// LDS layout shared by k_search_bal and k_filter_bal (per group of G lanes):
// lcap + 1 FP32 keys and indices, a byte permutation, SB_NB 16-bit bucket
// counters (two to a word: the counting adds 1 << 16 for an odd bucket, and
// no count exceeds the 256 entries of a list).
struct BalLds {
    float *gkey;
    int *gj;
    unsigned char *gperm;
    unsigned short *gbk;
    int *lout, *lk;  // after ranking: the block's ranked lists and their lengths
};

// bucket bb's counter += 1, returning its old value
__device__ __forceinline__ int bucket_add(unsigned short *gbk, int bb) {
    const unsigned sh = 16u * (unsigned)(bb & 1);
    const unsigned old = atomicAdd(reinterpret_cast<unsigned *>(gbk) + (bb >> 1), 1u << sh);
    return (int)((old >> sh) & 0xffffu);
}

template <int G>
__device__ __forceinline__ BalLds bal_lds(unsigned char *smem, int lcap, int grp) {
    constexpr int PPB = LP_BLOCK / G;
    const int stride = lcap + 1;  // odd group stride: groups of a wave hit different LDS banks
    float *lkey = reinterpret_cast<float *>(smem);
    int *lj = reinterpret_cast<int *>(lkey + PPB * stride);
    unsigned char *lperm = reinterpret_cast<unsigned char *>(lj + PPB * stride);
    unsigned short *lbk = reinterpret_cast<unsigned short *>(lperm + PPB * ((stride + 3) & ~3));
    BalLds l;
    l.gkey = lkey + grp * stride;
    l.gj = lj + grp * stride;
    l.gperm = lperm + grp * ((stride + 3) & ~3);
    l.gbk = lbk + grp * SB_GSTRIDE;
    l.lout = reinterpret_cast<int *>(smem);
    l.lk = reinterpret_cast<int *>(lbk);
    return l;
}

// zero a group's bucket counters (every lane of the group)
template <int G>
__device__ __forceinline__ void bucket_clear(unsigned short *gbk, int lane) {
    for (int q = lane; q < SB_NB / 2; q += G) reinterpret_cast<unsigned *>(gbk)[q] = 0u;
}

// The k hits staged in a group's slots (FP32 key of d2, cell-order index) are
// ranked by (d2, original id) and the block's lists written out: nbr, count,
// the capacity bit, the overflow queue (k > lcap) and the wave's largest
// count into *max_out.  Called by every thread of the block.
template <int D, int G, bool PER>
__device__ __forceinline__ void bal_rank_write(const BalLds &l, int k, bool active, int s, double r2,
                                               const double xi[3], const Sorted &srt, const DevCfg &cfg, int *nbr,
                                               int ldn, int *count, DevScalars *sc, int lcap, int *ovf_queue,
                                               int *ovf_count, int *max_out) {
    constexpr int PPB = LP_BLOCK / G;
    const int lane = threadIdx.x % G;
    const int grp = threadIdx.x / G;
    const int max_nb = cfg.max_nb;
    float *gkey = l.gkey;
    int *gj = l.gj;
    unsigned char *gperm = l.gperm;
    unsigned short *gbk = l.gbk;
    int *lout = l.lout;
    int *lk = l.lk;
    __syncthreads();
    // rank: bucket B(d2) = floor(SB_NB d2/r2) in FP32 is non-decreasing in d2
    // (every operation is monotone), so entries of lower buckets rank lower;
    // inside a bucket the exact (d2, id) comparison decides.  For a uniform
    // particle density the outermost bucket holds 1.5x the mean share.
    const bool ranked = active && k <= lcap;
    const float inv_r2 = ranked ? (float)(1.0 / r2) : 0.0f;
    constexpr int EMAX = 128 / G;  // entries per lane (k <= lcap <= 128)
    int bk[EMAX];                  // bucket of each of this lane's entries
    int pos[EMAX];                 // its place inside the bucket
    if (ranked) {
#pragma unroll
        for (int q = 0; q < EMAX; ++q) {
            const int e = lane + q * G;
            if (e < k) {
                const float x = gkey[e] * inv_r2;
                int bb = (int)((float)SB_NB * x);
                bb = bb < 0 ? 0 : (bb > SB_NB - 1 ? SB_NB - 1 : bb);
                bk[q] = bb;
                pos[q] = bucket_add(gbk, bb);
            }
        }
    }
    __syncthreads();
    if (ranked) {
        // exclusive scan of the bucket counts, in place (lane q holds buckets q, q + G, ...)
        constexpr int BPL = SB_NB / G > 0 ? SB_NB / G : 1;  // buckets per lane
        int cnt[BPL];
        int mine = 0;
#pragma unroll
        for (int q = 0; q < BPL; ++q) {
            const int bb = lane * BPL + q;
            cnt[q] = bb < SB_NB ? gbk[bb] : 0;
            mine += cnt[q];
        }
        int incl = mine;
#pragma unroll
        for (int o = 1; o < G; o <<= 1) {
            const int v = __shfl_up(incl, o, G);
            if (lane >= o) incl += v;
        }
        int run = incl - mine;
#pragma unroll
        for (int q = 0; q < BPL; ++q) {
            const int bb = lane * BPL + q;
            if (bb < SB_NB) gbk[bb] = (unsigned short)run;  // start of bucket bb
            run += cnt[q];
        }
    }
    __syncthreads();
    if (ranked) {
#pragma unroll
        for (int q = 0; q < EMAX; ++q) {
            const int e = lane + q * G;
            if (e < k) gperm[gbk[bk[q]] + pos[q]] = (unsigned char)e;
        }
    }
    __syncthreads();
    {
        // largest count of the wave: one atomic per wave (all lanes active here)
        int kmax = k;
        for (int o = 32; o > 0; o >>= 1) kmax = max(kmax, __shfl_xor(kmax, o));
        // the atomic only when it can raise the maximum: same-address atomics
        // serialise in L2, and one per wave costs milliseconds at 2M particles
        if ((threadIdx.x & 63) == 0 && kmax > __hip_atomic_load(max_out, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT))
            atomicMax(max_out, kmax);
    }
    if (active) {
        if (lane == 0) {
            count[s] = k;
            if (k > max_nb) atomicOr(&sc->error_bits, 1u);
            // the list does not fit the LDS buffer: one wave redoes it (and
            // for k > max_nb writes max_nb valid entries, so readers stay in bounds)
            if (k > lcap) ovf_queue[atomicAdd(ovf_count, 1)] = s;
        }
    }
    int rank[EMAX], jq[EMAX];
    if (ranked) {
#pragma unroll
        for (int q = 0; q < EMAX; ++q) {
            const int e = lane + q * G;
            if (e < k) {
                const float ke = gkey[e];
                const int je = gj[e];
                const int bb = bk[q];
                const int lo = gbk[bb];
                const int hi = bb + 1 < SB_NB ? gbk[bb + 1] : k;
                int rk = lo;
                bool have_de = false;
                double de = 0.0;
                for (int f = lo; f < hi; ++f) {
                    const int pf = gperm[f];
                    const float kf = gkey[pf];
                    if (kf < ke) {
                        ++rk;
                    } else if (kf == ke && pf != e) {
                        // equal keys: the exact d2, recomputed as the dealing
                        // loop computed it, then the original id
                        const int jf = gj[pf];
                        double dx[3];
                        if (!have_de) {
                            disp_to<D, PER>(cfg, srt.x, je, xi, dx);
                            de = dist2_exact<D>(dx);
                            have_de = true;
                        }
                        disp_to<D, PER>(cfg, srt.x, jf, xi, dx);
                        const double df = dist2_exact<D>(dx);
                        if (df < de || (df == de && srt.id[jf] < srt.id[je])) ++rk;
                    }
                }
                rank[q] = rk;
                jq[q] = je;
            }
        }
    }
    __syncthreads();  // every group is done with its slots and counters
    if (lane == 0) lk[grp] = ranked ? k : 0;
    if (ranked) {
#pragma unroll
        for (int q = 0; q < EMAX; ++q)
            if (lane + q * G < k) lout[rank[q] * (PPB + 1) + grp] = jq[q];
    }
    __syncthreads();
    // write the block's lists: with column-major lists the PPB particles of
    // the block are consecutive in every column, so a column is one segment
    const int s0 = xcd_remap(blockIdx.x, gridDim.x) * PPB;
    int kb = 0;
    for (int q = 0; q < PPB; ++q) kb = max(kb, lk[q]);
    for (int idx = threadIdx.x; idx < kb * PPB; idx += LP_BLOCK) {
        const int c = idx / PPB, gq = idx % PPB;
        if (c < lk[gq]) {
            const int sq = s0 + gq;
            nbr[list_at(ldn, sq, c, max_nb)] = lout[c * (PPB + 1) + gq];
        }
    }
}

// The cells of particle s's search box at the level of radius ri, and in
// them every candidate j != s: the G lanes of a group deal the box's cells,
// then the candidates of G cells at a time, two per lane and round (t and
// t + G).  round(ua, d2a, ja, ub, d2b, jb) gets each lane's pair with the
// exact d2 (u: a real candidate); the lanes of a group call it together.
// The next round's positions are loaded (unconditionally, so that the loads
// stay in flight) before round() runs.
template <int D, int G, bool PER, typename F>
__device__ __forceinline__ void for_cell_candidates(const Sorted &srt, const uint32_t *tables, const DevGrid &g,
                                                    const DevCfg &cfg, int s, const double xi[3], double ri,
                                                    double r2, F &&round) {
    const int lane = threadIdx.x % G;
    // a cell is skipped only when even its box widened by a rounding slack
    // (and unbounded on the outer side of edge cells, which hold the
    // particles clamped into the grid) is farther than r from x_i
    const double r2_keep = r2 * (1.0 + 1e-12);
    const int L = level_for_radius(g, ri);
    const double cs = ldexp(g.s[g.L_lo], g.L_lo - L);  // = s[L] exactly
    const double slack = 1e-12 * g.s[0];
    const uint32_t *tab = tables + g.off[L];
    int clo[3] = {0, 0, 0}, cn[3] = {1, 1, 1};
    search_box<D>(g, cfg, L, xi, ri, clo, cn);
    const int ncells = cn[0] * cn[1] * (D == 3 ? cn[2] : 1);
    const float rcp0 = 1.0f / (float)cn[0], rcp1 = 1.0f / (float)cn[1];
    // cells per axis at level L (indexed by a per-particle level, so read
    // once here rather than in every batch)
    int nL[3];
#pragma unroll
    for (int a = 0; a < 3; ++a) nL[a] = g.nc[L][a];
    // Morton code of cell c of the box; false for a cell past the end or
    // provably outside the ball
    auto cell_code = [&](int c, uint32_t &code) -> bool {
        code = 0u;
        if (c >= ncells) return false;
        int cc[3], rem;
        const int q0 = div_small(c, cn[0], rcp0, rem);
        cc[0] = clo[0] + rem;
        if (D == 3) {
            const int q1 = div_small(q0, cn[1], rcp1, rem);
            cc[1] = clo[1] + rem;
            cc[2] = clo[2] + q1;
        } else {
            cc[1] = clo[1] + q0;
            cc[2] = 0;
        }
        double dd = 0.0;
#pragma unroll
        for (int a = 0; a < D; ++a) {
            if (PER && cfg.periodic[a]) continue;
            const int n_a = nL[a];
            const double lo_a = cc[a] <= 0 ? -INFINITY : g.lo[a] + cc[a] * cs - slack;
            const double hi_a = cc[a] >= n_a - 1 ? INFINITY : g.lo[a] + (cc[a] + 1) * cs + slack;
            // distance of x_i to [lo_a, hi_a] along a (at most one term is positive)
            const double t = fmax(lo_a - xi[a], 0.0) + fmax(xi[a] - hi_a, 0.0);
            dd += t * t;
        }
        if (dd > r2_keep) return false;
#pragma unroll
        for (int a = 0; a < D; ++a)
            if (PER && cfg.periodic[a]) {
                const int n_a = nL[a];
                cc[a] = cc[a] < 0 ? cc[a] + n_a : (cc[a] >= n_a ? cc[a] - n_a : cc[a]);
            }
        code = morton<D>(cc);
        return true;
    };
    // the cell-table entries of the next batch are loaded (unconditionally:
    // a skipped cell reads entry 0) while this batch's candidates are tested
    uint32_t nb_code;
    bool nb_ok = cell_code(lane, nb_code);
    uint32_t nb_lo = tab[nb_code], nb_hi = tab[nb_code + 1];
    for (int c0 = 0; c0 < ncells; c0 += G) {
        const int b = (int)nb_lo;
        const int len = nb_ok ? (int)(nb_hi - nb_lo) : 0;
        nb_ok = cell_code(c0 + G + lane, nb_code);
        nb_lo = tab[nb_code];
        nb_hi = tab[nb_code + 1];
        // inclusive prefix sum of the candidate counts over the group
        int incl = len;
#pragma unroll
        for (int o = 1; o < G; o <<= 1) {
            const int v = __shfl_up(incl, o, G);
            if (lane >= o) incl += v;
        }
        const int excl = incl - len;
        const int total = __shfl(incl, G - 1, G);
        // two candidates per lane and round (t and t + G).  The positions
        // of the next round are loaded (unconditionally, so that the loads
        // stay in flight) before this round's hits are compacted.
        auto fetch = [&](int t0, int &ja, int &jb, bool &oka, bool &okb, double *pa, double *pb) {
            const int ta = t0 + lane, tb = ta + G;
            // the cell of candidate t: the last lane q with excl_q <= t
            int qa = 0, qb = 0;
#pragma unroll
            for (int step = G / 2; step > 0; step >>= 1) {
                const int va = __shfl(excl, qa + step, G);
                const int vb = __shfl(excl, qb + step, G);
                if (va <= ta) qa += step;
                if (vb <= tb) qb += step;
            }
            ja = __shfl(b, qa, G) + (ta - __shfl(excl, qa, G));
            jb = __shfl(b, qb, G) + (tb - __shfl(excl, qb, G));
            oka = ta < total && ja != s;
            okb = tb < total && jb != s;
            // slots past the end read the particle itself (a valid index)
            const int ia = oka ? ja : s, ib = okb ? jb : s;
#pragma unroll
            for (int a = 0; a < D; ++a) {
                pa[a] = srt.x[a][ia];
                pb[a] = srt.x[a][ib];
            }
        };
        int ja, jb;
        bool oka, okb;
        double pa[3] = {0.0, 0.0, 0.0}, pb[3] = {0.0, 0.0, 0.0};
        fetch(0, ja, jb, oka, okb, pa, pb);
        for (int t0 = 0; t0 < total; t0 += 2 * G) {
            const int ca = ja, cb = jb;
            const bool ua = oka, ub = okb;
            double dxa[3], dxb[3];
            disp_of<D, PER>(cfg, pa, xi, dxa);
            disp_of<D, PER>(cfg, pb, xi, dxb);
            fetch(t0 + 2 * G, ja, jb, oka, okb, pa, pb);
            round(ua, dist2_exact<D>(dxa), ca, ub, dist2_exact<D>(dxb), cb);
        }
    }
}

template <int D, int G, bool PER>
__global__ __launch_bounds__(LP_BLOCK) void k_search_bal(Sorted srt, const int *n_total_dev, int n_real,
                                                         const uint32_t *tables, DevGrid g, DevCfg cfg, int *nbr,
                                                         int ldn, int *count, DevScalars *sc, int lcap,
                                                         int *ovf_queue, double rscale, const unsigned *gate,
                                                         int *max_out) {
    if (gate && *gate == 0u) return;
    constexpr int PPB = LP_BLOCK / G;
    extern __shared__ unsigned char smem[];
    const int lane = threadIdx.x % G;
    const int grp = threadIdx.x / G;
    const int gshift = (int)(threadIdx.x & 63) - lane;  // first wave lane of the group
    const unsigned long long gmask = G == 64 ? ~0ull : ((1ull << G) - 1ull);
    const unsigned long long below = (1ull << lane) - 1ull;
    const int s = xcd_remap(blockIdx.x, gridDim.x) * PPB + grp;
    const int n_total = *n_total_dev;
    const bool active = s < n_total && srt.id[s] < n_real;
    // after ranking, the key slots hold the ranked lists lout[rank * (PPB + 1) + grp]
    // and the bucket counters the list length of every group (0: written elsewhere)
    BalLds l = bal_lds<G>(smem, lcap, grp);
    float *gkey = l.gkey;
    int *gj = l.gj;
    int k = 0;  // hits so far (the same in every lane of the group)
    double r2 = 0.0;
    double xi[3] = {0.0, 0.0, 0.0};

    bucket_clear<G>(l.gbk, lane);
    if (active) {
        xi[0] = srt.x[0][s];
        xi[1] = srt.x[1][s];
        if (D == 3) xi[2] = srt.x[2][s];
        const double ri = srt.r[s] * rscale;
        r2 = ri * ri;
        for_cell_candidates<D, G, PER>(
            srt, tables, g, cfg, s, xi, ri, r2, [&](bool ua, double d2a, int ca, bool ub, double d2b, int cb) {
                const bool hita = ua && d2a < r2, hitb = ub && d2b < r2;
                const unsigned long long ma = (__ballot(hita) >> gshift) & gmask;
                const unsigned long long mb = (__ballot(hitb) >> gshift) & gmask;
                if (hita) {
                    const int slot = k + __popcll(ma & below);
                    if (slot < lcap) {
                        gkey[slot] = (float)d2a;
                        gj[slot] = ca;
                    }
                }
                k += __popcll(ma);
                if (hitb) {
                    const int slot = k + __popcll(mb & below);
                    if (slot < lcap) {
                        gkey[slot] = (float)d2b;
                        gj[slot] = cb;
                    }
                }
                k += __popcll(mb);
            });
    }
    bal_rank_write<D, G, PER>(l, k, active, s, r2, xi, srt, cfg, nbr, ldn, count, sc, lcap, ovf_queue,
                              &sc->n_overflow, max_out);
}


// Candidate lists of a rebuild: every particle within the enlarged radius
// rscale r_s, in the order found.  The filter ranks what it keeps, so the
// candidates need no ranking and are written straight to their slots
// (interleaved layout, ccount[s] of them); a particle with more than max_nb
// gets ccount -1 and raises cand_short, which has this step's filter search
// its cells exactly and the next step rebuild again.  *max_out: the longest
// candidate list.  Runs only where *gate is set.
template <int D, int G, bool PER>
__global__ __launch_bounds__(LP_BLOCK) void k_search_cand(Sorted srt, const int *n_total_dev, int n_real,
                                                          const uint32_t *tables, DevGrid g, DevCfg cfg, int *cand,
                                                          int *ccount, DevScalars *sc, double rscale,
                                                          const unsigned *gate, int *max_out) {
    if (gate && *gate == 0u) return;
    constexpr int PPB = LP_BLOCK / G;
    const int lane = threadIdx.x % G;
    const int gshift = (int)(threadIdx.x & 63) - lane;
    const unsigned long long gmask = G == 64 ? ~0ull : ((1ull << G) - 1ull);
    const unsigned long long below = (1ull << lane) - 1ull;
    const int s = xcd_remap(blockIdx.x, gridDim.x) * PPB + (int)threadIdx.x / G;
    const int n_total = *n_total_dev;
    const bool active = s < n_total && srt.id[s] < n_real;
    const int max_nb = cfg.max_nb;
    int k = 0;
    if (active) {
        const double xi[3] = {srt.x[0][s], srt.x[1][s], D == 3 ? srt.x[2][s] : 0.0};
        const double ri = srt.r[s] * rscale;
        const double r2 = ri * ri;
        for_cell_candidates<D, G, PER>(
            srt, tables, g, cfg, s, xi, ri, r2, [&](bool ua, double d2a, int ca, bool ub, double d2b, int cb) {
                const bool hita = ua && d2a < r2, hitb = ub && d2b < r2;
                const unsigned long long ma = (__ballot(hita) >> gshift) & gmask;
                const unsigned long long mb = (__ballot(hitb) >> gshift) & gmask;
                if (hita) {
                    const int slot = k + __popcll(ma & below);
                    if (slot < max_nb) cand[list_at(0, s, slot, max_nb)] = ca;
                }
                k += __popcll(ma);
                if (hitb) {
                    const int slot = k + __popcll(mb & below);
                    if (slot < max_nb) cand[list_at(0, s, slot, max_nb)] = cb;
                }
                k += __popcll(mb);
            });
    }
    // longest list of the wave: an atomic only where it raises the maximum
    // (same-address atomics serialise in L2)
    int kmax = k;
    for (int o = 32; o > 0; o >>= 1) kmax = max(kmax, __shfl_xor(kmax, o));
    if ((threadIdx.x & 63) == 0 && kmax > __hip_atomic_load(max_out, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT))
        atomicMax(max_out, kmax);
    if (active && lane == 0) {
        if (k > max_nb) {
            ccount[s] = -1;
            atomicOr(&sc->cand_short, 1u);
        } else {
            ccount[s] = k;
        }
    }
}

// ---------------------------------------------------------------------------
// Lists from reused candidates.  Candidate c of cell-order particle s is
// cand[c * ldc + s] (c < ccount[s]), a particle found within the enlarged
// radius by the last rebuild; the cell order has not changed since.  Each is
// tested against the current positions and radius with the search's own
// exact d2 < r^2, and the hits are ranked as the search ranks them, so the
// lists are the search's bit for bit whenever the candidates cover every
// neighbour (which the reuse check guarantees).  The G lanes of a group take
// two candidates each per round; the next round's indices and positions are
// loaded before this round's hits are compacted.
// ---------------------------------------------------------------------------
template <int D, int G, bool PER>
__global__ __launch_bounds__(LP_BLOCK) void k_filter_bal(Sorted srt, const int *n_total_dev, int n_real, DevCfg cfg,
                                                         const int *cand, int ldc, const int *ccount, int *nbr,
                                                         int ldn, int *count, DevScalars *sc, int lcap,
                                                         int *ovf_queue, unsigned long long *octc) {
    constexpr int PPB = LP_BLOCK / G;
    extern __shared__ unsigned char smem[];
    const int lane = threadIdx.x % G;
    const int grp = threadIdx.x / G;
    const int gshift = (int)(threadIdx.x & 63) - lane;
    const unsigned long long gmask = G == 64 ? ~0ull : ((1ull << G) - 1ull);
    const unsigned long long below = (1ull << lane) - 1ull;
    const int s = xcd_remap(blockIdx.x, gridDim.x) * PPB + grp;
    const int n_total = *n_total_dev;
    // a particle deleted since the candidates were built has no radius
    const bool active = s < n_total && srt.id[s] < n_real && srt.r[s] > 0.0;
    BalLds l = bal_lds<G>(smem, lcap, grp);
    int k = 0;
    double r2 = 0.0;
    double xi[3] = {0.0, 0.0, 0.0};
    bucket_clear<G>(l.gbk, lane);
    if (active) {
        xi[0] = srt.x[0][s];
        xi[1] = srt.x[1][s];
        if (D == 3) xi[2] = srt.x[2][s];
        const double ri = srt.r[s];
        r2 = ri * ri;
        int kc = ccount[s];
        const bool have_cand = kc >= 0;
        if (!have_cand) {
            // no candidates kept (more than max_nb of them at this step's
            // rebuild): the overflow kernel searches the fresh cells exactly
            if (lane == 0) ovf_queue[atomicAdd(&sc->n_fovf, 1)] = s;
            kc = 0;
        }
        // members per octant of the offset, 8 bits each (a lane takes at
        // most max_nb / G <= 32 of them), for the fit's stencil selection
        unsigned long long oc = 0ull;
        kc = kc < cfg.max_nb ? kc : cfg.max_nb;
        // indices of rounds t0 / t0 + 2G are in ja/jb and na/nb; slots past
        // the end read the particle itself (a valid index, never a hit)
        // entry t of the candidate list at cbase + t cstep (list_at's layouts)
        const int64_t cbase = ldc > 0 ? (int64_t)s : ldc < 0 ? (int64_t)s * (-ldc)
                                                            : (int64_t)(s >> 3) * (8 * cfg.max_nb) + (s & 7);
        const int64_t cstep = ldc > 0 ? (int64_t)ldc : ldc < 0 ? 1 : 8;
        auto index_at = [&](int t) -> int { return t < kc ? cand[cbase + t * cstep] : s; };
        int ja = index_at(lane), jb = index_at(lane + G);
        int na = index_at(lane + 2 * G), nb = index_at(lane + 3 * G);
        double pa[3] = {0.0, 0.0, 0.0}, pb[3] = {0.0, 0.0, 0.0};
#pragma unroll
        for (int a = 0; a < D; ++a) {
            pa[a] = srt.x[a][ja];
            pb[a] = srt.x[a][jb];
        }
        for (int t0 = 0; t0 < kc; t0 += 2 * G) {
            const int ca = ja, cb = jb;
            const bool ua = t0 + lane < kc, ub = t0 + lane + G < kc;
            double dxa[3], dxb[3];
            disp_of<D, PER>(cfg, pa, xi, dxa);
            disp_of<D, PER>(cfg, pb, xi, dxb);
            ja = na;
            jb = nb;
#pragma unroll
            for (int a = 0; a < D; ++a) {
                pa[a] = srt.x[a][ja];
                pb[a] = srt.x[a][jb];
            }
            na = index_at(t0 + 4 * G + lane);
            nb = index_at(t0 + 5 * G + lane);
            const double d2a = dist2_exact<D>(dxa), d2b = dist2_exact<D>(dxb);
            const bool hita = ua && d2a < r2, hitb = ub && d2b < r2;
            const unsigned long long ma = (__ballot(hita) >> gshift) & gmask;
            const unsigned long long mb = (__ballot(hitb) >> gshift) & gmask;
            if (hita) {
                const int slot = k + __popcll(ma & below);
                if (slot < lcap) {
                    l.gkey[slot] = (float)d2a;
                    l.gj[slot] = ca;
                }
                oc += 1ull << (8 * octant<D>(dxa));
            }
            k += __popcll(ma);
            if (hitb) {
                const int slot = k + __popcll(mb & below);
                if (slot < lcap) {
                    l.gkey[slot] = (float)d2b;
                    l.gj[slot] = cb;
                }
                oc += 1ull << (8 * octant<D>(dxb));
            }
            k += __popcll(mb);
        }
        // group sum (every lane of the group is here); no field can carry
        // while k <= 255.  Not counted: lists the overflow kernel searches.
#pragma unroll
        for (int o = 1; o < G; o <<= 1) oc += __shfl_xor(oc, o, G);
        if (lane == 0) octc[s] = (have_cand && k <= 255) ? oc : ~0ull;
    }
    bal_rank_write<D, G, PER>(l, k, active, s, r2, xi, srt, cfg, nbr, ldn, count, sc, lcap, ovf_queue,
                              &sc->n_fovf, &sc->max_count);
}

// Filtered lists longer than the LDS buffer of k_filter_bal: one wave per
// particle, a buffer of max_nb entries, exact (d2, id) ranking.
template <int D>
__global__ __launch_bounds__(64) void k_filter_overflow(Sorted srt, DevCfg cfg, const int *cand, int ldc,
                                                         const int *ccount, int *nbr, int ldn, int *count,
                                                         const uint32_t *tables, DevGrid g, DevScalars *sc,
                                                         const int *ovf_queue) {
    __shared__ double gd2[256];
    __shared__ int gj[256];
    __shared__ int lcnt;
    const int lane = threadIdx.x;
    const int nq = sc->n_fovf;
    for (int w = blockIdx.x; w < nq; w += gridDim.x) {
        const int s = ovf_queue[w];
        if (lane == 0) lcnt = 0;
        __syncthreads();
        const double xi[3] = {srt.x[0][s], srt.x[1][s], D == 3 ? srt.x[2][s] : 0.0};
        const double ri = srt.r[s];
        const double r2 = ri * ri;
        int kc = ccount[s];
        auto hit = [&](int j) {
            double dx[3];
            disp_to<D>(cfg, srt.x, j, xi, dx);
            const double d2 = dist2_exact<D>(dx);
            if (d2 < r2) {
                const int slot = atomicAdd(&lcnt, 1);
                if (slot < cfg.max_nb) {
                    gd2[slot] = d2;
                    gj[slot] = j;
                }
            }
        };
        if (kc >= 0) {
            kc = kc < cfg.max_nb ? kc : cfg.max_nb;
            for (int t = lane; t < kc; t += 64) hit(cand[list_at(ldc, s, t, cfg.max_nb)]);
        } else {
            // no candidates kept: the exact search over the cells, which this
            // step's rebuild has just laid out for the current positions
            const int L = level_for_radius(g, ri);
            const uint32_t *tab = tables + g.off[L];
            int clo[3] = {0, 0, 0}, cn[3] = {1, 1, 1};
            search_box<D>(g, cfg, L, xi, ri, clo, cn);
            const int ncells = cn[0] * cn[1] * (D == 3 ? cn[2] : 1);
            for (int c = lane; c < ncells; c += 64) {
                const uint32_t code = cell_code<D>(g, cfg, L, clo, cn, c);
                const uint32_t b = tab[code], e = tab[code + 1];
                for (uint32_t j = b; j < e; ++j)
                    if ((int)j != s) hit((int)j);
            }
        }
        __syncthreads();
        if (ccount[s] < 0 && lane == 0) {
            count[s] = lcnt;
            if (lcnt > cfg.max_nb) atomicOr(&sc->error_bits, 1u);
            atomicMax(&sc->max_count, lcnt);
        }
        const int k = lcnt < cfg.max_nb ? lcnt : cfg.max_nb;
        for (int e = lane; e < k; e += 64) {
            const double de = gd2[e];
            const int je = gj[e];
            int rank = 0;
            for (int f = 0; f < k; ++f) {
                const double df = gd2[f];
                if (df < de) ++rank;
                else if (df == de && f != e && srt.id[gj[f]] < srt.id[je]) ++rank;
            }
            nbr[list_at(ldn, s, rank, cfg.max_nb)] = je;
        }
        __syncthreads();
    }
}

static size_t search_smem(int G, int lcap) {
    int ppb = LP_BLOCK / G;
    return (size_t)ppb * lcap * (8 + 4) + (size_t)ppb * 4;
}

// LDS of k_search_bal: per group, lcap + 1 (FP32 key, index) slots, a byte
// permutation and SB_NB bucket counters (the ranked lists reuse the key slots)
static size_t search_bal_smem(int G, int lcap) {
    size_t ppb = (size_t)(LP_BLOCK / G);
    size_t stride = (size_t)lcap + 1;
    return ppb * stride * 8 + ppb * ((stride + 3) & ~(size_t)3) + ppb * SB_GSTRIDE * 2;
}

template <int D, int G>
static void launch_search_t(const Sorted &s, const int *n_total_dev, int n_total_cap, int n_real, const uint32_t *tables,
                            const DevGrid &g, const DevCfg &cfg, int *nbr, int ldn, int *count, DevScalars *sc,
                            int lcap, int *ovf_queue, bool balanced, hipStream_t st, double rscale,
                            const unsigned *gate, int *max_out) {
    constexpr int PPB = LP_BLOCK / G;
    unsigned blocks = (unsigned)((n_total_cap + PPB - 1) / PPB);
    if (blocks < 1) blocks = 1;
    size_t shm = balanced ? search_bal_smem(G, lcap) : search_smem(G, lcap);
    const bool per = cfg.periodic[0] || cfg.periodic[1] || (D == 3 && cfg.periodic[2]);
    if (balanced && per)
        hipLaunchKernelGGL((k_search_bal<D, G, true>), dim3(blocks), dim3(LP_BLOCK), shm, st, s, n_total_dev, n_real,
                           tables, g, cfg, nbr, ldn, count, sc, lcap, ovf_queue, rscale, gate, max_out);
    else if (balanced)
        hipLaunchKernelGGL((k_search_bal<D, G, false>), dim3(blocks), dim3(LP_BLOCK), shm, st, s, n_total_dev, n_real,
                           tables, g, cfg, nbr, ldn, count, sc, lcap, ovf_queue, rscale, gate, max_out);
    else
        hipLaunchKernelGGL((k_search<D, G>), dim3(blocks), dim3(LP_BLOCK), shm, st, s, n_total_dev, n_real, tables, g,
                           cfg, nbr, ldn, count, sc, lcap, ovf_queue, rscale, gate, max_out);
    unsigned ob = (unsigned)(n_total_cap < 1024 ? (n_total_cap > 0 ? n_total_cap : 1) : 1024);
    hipLaunchKernelGGL(k_search_overflow<D>, dim3(ob), dim3(64), 0, st, s, tables, g, cfg, nbr, ldn, sc, ovf_queue,
                       rscale, gate);
}

template <int D, int G>
static void launch_search_cand_t(const Sorted &s, const int *n_total_dev, int n_total_cap, int n_real,
                                 const uint32_t *tables, const DevGrid &g, const DevCfg &cfg, int *cand, int *ccount,
                                 DevScalars *sc, double rscale, const unsigned *gate, int *max_out, hipStream_t st) {
    constexpr int PPB = LP_BLOCK / G;
    unsigned blocks = (unsigned)((n_total_cap + PPB - 1) / PPB);
    if (blocks < 1) blocks = 1;
    const bool per = cfg.periodic[0] || cfg.periodic[1] || (D == 3 && cfg.periodic[2]);
    if (per)
        hipLaunchKernelGGL((k_search_cand<D, G, true>), dim3(blocks), dim3(LP_BLOCK), 0, st, s, n_total_dev, n_real,
                           tables, g, cfg, cand, ccount, sc, rscale, gate, max_out);
    else
        hipLaunchKernelGGL((k_search_cand<D, G, false>), dim3(blocks), dim3(LP_BLOCK), 0, st, s, n_total_dev, n_real,
                           tables, g, cfg, cand, ccount, sc, rscale, gate, max_out);
}

void launch_search_cand(const Sorted &s, const int *n_total_dev, int n_total_cap, int n_real, const uint32_t *tables,
                        const DevGrid &g, const DevCfg &cfg, int *cand, int *ccount, DevScalars *sc, int group,
                        double rscale, const unsigned *gate, int *max_out, hipStream_t st) {
    int G = group;
    if (G != 4 && G != 8 && G != 16 && G != 32) G = 16;
#define LC(DD, GG) launch_search_cand_t<DD, GG>(s, n_total_dev, n_total_cap, n_real, tables, g, cfg, cand, ccount, sc, rscale, gate, max_out, st)
    if (cfg.D == 3) {
        if (G == 4) LC(3, 4); else if (G == 8) LC(3, 8); else if (G == 16) LC(3, 16); else LC(3, 32);
    } else {
        if (G == 4) LC(2, 4); else if (G == 8) LC(2, 8); else if (G == 16) LC(2, 16); else LC(2, 32);
    }
#undef LC
    (void)hipGetLastError();
}

template <int D, int G>
static void launch_filter_t(const Sorted &s, const int *n_total_dev, int n_total_cap, int n_real, const DevCfg &cfg,
                            const int *cand, int ldc, const int *ccount, int *nbr, int ldn, int *count,
                            const uint32_t *tables, const DevGrid &g, DevScalars *sc, int lcap, int *ovf_queue,
                            unsigned long long *octc, hipStream_t st) {
    constexpr int PPB = LP_BLOCK / G;
    unsigned blocks = (unsigned)((n_total_cap + PPB - 1) / PPB);
    if (blocks < 1) blocks = 1;
    size_t shm = search_bal_smem(G, lcap);
    const bool per = cfg.periodic[0] || cfg.periodic[1] || (D == 3 && cfg.periodic[2]);
    // the filter's overflow queue and counter (n_fovf) are its own: the
    // rebuild search of the same step uses n_overflow
    if (per)
        hipLaunchKernelGGL((k_filter_bal<D, G, true>), dim3(blocks), dim3(LP_BLOCK), shm, st, s, n_total_dev, n_real,
                           cfg, cand, ldc, ccount, nbr, ldn, count, sc, lcap, ovf_queue, octc);
    else
        hipLaunchKernelGGL((k_filter_bal<D, G, false>), dim3(blocks), dim3(LP_BLOCK), shm, st, s, n_total_dev, n_real,
                           cfg, cand, ldc, ccount, nbr, ldn, count, sc, lcap, ovf_queue, octc);
    unsigned ob = (unsigned)(n_total_cap < 1024 ? (n_total_cap > 0 ? n_total_cap : 1) : 1024);
    hipLaunchKernelGGL(k_filter_overflow<D>, dim3(ob), dim3(64), 0, st, s, cfg, cand, ldc, ccount, nbr, ldn, count,
                       tables, g, sc, ovf_queue);
}

void launch_filter(const Sorted &s, const int *n_total_dev, int n_total_cap, int n_real, const DevCfg &cfg,
                   const int *cand, int ldc, const int *ccount, int *nbr, int ldn, int *count,
                   const uint32_t *tables, const DevGrid &g, DevScalars *sc, int group, int lcap_req,
                   int *ovf_queue, unsigned long long *octc, hipStream_t st) {
    int G = group;
    if (G != 4 && G != 8 && G != 16 && G != 32) G = 16;
    int lcap = cfg.max_nb < 128 ? cfg.max_nb : 128;
    if (lcap_req > 0 && lcap_req < lcap) lcap = lcap_req;
    while (search_bal_smem(G, lcap) > 65536 && G < 64) G *= 2;
#define LF(DD, GG) launch_filter_t<DD, GG>(s, n_total_dev, n_total_cap, n_real, cfg, cand, ldc, ccount, nbr, ldn, count, tables, g, sc, lcap, ovf_queue, octc, st)
    if (cfg.D == 3) {
        if (G == 4) LF(3, 4); else if (G == 8) LF(3, 8); else if (G == 16) LF(3, 16); else if (G == 32) LF(3, 32); else LF(3, 64);
    } else {
        if (G == 4) LF(2, 4); else if (G == 8) LF(2, 8); else if (G == 16) LF(2, 16); else if (G == 32) LF(2, 32); else LF(2, 64);
    }
#undef LF
    (void)hipGetLastError();
}

void launch_search(const Sorted &s, const int *n_total_dev, int n_total_cap, int n_real, const uint32_t *tables,
                   const DevGrid &g, const DevCfg &cfg, int *nbr, int ldn, int *count, DevScalars *sc, int group,
                   int lcap_req, int *ovf_queue, bool balanced, hipStream_t st, double rscale, const unsigned *gate,
                   int *max_out) {
    if (!max_out) max_out = &sc->max_count;
    int G = group;
    if (G != 4 && G != 8 && G != 16 && G != 32) G = 16;
    // slots per particle in LDS (longer lists take the overflow kernel); a
    // smaller buffer lets more blocks share a CU
    int lcap = cfg.max_nb < 128 ? cfg.max_nb : 128;
    if (lcap_req > 0 && lcap_req < lcap) lcap = lcap_req;
    // LDS per block within 64 KiB
    while ((balanced ? search_bal_smem(G, lcap) : search_smem(G, lcap)) > 65536 && G < 64) G *= 2;
#define LS(DD, GG) launch_search_t<DD, GG>(s, n_total_dev, n_total_cap, n_real, tables, g, cfg, nbr, ldn, count, sc, lcap, ovf_queue, balanced, st, rscale, gate, max_out)
    if (cfg.D == 3) {
        if (G == 4) LS(3, 4); else if (G == 8) LS(3, 8); else if (G == 16) LS(3, 16); else if (G == 32) LS(3, 32); else LS(3, 64);
    } else {
        if (G == 4) LS(2, 4); else if (G == 8) LS(2, 8); else if (G == 16) LS(2, 16); else if (G == 32) LS(2, 32); else LS(2, 64);
    }
#undef LS
    (void)hipGetLastError();
}

// ===========================================================================
// Tiled search: a block takes one tile -- the coarsest cell holding at most
// TLEAF particles -- finds the cells that cover the union of its particles'
// search balls, and streams the particles of those cells through LDS.
// ===========================================================================
#define TILE 256    // threads per block of the tiled search
#define TLEAF 64    // particles per tile (leaf cell capacity)
#define MAXRUN 1024

// Adaptive tiles: the coarsest cell holding at most TLEAF particles (the
// octree leaf of the paper's step 2), split into runs of TLEAF when the finest
// level is still fuller.  Every particle that starts a tile is flagged.
__global__ void k_tile_flags(Sorted srt, const int *n_total_dev, int cap, const uint32_t *key,
                             const uint32_t *tables, DevGrid g, int D, uint32_t *flag) {
    int s = blockIdx.x * blockDim.x + threadIdx.x;
    int n = *n_total_dev;
    if (s >= cap) return;
    if (s >= n) { flag[s] = 0u; return; }
    uint32_t k = key[srt.id[s]];
    uint32_t cs = 0, ce = 0;
    for (int L = g.L_lo; L <= g.L_hi; ++L) {
        uint32_t code = k >> (D * (g.L_hi - L));
        const uint32_t *tab = tables + g.off[L];
        cs = tab[code];
        ce = tab[code + 1];
        if (ce - cs <= TLEAF) break;
    }
    flag[s] = ((uint32_t)s - cs) % TLEAF == 0 ? 1u : 0u;
    (void)ce;
}

__global__ void k_tile_list(Sorted srt, const int *n_total_dev, const uint32_t *key, const uint32_t *tables,
                            DevGrid g, int D, const uint32_t *off, int *tile_lo, int *tile_hi) {
    int s = blockIdx.x * blockDim.x + threadIdx.x;
    int n = *n_total_dev;
    if (s >= n) return;
    if (off[s + 1] == off[s]) return;  // not a tile head
    uint32_t k = key[srt.id[s]];
    uint32_t ce = 0;
    for (int L = g.L_lo; L <= g.L_hi; ++L) {
        uint32_t code = k >> (D * (g.L_hi - L));
        const uint32_t *tab = tables + g.off[L];
        uint32_t cs = tab[code];
        ce = tab[code + 1];
        if (ce - cs <= TLEAF) break;
    }
    uint32_t e = (uint32_t)s + TLEAF < ce ? (uint32_t)s + TLEAF : ce;
    tile_lo[off[s]] = s;
    tile_hi[off[s]] = (int)e;
}

// ===========================================================================
// Wave per particle: the tile's halo is staged in LDS; each wave then takes
// one particle at a time and its 64 lanes test 64 staged candidates at once.
// Hits are compacted with a ballot into the wave's LDS buffer, ranked there by
// (d2, original id), and the row is written in order.  A halo larger than one
// LDS chunk (rare) is streamed in chunks with the hits appended to a scratch
// row in global memory instead.  Output layout: row-major nbr[s * max_nb + c].
// ===========================================================================
#define CHUNK2 768
#define SORTCAP 256
#define TW (TILE / 64)

template <int D>
__device__ __forceinline__ void rank_and_write(const double *sd2, const int *sid, const int *sjj, int kk, int lane,
                                               int *row) {
    for (int e = lane; e < kk; e += 64) {
        double de = sd2[e];
        int ie = sid[e];
        int rank = 0;
        for (int f = 0; f < kk; ++f) {
            double df = sd2[f];
            int idf = sid[f];
            rank += (df < de) || (df == de && idf < ie);
        }
        row[rank] = sjj[e];
    }
}

template <int D>
__global__ __launch_bounds__(TILE) void k_search_tile2(Sorted srt, const int *n_total_dev, int n_real,
                                                      const uint32_t *tables, DevGrid g, DevCfg cfg, double *hit_d2,
                                                      int *hit_j, int *nbr, int *count, DevScalars *sc,
                                                      const int *tile_lo, const int *tile_hi, const int *ntiles_dev) {
    __shared__ double cx[CHUNK2], cy[CHUNK2], cz[CHUNK2];
    __shared__ int cj[CHUNK2], cid[CHUNK2];
    __shared__ uint32_t run_b[MAXRUN];
    __shared__ uint32_t run_p[MAXRUN + 1];
    __shared__ double red[7][TW];
    __shared__ int geo[2];
    __shared__ uint32_t wsum[TW];
    __shared__ int pcnt[TILE];
    __shared__ double tpx[TILE], tpy[TILE], tpz[TILE], tpr[TILE];
    __shared__ int tpid[TILE];
    __shared__ double sd2[TW][SORTCAP];
    __shared__ int sid[TW][SORTCAP];
    __shared__ int sjj[TW][SORTCAP];

    const int t = threadIdx.x;
    const int lane = t & 63, wave = t >> 6;
    const unsigned long long lt_mask = lane == 0 ? 0ull : (~0ull >> (64 - lane));
    const int ntiles = *ntiles_dev;
    const int nb = gridDim.x;
    const int b = xcd_remap(blockIdx.x, nb);
    const int per = (ntiles + nb - 1) / nb;
    const int t_begin = b * per;
    const int t_end = t_begin + per < ntiles ? t_begin + per : ntiles;
    const int max_nb = cfg.max_nb;
    for (int tile = t_begin; tile < t_end; ++tile) {
        const int s0 = tile_lo[tile];
        const int np = tile_hi[tile] - s0;
        const int s = s0 + t;
        bool valid = false;
        double ri = 0.0, xi[3] = {0.0, 0.0, 0.0};
        if (t < np) {
            int id = srt.id[s];
            valid = id < n_real;
            xi[0] = srt.x[0][s];
            xi[1] = srt.x[1][s];
            if (D == 3) xi[2] = srt.x[2][s];
            ri = srt.r[s];
            tpx[t] = xi[0]; tpy[t] = xi[1]; tpz[t] = xi[2]; tpr[t] = ri; tpid[t] = id;
        }
        pcnt[t] = 0;
        double v[7];
        for (int a = 0; a < 3; ++a) {
            v[a] = valid ? xi[a] - ri : INFINITY;
            v[3 + a] = valid ? -(xi[a] + ri) : INFINITY;
        }
        v[6] = valid ? -ri : INFINITY;
        for (int q = 0; q < 7; ++q) {
            double w = v[q];
            for (int o = 32; o > 0; o >>= 1) w = fmin(w, __shfl_xor(w, o));
            v[q] = w;
        }
        if (lane == 0)
            for (int q = 0; q < 7; ++q) red[q][wave] = v[q];
        __syncthreads();
        double blo[3], bhi[3], rmax;
        {
            double m[7];
            for (int q = 0; q < 7; ++q) {
                m[q] = red[q][0];
                for (int w = 1; w < TW; ++w) m[q] = fmin(m[q], red[q][w]);
            }
            for (int a = 0; a < 3; ++a) { blo[a] = m[a]; bhi[a] = -m[3 + a]; }
            rmax = -m[6];
        }
        __syncthreads();
        if (!(rmax > 0.0)) continue;  // uniform
        int L = level_for_radius(g, rmax);
        int clo[3] = {0, 0, 0}, cn[3] = {1, 1, 1};
        for (;;) {
            long long tot = 1;
            for (int a = 0; a < D; ++a) {
                int n = g.nc[L][a];
                int lo = floor_clamped((blo[a] - g.lo[a]) * g.inv_s[L] - 1e-9);
                int hi = floor_clamped((bhi[a] - g.lo[a]) * g.inv_s[L] + 1e-9);
                if (cfg.periodic[a]) {
                    if (hi - lo + 1 >= n || hi < lo) { lo = 0; hi = n - 1; }
                } else {
                    lo = lo < 0 ? 0 : (lo > n - 1 ? n - 1 : lo);
                    hi = hi > n - 1 ? n - 1 : (hi < 0 ? 0 : hi);
                }
                clo[a] = lo;
                cn[a] = hi - lo + 1;
                tot *= cn[a];
            }
            if (tot <= MAXRUN || L == g.L_lo) break;
            --L;
        }
        const int ncells = cn[0] * cn[1] * (D == 3 ? cn[2] : 1);
        const uint32_t *tab = tables + g.off[L];
        bool in_lds = true;  // hits kept in LDS (single batch and single chunk)
        for (int cb = 0; cb < ncells; cb += MAXRUN) {
            const int nrun = ncells - cb < MAXRUN ? ncells - cb : MAXRUN;
            uint32_t mylen[MAXRUN / TILE];
            uint32_t mysum = 0;
            for (int k = 0; k < MAXRUN / TILE; ++k) {
                int q = t * (MAXRUN / TILE) + k;
                uint32_t len = 0;
                if (q < nrun) {
                    int qq = cb + q;
                    int cc[3];
                    cc[0] = clo[0] + qq % cn[0];
                    cc[1] = clo[1] + (qq / cn[0]) % cn[1];
                    cc[2] = D == 3 ? clo[2] + qq / (cn[0] * cn[1]) : 0;
                    for (int a = 0; a < D; ++a)
                        if (cfg.periodic[a]) {
                            int n = g.nc[L][a];
                            cc[a] = ((cc[a] % n) + n) % n;
                        }
                    uint32_t code = morton<D>(cc);
                    uint32_t bb = tab[code], ee = tab[code + 1];
                    run_b[q] = bb;
                    len = ee - bb;
                }
                mylen[k] = len;
                mysum += len;
            }
            {
                uint32_t inc = mysum;
                for (int o = 1; o < 64; o <<= 1) {
                    uint32_t y = __shfl_up(inc, o);
                    if (lane >= o) inc += y;
                }
                if (lane == 63) wsum[wave] = inc;
                __syncthreads();
                uint32_t off = 0, tot = 0;
                for (int w = 0; w < TW; ++w) {
                    if (w < wave) off += wsum[w];
                    tot += wsum[w];
                }
                uint32_t run = off + inc - mysum;
                for (int k = 0; k < MAXRUN / TILE; ++k) {
                    int q = t * (MAXRUN / TILE) + k;
                    run_p[q] = run;
                    run += mylen[k];
                }
                if (t == 0) { run_p[MAXRUN] = tot; geo[0] = (int)tot; }
            }
            __syncthreads();
            const int H = geo[0];
            if (ncells > MAXRUN || H > CHUNK2) in_lds = false;  // uniform
            for (int base = 0; base < H; base += CHUNK2) {
                const int m = H - base < CHUNK2 ? H - base : CHUNK2;
                for (int k = t; k < m; k += TILE) {
                    uint32_t gk = (uint32_t)(base + k);
                    int lo = 0, hi = nrun - 1;
                    while (lo < hi) {
                        int mid = (lo + hi + 1) >> 1;
                        if (run_p[mid] <= gk) lo = mid; else hi = mid - 1;
                    }
                    int j = (int)(run_b[lo] + (gk - run_p[lo]));
                    cx[k] = srt.x[0][j];
                    cy[k] = srt.x[1][j];
                    cz[k] = D == 3 ? srt.x[2][j] : 0.0;
                    cj[k] = j;
                    cid[k] = srt.id[j];
                }
                __syncthreads();
                for (int p = wave; p < np; p += TW) {
                    if (tpid[p] >= n_real) continue;  // wave-uniform
                    const int sp = s0 + p;
                    const double px = tpx[p], py = tpy[p], pz = tpz[p], pr = tpr[p];
                    const double pr2 = pr * pr;
                    int c = pcnt[p];
                    double *rd2 = hit_d2 + (int64_t)sp * max_nb;
                    int *rj = hit_j + (int64_t)sp * max_nb;
                    for (int k0 = 0; k0 < m; k0 += 64) {
                        int k = k0 + lane;
                        bool hit = false;
                        double d2 = 0.0;
                        int j = -1;
                        if (k < m) {
                            j = cj[k];
                            double dx[3];
                            dx[0] = min_image(cfg, 0, cx[k] - px);
                            dx[1] = min_image(cfg, 1, cy[k] - py);
                            dx[2] = D == 3 ? min_image(cfg, 2, cz[k] - pz) : 0.0;
                            d2 = dist2_exact<D>(dx);
                            hit = d2 < pr2 && j != sp;
                        }
                        unsigned long long mask = __ballot(hit);
                        if (hit) {
                            int pos = c + __popcll(mask & lt_mask);
                            if (in_lds) {
                                if (pos < max_nb) {
                                    sd2[wave][pos] = d2;
                                    sjj[wave][pos] = j;
                                    sid[wave][pos] = cid[k];
                                }
                            } else if (pos < max_nb) {
                                rd2[pos] = d2;
                                rj[pos] = j;
                            }
                        }
                        c += __popcll(mask);
                    }
                    if (in_lds) {
                        // the halo fitted one chunk: the row is complete, rank it now
                        __builtin_amdgcn_wave_barrier();
                        __builtin_amdgcn_fence(__ATOMIC_RELEASE, "workgroup");
                        const int kk = c < max_nb ? c : max_nb;
                        rank_and_write<D>(sd2[wave], sid[wave], sjj[wave], kk, lane, nbr + (int64_t)sp * max_nb);
                        if (lane == 0) {
                            count[sp] = c;
                            if (c > max_nb) atomicOr(&sc->error_bits, 1u);
                            atomicMax(&sc->max_count, c);
                        }
                        __builtin_amdgcn_wave_barrier();
                        __builtin_amdgcn_fence(__ATOMIC_RELEASE, "workgroup");
                    } else if (lane == 0) {
                        pcnt[p] = c;
                    }
                }
                __syncthreads();
            }
        }
        if (!in_lds) {
            // rows were appended in global memory: rank each one by (d2, id)
            for (int p = wave; p < np; p += TW) {
                if (tpid[p] >= n_real) continue;  // wave-uniform
                const int sp = s0 + p;
                const int k = pcnt[p];
                const int kk = k < max_nb ? k : max_nb;
                for (int e = lane; e < kk; e += 64) {
                    int j = hit_j[(int64_t)sp * max_nb + e];
                    sd2[wave][e] = hit_d2[(int64_t)sp * max_nb + e];
                    sjj[wave][e] = j;
                    sid[wave][e] = srt.id[j];
                }
                __builtin_amdgcn_wave_barrier();
                __builtin_amdgcn_fence(__ATOMIC_RELEASE, "workgroup");
                rank_and_write<D>(sd2[wave], sid[wave], sjj[wave], kk, lane, nbr + (int64_t)sp * max_nb);
                if (lane == 0) {
                    count[sp] = k;
                    if (k > max_nb) atomicOr(&sc->error_bits, 1u);
                    atomicMax(&sc->max_count, k);
                }
                __builtin_amdgcn_wave_barrier();
                __builtin_amdgcn_fence(__ATOMIC_RELEASE, "workgroup");
            }
        }
        __syncthreads();
    }
}

void launch_search_tiles(const Sorted &s, const int *n_total_dev, int n_total_cap, int n_real,
                         const uint32_t *tables, const DevGrid &g, const DevCfg &cfg, double *hit_d2, int *hit_j,
                         int *nbr, int ldn, int *count, DevScalars *sc, const uint32_t *key, uint32_t *flags,
                         uint32_t *scan_tmp, int *tile_lo, int *tile_hi, int *ntiles_dev, hipStream_t st) {
    unsigned nbp = (unsigned)((n_total_cap + LP_BLOCK - 1) / LP_BLOCK);
    if (nbp < 1) nbp = 1;
    hipLaunchKernelGGL(k_tile_flags, dim3(nbp), dim3(LP_BLOCK), 0, st, s, n_total_dev, n_total_cap, key, tables, g,
                       cfg.D, flags);
    launch_scan_u32(flags, (uint64_t)n_total_cap, scan_tmp, ntiles_dev, st);
    hipLaunchKernelGGL(k_tile_list, dim3(nbp), dim3(LP_BLOCK), 0, st, s, n_total_dev, key, tables, g, cfg.D, flags,
                       tile_lo, tile_hi);
    int nb = 2048;
    if (cfg.D == 3)
        hipLaunchKernelGGL(k_search_tile2<3>, dim3(nb), dim3(TILE), 0, st, s, n_total_dev, n_real, tables, g, cfg,
                           hit_d2, hit_j, nbr, count, sc, tile_lo, tile_hi, ntiles_dev);
    else
        hipLaunchKernelGGL(k_search_tile2<2>, dim3(nb), dim3(TILE), 0, st, s, n_total_dev, n_real, tables, g, cfg,
                           hit_d2, hit_j, nbr, count, sc, tile_lo, tile_hi, ntiles_dev);
    (void)ldn;
    (void)hipGetLastError();
}
