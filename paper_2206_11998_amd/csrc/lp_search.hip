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

template <int D, int G>
__global__ __launch_bounds__(LP_BLOCK) void k_search(Sorted srt, const int *n_total_dev, int n_real,
                                                     const uint32_t *tables, DevGrid g, DevCfg cfg, int *nbr, int ldn,
                                                     int *count, DevScalars *sc) {
    constexpr int PPB = LP_BLOCK / G;
    extern __shared__ unsigned char smem[];
    const int max_nb = cfg.max_nb;
    double *ld2 = reinterpret_cast<double *>(smem);
    int *lid = reinterpret_cast<int *>(ld2 + PPB * max_nb);
    int *lj = lid + PPB * max_nb;
    int *lcnt = lj + PPB * max_nb;

    const int lane = threadIdx.x % G;
    const int grp = threadIdx.x / G;
    const int s = blockIdx.x * PPB + grp;
    const int n_total = *n_total_dev;
    const bool active = s < n_total && srt.id[s] < n_real;
    double *gd2 = ld2 + grp * max_nb;
    int *gid = lid + grp * max_nb;
    int *gj = lj + grp * max_nb;
    if (lane == 0) lcnt[grp] = 0;
    __syncthreads();

    if (active) {
        double xi[3] = {srt.x[0][s], srt.x[1][s], D == 3 ? srt.x[2][s] : 0.0};
        double ri = srt.r[s];
        double r2 = ri * ri;
        int L = level_for_radius(g, ri);
        const uint32_t *tab = tables + g.off[L];
        int clo[3] = {0, 0, 0}, cn[3] = {1, 1, 1};
        for (int a = 0; a < D; ++a) {
            int n = g.nc[L][a];
            double tl = (xi[a] - ri - g.lo[a]) * g.inv_s[L];
            double th = (xi[a] + ri - g.lo[a]) * g.inv_s[L];
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
        const int ncells = cn[0] * cn[1] * (D == 3 ? cn[2] : 1);
        for (int c = lane; c < ncells; c += G) {
            int cc[3];
            cc[0] = clo[0] + c % cn[0];
            cc[1] = clo[1] + (c / cn[0]) % cn[1];
            cc[2] = D == 3 ? clo[2] + c / (cn[0] * cn[1]) : 0;
            for (int a = 0; a < D; ++a)
                if (cfg.periodic[a]) {
                    int n = g.nc[L][a];
                    cc[a] = ((cc[a] % n) + n) % n;
                }
            uint32_t code = morton<D>(cc);
            uint32_t b = tab[code], e = tab[code + 1];
            for (uint32_t j = b; j < e; ++j) {
                if ((int)j == s) continue;
                double dx[3];
                dx[0] = min_image(cfg, 0, srt.x[0][j] - xi[0]);
                dx[1] = min_image(cfg, 1, srt.x[1][j] - xi[1]);
                dx[2] = D == 3 ? min_image(cfg, 2, srt.x[2][j] - xi[2]) : 0.0;
                double d2 = dist2_exact<D>(dx);
                if (d2 < r2) {
                    int slot = atomicAdd(&lcnt[grp], 1);
                    if (slot < max_nb) {
                        gd2[slot] = d2;
                        gid[slot] = srt.id[j];
                        gj[slot] = (int)j;
                    }
                }
            }
        }
    }
    __syncthreads();
    if (active) {
        int k = lcnt[grp];
        int kk = k < max_nb ? k : max_nb;
        if (lane == 0) {
            count[s] = k;
            atomicMax(&sc->max_count, k);
            if (k > max_nb) atomicOr(&sc->error_bits, 1u);
        }
        for (int e = lane; e < kk; e += G) {
            double de = gd2[e];
            int ie = gid[e];
            int rank = 0;
            for (int f = 0; f < kk; ++f) {
                double df = gd2[f];
                int idf = gid[f];
                rank += (df < de) || (df == de && idf < ie);
            }
            nbr[(int64_t)rank * ldn + s] = gj[e];
        }
    }
}

static size_t search_smem(int G, int max_nb) {
    int ppb = LP_BLOCK / G;
    return (size_t)ppb * max_nb * (8 + 4 + 4) + (size_t)ppb * 4;
}

template <int D, int G>
static void launch_search_t(const Sorted &s, const int *n_total_dev, int n_total_cap, int n_real, const uint32_t *tables,
                            const DevGrid &g, const DevCfg &cfg, int *nbr, int ldn, int *count, DevScalars *sc,
                            hipStream_t st) {
    constexpr int PPB = LP_BLOCK / G;
    unsigned blocks = (unsigned)((n_total_cap + PPB - 1) / PPB);
    if (blocks < 1) blocks = 1;
    size_t shm = search_smem(G, cfg.max_nb);
    hipLaunchKernelGGL((k_search<D, G>), dim3(blocks), dim3(LP_BLOCK), shm, st, s, n_total_dev, n_real, tables, g, cfg,
                       nbr, ldn, count, sc);
}

void launch_search(const Sorted &s, const int *n_total_dev, int n_total_cap, int n_real, const uint32_t *tables,
                   const DevGrid &g, const DevCfg &cfg, int *nbr, int ldn, int *count, DevScalars *sc, int group,
                   hipStream_t st) {
    // LDS per block must stay within 64 KiB for the default launch
    int G = group;
    if (G != 4 && G != 8 && G != 16 && G != 32) G = 16;
    while (search_smem(G, cfg.max_nb) > 65536 && G < 64) G *= 2;
#define LS(DD, GG) launch_search_t<DD, GG>(s, n_total_dev, n_total_cap, n_real, tables, g, cfg, nbr, ldn, count, sc, st)
    if (cfg.D == 3) {
        if (G == 4) LS(3, 4); else if (G == 8) LS(3, 8); else if (G == 16) LS(3, 16); else if (G == 32) LS(3, 32); else LS(3, 64);
    } else {
        if (G == 4) LS(2, 4); else if (G == 8) LS(2, 8); else if (G == 16) LS(2, 16); else if (G == 32) LS(2, 32); else LS(2, 64);
    }
#undef LS
    (void)hipGetLastError();
}
