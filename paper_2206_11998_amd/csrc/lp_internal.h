// lp_internal.h -- device data structures, launchers and shared device helpers
// of liblp (gfx950).  Included by every translation unit of the library.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "../../include/lp.h"

#define LP_MAX_LEVEL 16
#define LP_BLOCK 256
#define LP_QTILE 1024  // largest tile of the stencil-size work queue

// ---------------------------------------------------------------------------
// Configuration as seen by the kernels (passed by value).
// ---------------------------------------------------------------------------
struct DevCfg {
    int D, nu, nf;              // dimension, second-order unknowns, fields (V, u.., P)
    int lw_cap, uw_cap, max_nb;
    int vacuum, est_mode, precision, refine;
    float refine_cond;              // > 0: refine only fits whose condition estimate exceeds it
    double gamma, kappa, cfl, est_eps, cond_max, uw_cond_max, cond_fb;
    double lo[3], hi[3], L[3], half[3];
    int periodic[3], wall_lo[3], wall_hi[3];
    float mlp_band, mlp_feat_max;   // network estimator: trusted away from 1/2 by mlp_band, inputs within +-max
    float limiter_cap;              // > 0: phi = min(phi, limiter_cap); 0: the limiter as printed
};

// Hierarchy of uniform cell grids over the cube [lo, lo + S)^D.  Level L has
// cells of size S / 2^L; per level, a table start[code] (Morton code of the
// cell, plus one sentinel) gives the first sorted particle of every cell.
struct DevGrid {
    double lo[3];
    int L_lo, L_hi;
    int nc[LP_MAX_LEVEL][3];        // cells per axis
    double inv_s[LP_MAX_LEVEL];     // 2^L / S (exact power-of-two scaling of 1/S)
    double s[LP_MAX_LEVEL];         // S / 2^L
    unsigned long long off[LP_MAX_LEVEL];  // offset of the level's table (entries)
};

// Device-resident scalars of one context.
struct DevScalars {
    unsigned long long min_hc;      // bits of min h/c (positive doubles order as integers)
    unsigned long long rmax;        // bits of max r
    unsigned long long rmin;        // bits of min r
    double dt, t, t_end, dt_in;
    int n_total;                    // real + ghost particles
    int n_ghost;
    int max_count;
    int prev_max_count;             // max_count of the step before (kept by k_reset_scalars)
    int n_fallback;
    int n_refine;                   // fits queued for the refinement launch
    unsigned int error_bits;        // 1: capacity, 2: numeric
    unsigned int done;              // lp_run: t reached t_end
    unsigned int clipped;           // this step's dt was shortened to end on t_end
    unsigned int halt;              // a graph-replayed step found more ghosts than its workspace holds
    int n_tiles;                    // search tiles of the last search
    int n_overflow;                 // lists longer than the search kernel's LDS buffer
    unsigned long long xlo[3], xhi[3];  // bounding box of real particles (order-preserving keys)
    unsigned long long n_limited;
    unsigned long long steps;       // steps executed (skipped steps do not count)
    unsigned long long n_mlp;       // particles whose phi came from the network in the last step
    unsigned long long n_mlp_plain; // particles for which the network was not trusted
    unsigned int head[2][8];        // chunk counters of the persistent fit / update launches, per XCD range
    // neighbour-list reuse (candidate lists built within an enlarged radius)
    unsigned int rebuild;           // this step rebuilds the cells and the candidate lists
    unsigned int have_cand;         // a candidate set exists (the last rebuild's)
    int max_cand;                   // longest candidate list of the last rebuild
    int n_fovf;                     // candidate filters whose hits overflow the LDS buffer
    unsigned long long reuse_a;     // max_i (r_i + d_i - R_i) as an order-preserving key (d_i: displacement)
    unsigned long long reuse_d;     // bits of max_i d_i
    unsigned long long n_builds;    // rebuilds so far
    unsigned int cand_short;        // the last rebuild found more candidates than max_nb for some particle
    // particles of zero mass are absent (lp_run_open: deleted, or slots not yet filled)
    int n_in;                       // real slots + ghosts: the extent the cell sort reads
    int n_dead;                     // real slots of zero mass (k_prep); n_total = n_in - n_dead
    int n_hw;                       // lp_run_open: slots in use (live or deleted); layers are appended here
    unsigned int pop_changed;       // a particle was added since the last list build
    int n_sorted;                   // entries of the cell order of the last build (present then)
    unsigned long long open_k;      // lp_run_open: steps run
    unsigned int insert_now;        // lp_run_open: this step ends with an inflow layer
};

// Open boundaries inside the steps of lp_run_open (device copy of the setup).
struct OpenDev {
    uint32_t lo_mask, hi_mask;      // outflow faces
    int in_every;                   // a layer after every in_every-th step (0: no inflow)
    int axis, side, o0, o1;         // inflow face and the other axes
    int64_t count, cnt0;            // lattice points of a layer, along the first other axis
    int64_t cap;                    // slots of the caller's arrays
    double spacing, xa;             // lattice spacing, position of the layer's plane
    double un, V, P, mass;          // fixed state of the entering particles (res_width <= 0)
    double res_width, res_face, res_p, res_rho, gamma;  // res_width > 0: reservoir state at each layer
    double *res_part;               // res_blocks x 2 partial sums, then 4 outputs (P_in, rho_in, u_in, count)
    int res_blocks;
};

// Particle state in the caller's order (real particles only).
struct Soa {
    double *x[3], *V, *u[3], *P;
    const double *m;
    float *phi;
    uint8_t *flags;
    int n;
};

// Mirror ghosts (ids n .. n + n_ghost - 1).
struct Ghosts {
    double *x[3], *V, *u[3], *P, *h, *r;
};

// Sorted (cell-ordered) copies of real + ghost particles.
struct Sorted {
    double *x[3], *V, *u[3], *P, *h, *r;
    double *rec;                    // packed gather records (LP_REC doubles each), or NULL
    float *recf;                    // packed FP32-field gather records (LP_RECF_BYTES each), or NULL
    int *id;                        // original id (ghosts: n + g)
};

// Packed gather record of a cell-order particle, LP_REC doubles (64 B, one
// half cache line): x_0 .. x_{D-1}, V, u_0 .. u_{D-1}, P (2D: two unused).
// The fits gather a neighbour's position and fields from it in four 16-byte
// loads of one line, instead of eight loads from eight arrays.
#define LP_REC 8

// The FP32 kernels' record, 48 B (three 16-byte loads): the positions in FP64
// (the stencil's octants and the displacements need them exactly), then V,
// u_0 .. u_{D-1}, P rounded to FP32 (round to nearest, as those kernels round
// the FP64 values themselves).  3D: x0 x1 | x2 V u0 | u1 u2 P -;
// 2D: x0 x1 | V u0 u1 P.
#define LP_RECF_BYTES 48

// octant of an offset: bit a set where dx[a] >= 0
template <int D>
__device__ __forceinline__ int octant(const double dx[3]) {
    int o = 0;
#pragma unroll
    for (int a = 0; a < D; ++a) o |= (dx[a] >= 0.0 ? 1 : 0) << a;
    return o;
}

template <int D>
__device__ __forceinline__ void rec_pos(const double *rec, int j, double p[3]) {
    const double2 *r = reinterpret_cast<const double2 *>(rec + (int64_t)LP_REC * j);
    const double2 a = r[0];
    p[0] = a.x;
    p[1] = a.y;
    p[2] = D == 3 ? r[1].x : 0.0;
}

// V, u_0 .. u_{D-1}, P of cell-order particle j (from its record when there is one)
template <int D>
__device__ __forceinline__ void gather_fields(const Sorted &srt, int j, double f[D + 2]) {
    if (srt.rec) {
        const double2 *r = reinterpret_cast<const double2 *>(srt.rec + (int64_t)LP_REC * j);
        if constexpr (D == 3) {
            const double2 b = r[1], c = r[2], d = r[3];
            f[0] = b.y; f[1] = c.x; f[2] = c.y; f[3] = d.x; f[4] = d.y;
        } else {
            const double2 b = r[1], c = r[2];
            f[0] = b.x; f[1] = b.y; f[2] = c.x; f[3] = c.y;
        }
    } else {
        f[0] = srt.V[j];
#pragma unroll
        for (int q = 0; q < D; ++q) f[1 + q] = srt.u[q][j];
        f[D + 1] = srt.P[j];
    }
}

// Generic gather of up to 12 double arrays into cell order.
struct ScatterArgs {
    int nd;
    const double *src[12];          // caller order (ids < n_real)
    const double *gsrc[12];         // ghosts (ids >= n_real); may be NULL
    double *dst[12];
    double *rec;                    // packed gather records (LP_REC doubles), or NULL
    float *recf;                    // FP32-field gather records (LP_RECF_BYTES each), or NULL
    int rec_src[LP_REC];            // value index of each record entry (-1: zero)
    int dim;                        // layout of the FP32-field record
    const double *m;                // masses (caller order) or NULL: a real particle of zero mass that
                                    // still holds a cell slot gets infinite coordinates (no one's neighbour)
};

// ---------------------------------------------------------------------------
// Host launchers (defined in the .hip files).
// ---------------------------------------------------------------------------
void launch_reset_scalars(DevScalars *sc, double dt_in, int n_real, int clear_halt, hipStream_t st);
void launch_gate(DevScalars *sc, int n_real, int64_t cap_ghost, int stop_on_error, hipStream_t st);
void launch_rminmax(const double *r, const double *const x[3], int D, int n, DevScalars *sc, hipStream_t st);
void launch_advance_time(DevScalars *sc, hipStream_t st);
// xb, Rb (may be NULL): positions and enlarged radii of the last list build;
// given, the pass also reduces the list-reuse check's maxima
void launch_prep(const Soa &p, const DevCfg &cfg, DevScalars *sc, double *h, double *r, double *part,
                 hipStream_t st, double *const xb[3] = nullptr, const double *Rb = nullptr);
size_t prep_partial_words(int64_t n);
void launch_dt(const DevCfg &cfg, DevScalars *sc, int clip_t_end, hipStream_t st);
void launch_ghost_count(const Soa &p, const DevCfg &cfg, DevScalars *sc, uint32_t *gcnt, hipStream_t st);
void launch_ghost_write(const Soa &p, const DevCfg &cfg, DevScalars *sc, const uint32_t *goff,
                        const double *h, const double *r, Ghosts g, int64_t cap_ghost, hipStream_t st);
// gate (may be NULL): the kernels do nothing unless *gate != 0 (read on the device)
void launch_fill_u32(uint32_t *p, uint64_t n, uint32_t v, hipStream_t st, const unsigned *gate = nullptr);
// m (may be NULL): a real particle of zero mass is absent: key LP_KEY_ABSENT, no
// slot, and k_scatter leaves it out, so the cell order holds the present
// particles (n_total of them) and nothing after them
#define LP_KEY_ABSENT 0xFFFFFFFFu
void launch_keys(const double *const x[3], const double *const gx[3], int n_real, const int *n_total_dev,
                 int n_total_cap, const DevGrid &g, int D, uint32_t *key, uint32_t *slot, uint32_t *cnt,
                 hipStream_t st, const unsigned *gate = nullptr, const double *m = nullptr);
// exclusive scan of n u32 values in place; out[n] receives the total; tmp needs scan_tmp_words(n)
uint64_t scan_tmp_words(uint64_t n);
void launch_scan_u32(uint32_t *data, uint64_t n, uint32_t *tmp, int *total_dev, hipStream_t st,
                     const unsigned *gate = nullptr);
void launch_scatter(const ScatterArgs &a, int n_real, const int *n_total_dev, int n_total_cap,
                    const uint32_t *key, const uint32_t *slot, const uint32_t *start, int *sorted_id,
                    hipStream_t st);
void launch_coarsen(uint32_t *tables, const DevGrid &g, int D, const int *n_total_dev, hipStream_t st,
                    const unsigned *gate = nullptr);
// rscale: the search radius is r * rscale (1: the neighbour lists themselves);
// max_out receives the longest list (NULL: sc->max_count)
void launch_search(const Sorted &s, const int *n_total_dev, int n_total_cap, int n_real, const uint32_t *tables,
                   const DevGrid &g, const DevCfg &cfg, int *nbr, int ldn, int *count, DevScalars *sc,
                   int group, int lcap, int *ovf_queue, bool balanced, hipStream_t st, double rscale = 1.0,
                   const unsigned *gate = nullptr, int *max_out = nullptr);
// candidate lists of a rebuild (interleaved layout, unranked): every particle
// within r_s * rscale; runs where *gate is set; max_out: the longest
void launch_search_cand(const Sorted &s, const int *n_total_dev, int n_total_cap, int n_real, const uint32_t *tables,
                        const DevGrid &g, const DevCfg &cfg, int *cand, int *ccount, DevScalars *sc, int group,
                        double rscale, const unsigned *gate, int *max_out, hipStream_t st);
// neighbour lists from reused candidate lists cand[c * ldc + s], c < ccount[s]:
// the exact test d2 < r_s^2 on the current positions, (d2, id) order
// (ccount[s] < 0: no candidates were kept; the cells -- laid out by this
// step's rebuild -- are searched exactly instead).  octc[s]: for lists longer
// than lw_cap, the members per octant of the offset (8 bits each; ~0 where
// not counted)
void launch_filter(const Sorted &s, const int *n_total_dev, int n_total_cap, int n_real, const DevCfg &cfg,
                   const int *cand, int ldc, const int *ccount, int *nbr, int ldn, int *count,
                   const uint32_t *tables, const DevGrid &g, DevScalars *sc, int group, int lcap, int *ovf_queue,
                   unsigned long long *octc, hipStream_t st);
// reuse decision: displacement since the last rebuild and radius growth
// against the enlarged radius; force != 0 rebuilds; a rebuild step copies
// the positions and r * rscale of every particle
void launch_reuse(const Soa &p, const DevCfg &cfg, const double *r, double *const xb[3], double *Rb, int n,
                  double rscale, int force, DevScalars *sc, hipStream_t st);
// end of a step of lp_run_open: outflow deletion (mass set to zero), the step
// count, and on every in_every-th step an inflow layer appended at n_hw
void launch_open_end(const Soa &p, const DevCfg &cfg, const OpenDev &o, DevScalars *sc, hipStream_t st);
// keep[i] = 1 for a particle of positive mass in slots 0 .. n - 1
void launch_alive_keep(const Soa &p, uint32_t *keep, hipStream_t st);
void launch_search_tiles(const Sorted &s, const int *n_total_dev, int n_total_cap, int n_real,
                         const uint32_t *tables, const DevGrid &g, const DevCfg &cfg, double *hit_d2, int *hit_j,
                         int *nbr, int ldn, int *count, DevScalars *sc, const uint32_t *key, uint32_t *flags,
                         uint32_t *scan_tmp, int *tile_lo, int *tile_hi, int *ntiles_dev, hipStream_t st);
void launch_lists_out(const int *sorted_id, const int *nbr, int ldn, const int *count, int n, int max_nb,
                      int *count_out, int *idx_out, hipStream_t st);
int der_count(int D);
int refine_keep_count(int D);
// Staging of the update when the network estimator decides phi: per
// cell-order particle s its 16 inputs feat[16 s + q], the LW and upwind rates
// rates[f * ld + s] and rates[(NF + f) * ld + s], the quotient estimator's
// phi and the particle flags (LP_MLP_FORCE0: phi = 0 whatever the network says).
#define LP_MLP_FORCE0 128
struct MlpStage {
    float *feat;
    double *rates;
    double *phi_plain;
    uint8_t *mflag;
    int64_t ld;
    const float *theta;  // non-NULL: the network's parameters, applied by the fused kernel itself
};

// Everything the fit and update kernels read or write.
struct SolveArgs {
    Sorted srt;
    Soa p;
    const int *nbr;
    int ldn;
    const int *count;
    const int *n_total_dev;
    int n_real;
    DevCfg cfg;
    DevScalars *sc;
    int *queue;                     // FP64 fallback queue (written by the fit)
    double *der;                    // derivatives between fit and update, der[q * ld + work slot]
    int64_t ld;
    uint8_t *lwst;                  // per particle: 0 fast path, 1 queued for the fallback
    const int *wq;                  // work queue of launch_bin_tiles (NULL: direct indexing)
    int *rq;                        // refinement queue: (cell-order particle, work slot) pairs
    float *rkeep;                   // per refinement-queue slot: factor, 1/diag and FP32 coefficients
    MlpStage ms;                    // feat != NULL: stage for the network estimator instead of updating
    const unsigned long long *octc; // per particle with a list longer than lw_cap: its octant counts
                                    // (8 bits each, written by the list filter; ~0: not counted), or NULL
};
// whether launch_solve with these arguments and mode runs the network itself
// (the fused kernel, with ms.theta set): then only the particles staged by the
// refinement and the FP64 fallback are left for launch_mlp_apply
bool solve_fuses_network(const SolveArgs &a, int mode);
// mode: 0 direct, 1 work queue, 2 persistent launch over the work queue
void launch_solve(const SolveArgs &a, int n_total_cap, int block, int mode, void (*between)(void *),
                  void *between_arg, hipStream_t st);
void launch_bin_tiles(const int *count, const int *sid, const int *n_total_dev, int n_total_cap, int n_real,
                      int max_nb, int tile, int *wq, hipStream_t st);
void launch_solve_fallback(const Sorted &s, const Soa &p, const int *nbr, int ldn, const int *count,
                           int n_real, const DevCfg &cfg, DevScalars *sc, const int *queue, int queue_cap,
                           const MlpStage &ms, hipStream_t st);
// network estimator (lp_mlp.hip)
void launch_mlp_forward(const float *th, int64_t n, const float *feat, float *z, float *y, hipStream_t st);
void launch_mlp_apply(const float *th, const Sorted &s, const Soa &p, const DevCfg &cfg, DevScalars *sc,
                      int64_t n_total_cap, int n_real, const MlpStage &ms, int queued, const int *fq, const int *rq,
                      hipStream_t st);
int mlp_grad_blocks(int64_t nb);
void launch_mlp_grad(const float *th, int64_t b0, int64_t nb, const float *feat, const float *target, float *part,
                     float *loss_part, float *grad, float *loss, hipStream_t st);
void launch_mlp_adam(float *th, float *m, float *v, const float *grad, float lr, float b1, float b2, float eps,
                     int t, const float *loss, float *loss_acc, hipStream_t st);
void launch_features_out(const Sorted &s, const MlpStage &ms, const int *n_total_dev, int64_t n_total_cap,
                         int n_real, float *feat, float *phi, uint8_t *valid, hipStream_t st);
void launch_fill_f32(float *p, int n, float v, hipStream_t st);
void launch_gfd(const Sorted &s, const double *const *fs, int nf, const int *nbr, int ldn, const int *count,
                int n, const DevCfg &cfg, DevScalars *sc, int *queue, double *deriv, uint8_t *status,
                hipStream_t st);
void launch_gfd_fallback(const Sorted &s, const double *const *fs, int nf, const int *nbr, int ldn,
                         const int *count, int n, const DevCfg &cfg, DevScalars *sc, const int *queue,
                         int queue_cap, double *deriv, uint8_t *status, hipStream_t st);
void launch_gfd3(const Sorted &s, const double *const *fs, int nf, const int *nbr, int ldn, const int *count,
                 int n, const DevCfg &cfg, DevScalars *sc, int *queue, double *deriv, uint8_t *status,
                 hipStream_t st);
void launch_out_keep(const Soa &p, const DevCfg &cfg, uint32_t lo_mask, uint32_t hi_mask, uint32_t *keep,
                     hipStream_t st);
// bytes of the outflow staging area for n particles in D dimensions
size_t out_stage_bytes(int D, int64_t n);
void launch_out_compact(const Soa &p, int D, const uint32_t *pos, uint32_t kept, double *tmp, hipStream_t st);
void launch_inflow_layer(const Soa &p, const DevCfg &cfg, int64_t n0, int64_t count, int64_t cnt0, int axis, int o0,
                         int o1, double spacing, double xa, double un, double V, double P, double mass,
                         hipStream_t st);
void launch_reservoir(const double *xa, const double *P, int n, int side, double face, double width, double p_res,
                      double rho_res, double gamma, double *part, int nblocks, double *out, hipStream_t st);
void launch_conservation(const Soa &p, const DevCfg &cfg, double *partials, int nblocks, double *out,
                         hipStream_t st);

// ---------------------------------------------------------------------------
// Shared device helpers.
// ---------------------------------------------------------------------------
__device__ __forceinline__ unsigned long long dbl_bits(double v) { return (unsigned long long)__double_as_longlong(v); }
// Order-preserving map of any double to an unsigned key (for atomic min/max).
__device__ __forceinline__ unsigned long long dbl_key(double v) {
    unsigned long long b = dbl_bits(v);
    return (b >> 63) ? ~b : (b | 0x8000000000000000ull);
}
__device__ __forceinline__ double bits_dbl(unsigned long long b) { return __longlong_as_double((long long)b); }

// Minimum-image displacement x_j - x_i along axis a.  Evaluated exactly as
// written (IEEE binary64 add/sub only); the fold is a select, not a branch, so
// loads around it are not serialised by divergent control flow.
__device__ __forceinline__ double min_image(const DevCfg &c, int a, double d) {
    const bool p = c.periodic[a] != 0;
    const double down = d - c.L[a], up = d + c.L[a];
    double r = d;
    r = (p && d < -c.half[a]) ? up : r;
    r = (p && d > c.half[a]) ? down : r;
    return r;
}

// Displacements x_j - x_i (minimum image) of particle j of a SoA position set;
// the coordinates of j are all loaded before any arithmetic, so the loads are
// in flight together.
// PER = false: the caller knows that no axis is periodic (plain differences).
template <int D, bool PER = true>
__device__ __forceinline__ void disp_of(const DevCfg &c, const double xj[3], const double xi[3], double dx[3]) {
    dx[0] = PER ? min_image(c, 0, xj[0] - xi[0]) : xj[0] - xi[0];
    dx[1] = PER ? min_image(c, 1, xj[1] - xi[1]) : xj[1] - xi[1];
    dx[2] = D == 3 ? (PER ? min_image(c, 2, xj[2] - xi[2]) : xj[2] - xi[2]) : 0.0;
}

template <int D, bool PER = true>
__device__ __forceinline__ void disp_to(const DevCfg &c, const double *const x[3], int j, const double xi[3],
                                        double dx[3]) {
    const double xj[3] = {x[0][j], x[1][j], D == 3 ? x[2][j] : 0.0};
    disp_of<D, PER>(c, xj, xi, dx);
}

// Squared distance ((dx*dx) + (dy*dy)) + (dz*dz) with every product and sum
// rounded separately (no fused multiply-add), so that neighbour sets agree bit
// for bit with any other IEEE binary64 evaluation of the same expression.
template <int D>
__device__ __forceinline__ double dist2_exact(const double dx[3]) {
#pragma clang fp contract(off)
    double s = dx[0] * dx[0] + dx[1] * dx[1];
    if (D == 3) s = s + dx[2] * dx[2];
    return s;
}

__device__ __forceinline__ uint32_t spread3(uint32_t v) {
    v &= 0x3ffu;
    v = (v | (v << 16)) & 0x030000FFu;
    v = (v | (v << 8)) & 0x0300F00Fu;
    v = (v | (v << 4)) & 0x030C30C3u;
    v = (v | (v << 2)) & 0x09249249u;
    return v;
}
__device__ __forceinline__ uint32_t spread2(uint32_t v) {
    v &= 0xffffu;
    v = (v | (v << 8)) & 0x00FF00FFu;
    v = (v | (v << 4)) & 0x0F0F0F0Fu;
    v = (v | (v << 2)) & 0x33333333u;
    v = (v | (v << 1)) & 0x55555555u;
    return v;
}
template <int D>
__device__ __forceinline__ uint32_t morton(const int c[3]) {
    if (D == 3) return spread3((uint32_t)c[0]) | (spread3((uint32_t)c[1]) << 1) | (spread3((uint32_t)c[2]) << 2);
    return spread2((uint32_t)c[0]) | (spread2((uint32_t)c[1]) << 1);
}

// Cell coordinate along one axis at level L (clamped into the grid).
// Clamping happens in floating point before the conversion, so positions far
// outside the grid (or NaN) map to an edge cell instead of overflowing.
__device__ __forceinline__ int cell_coord(const DevGrid &g, int L, int a, double x) {
    double t = (x - g.lo[a]) * g.inv_s[L];
    int n = g.nc[L][a];
    if (!(t >= 0.0)) return 0;
    if (t >= (double)n) return n - 1;
    int c = (int)t;
    return c < n ? c : n - 1;
}

// floor(t) as an int, with t first clamped to +-2^24 (NaN -> 0)
__device__ __forceinline__ int floor_clamped(double t) {
    if (!(t == t)) return 0;
    t = fmin(fmax(t, -16777216.0), 16777216.0);
    return (int)floor(t);
}

// Blocks are dispatched round-robin over the 8 XCDs of the chip, each with its
// own L2.  Mapping block b to work item w so that every XCD gets one
// contiguous range of work keeps spatially adjacent (cell-ordered) particles
// -- and the neighbour data they share -- in the same L2.  Bijective for any
// block count.
__device__ __forceinline__ int xcd_remap(int b, int nb) {
    const int X = 8;
    int q = nb / X, rem = nb % X;
    int xcd = b % X, idx = b / X;
    return xcd * q + (xcd < rem ? xcd : rem) + idx;
}

// Persistent work loop: the ceil(n / blockDim) chunks of blockDim items are
// split into 8 contiguous ranges, one per XCD.  A block claims chunks of its
// own XCD's range (blocks are dispatched round-robin over the XCDs) through
// head[range], then helps with the other ranges; body(t) runs for every item
// index t of every chunk claimed (t may exceed n - 1 in the last chunk).
// Every block leaves once all 8 counters have passed their range's end.
template <typename F>
__device__ __forceinline__ void persistent_chunks(unsigned *head, int n, F &&body) {
    __shared__ int sh_chunk;
    const int B = blockDim.x;
    const int nch = (n + B - 1) / B;
    const int home = blockIdx.x % 8;
    for (int x = 0; x < 8; ++x) {
        const int rg = (home + x) % 8;
        const int lo = (int)((int64_t)nch * rg / 8), hi = (int)((int64_t)nch * (rg + 1) / 8);
        for (;;) {
            if (threadIdx.x == 0) {
                unsigned c = atomicAdd(&head[rg], 1u);
                sh_chunk = c < (unsigned)(hi - lo) ? lo + (int)c : -1;
            }
            __syncthreads();
            const int c = sh_chunk;
            __syncthreads();
            if (c < 0) break;
            body(c * B + (int)threadIdx.x);
        }
    }
}

// Neighbour-list element c of cell-order particle s.  ldn > 0: column-major
// lists nbr[c * ldn + s]; ldn < 0: row-major lists nbr[s * (-ldn) + c].
__device__ __forceinline__ int nb_at(const int *nbr, int ldn, int s, int c) {
    return ldn > 0 ? nbr[(int64_t)c * ldn + s] : nbr[(int64_t)s * (-ldn) + c];
}

// Level used by a particle of radius r: the coarsest level whose cells are not
// larger than r (so the search box spans 2-5 cells per axis), clamped.
__device__ __forceinline__ int level_for_radius(const DevGrid &g, double r) {
    // s[L] = S 2^-L: halving is exact, so only the first level's side is read
    int L = g.L_lo;
    double sL = g.s[g.L_lo];
    while (L < g.L_hi && sL > r) {
        ++L;
        sL *= 0.5;
    }
    return L;
}
