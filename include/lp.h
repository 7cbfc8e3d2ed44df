/*
 * lp.h -- C ABI of liblp, an MI355X (gfx950) implementation of the hot path of
 * the Lagrangian particle (LP) method of Yuan, Zepeda Aguilar, Naitlho &
 * Samulyak, "Massively-Parallel Lagrangian Particle Code and Applications"
 * (arXiv 2206.11998):
 *
 *   neighbour search (Sec. 2.2, step 3), generalized-finite-difference
 *   least-squares fits (Sec. 2.1, GFD system and its QR solution), and the
 *   unsplit Lax-Wendroff update blended with first-order upwind where the
 *   state estimator selects a particle (Sec. 2.1, blend, estimator, limiter),
 *   followed by the particle mover (Sec. 2.1, mover; Sec. 2.2, step 6).
 *
 * Conventions (all entry points):
 *  - Every call returns an lp_status; nothing throws across the ABI.  On error
 *    lp_last_error() holds a message.
 *  - Particle arrays are structure-of-arrays DEVICE pointers owned by the
 *    caller; the library never frees them.  Indices in and out are the
 *    caller's particle indices (0..n-1); internal orderings never leak out.
 *  - `stream` is a hipStream_t passed as void* (NULL = the default stream).
 *    Work is enqueued asynchronously on it; only calls documented as
 *    synchronising wait for it.
 *  - A context is not thread-safe; use one per stream.  The library allocates
 *    its own device workspace, grown on demand and kept until lp_destroy().
 *  - Errors found by kernels (list capacity overflow, non-positive V or P after
 *    an update) accumulate in the context and are reported by lp_check().
 */
#ifndef LP_H
#define LP_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef int32_t lp_status;
enum {
    LP_OK = 0,
    LP_E_ARG = 1,       /* invalid argument or configuration */
    LP_E_CAPACITY = 2,  /* a neighbour list exceeded max_nb (counts are still true counts) */
    LP_E_NUMERIC = 3,   /* non-positive specific volume or pressure after an update */
    LP_E_DEVICE = 4,    /* HIP runtime error */
    LP_E_NOMEM = 5,     /* device allocation failed */
    LP_E_STATE = 6      /* call sequence error */
};

enum { LP_FP64 = 0, LP_MIXED = 1 };                         /* lp_config.precision */
/* lp_config.estimator: PLAIN is the quotient estimator of Sec. 2.1; INJECTED
 * reads phi from lp_particles.phi; MLP lets the estimator network of
 * lp_mlp_* decide phi where it is trusted (see mlp_band), with PLAIN as the
 * fallback and phi = 0 kept for degenerate and vacuum particles. */
enum { LP_EST_PLAIN = 0, LP_EST_INJECTED = 1, LP_EST_MLP = 2 };

/* Per-particle flag bits written to lp_particles.flags. */
enum {
    LP_FLAG_LIMITED = 1,      /* phi < 1: blended towards upwind */
    LP_FLAG_DEGENERATE = 2,   /* second-order fit rank deficient: linear fit, phi = 0 */
    LP_FLAG_VACUUM = 4,       /* a half-ball was completed by vacuum ghosts, phi = 0 */
    LP_FLAG_SUBSTITUTED = 8,  /* a half-ball fit was unusable: LW gradient used for that side */
    LP_FLAG_FALLBACK = 16,    /* the FP64 pivoted-QR path solved this particle */
    LP_FLAG_NUMERIC = 32      /* non-positive V or P after the update */
};

typedef struct lp_config {
    int32_t dim;            /* 2 or 3 */
    int32_t precision;      /* LP_FP64 or LP_MIXED (FP32 gathers/fits, FP64 state) */
    int32_t estimator;      /* LP_EST_* */
    int32_t max_nb;         /* neighbour-list capacity per particle, 1..256 */
    int32_t lw_cap;         /* Lax-Wendroff stencil size; 0 -> 54 (3D) / 32 (2D); at most 64 */
    int32_t uw_cap;         /* upwind half-ball size; 0 -> 8; at most 16 */
    int32_t refine;         /* LP_MIXED: 1 = one FP64-residual refinement of the fit (see refine_cond) */
    int32_t vacuum;         /* free boundary: incomplete half-balls get vacuum ghosts */
    double gamma;           /* ideal-gas exponent */
    double cfl;             /* dt = cfl * min_i h_i / c_i */
    double kappa;           /* search radius r_i = kappa * h_i, h_i = (m_i V_i)^(1/dim) */
    double est_eps;         /* estimator activity threshold (relative, per h) */
    double cond_max;        /* pivoted |R11|/|Rnn| above this: 2nd-order fit deficient */
    double uw_cond_max;     /* pivoted |R11|/|Rnn| above this: half-ball fit unusable */
    double cond_fallback;   /* fast fit: normal-matrix condition estimate above this -> FP64 QR */
    double box_lo[3];       /* domain box; periodic extents must be S / 2^j of the */
    double box_hi[3];       /*   largest extent S */
    uint32_t periodic_mask; /* bit a: axis a periodic (minimum image, wrap on move) */
    uint32_t wall_lo_mask;  /* bit a: mirror wall at box_lo[a] */
    uint32_t wall_hi_mask;  /* bit a: mirror wall at box_hi[a] */
    float mlp_band;         /* LP_EST_MLP: the network's phi is used when |phi - 1/2| >= mlp_band ... */
    float mlp_feat_max;     /* ... and every input lies within +-mlp_feat_max; otherwise the quotient
                               estimator's phi (defaults 0.05 and 8) */
    float refine_cond;      /* LP_MIXED with refine: 0 (default) refines every fast-path fit; > 0 refines
                               only the fits whose normal-matrix condition estimate ||R||_F^2 ||R^-1||_F^2
                               exceeds it (an upper bound on cond(A)^2, so the FP32 solve's relative
                               error is at most about refine_cond * 2^-24 elsewhere); the rest keep
                               the FP32 solution.  A refined fit is computed by a separate launch over
                               the queued particles, with the same arithmetic as refine_cond = 0 */
    float limiter_cap;      /* Sec. 2.1 limiter: > 0 caps phi at this value (default 1: a particle the
                               estimator does not select advances with the pure Lax-Wendroff rate);
                               0 leaves the limiter as printed, whose largest value is 1.25 at r = 1 */
    int32_t reserved[5];
} lp_config;

typedef struct lp_particles {
    int64_t n;              /* number of particles */
    double *x[3];           /* positions (x[2] unused in 2D); advanced in place */
    double *V;              /* specific volume 1/rho; advanced in place */
    double *u[3];           /* velocity; advanced in place */
    double *P;              /* pressure; advanced in place */
    const double *m;        /* mass (constant) */
    float *phi;             /* out: limiter value per particle (in with LP_EST_INJECTED); may be NULL */
    uint8_t *flags;         /* out: LP_FLAG_* bits; may be NULL */
} lp_particles;

typedef struct lp_info {
    double t;               /* time accumulated by lp_step / lp_run */
    double dt;              /* last time step */
    int64_t n_ghost;        /* mirror ghosts of the last step */
    int32_t max_count;      /* largest neighbour count of the last search */
    int32_t n_fallback;     /* particles solved by the FP64 pivoted-QR path in the last step */
    int64_t n_limited;      /* particles with phi < 1 in the last step */
    uint32_t error_bits;    /* bit 0: capacity overflow, bit 1: numeric, bit 2: inflow layer past cap */
    int32_t levels[2];      /* cell-grid levels used by the last search (coarsest, finest) */
    int64_t n_mlp;          /* LP_EST_MLP: particles whose phi came from the network in the last step */
    int64_t n_mlp_plain;    /* LP_EST_MLP: particles that fell back to the quotient estimator */
    int64_t n_refined;      /* LP_MIXED with refine: fits refined in the last step */
    int64_t n_list_builds;  /* full neighbour searches of the steps so far (LP_TUNE_LIST_SKIN: the
                               steps in between reuse their candidate lists) */
    int64_t n_captures;     /* step graphs captured by lp_run / lp_run_open so far */
} lp_info;

/* Fill cfg with the defaults for the given dimension (gamma 1.4, cfl 0.5,
 * kappa 2.5 / 2.1, max_nb 128, est_eps 1e-5, cond_max 1e12, uw_cond_max 1e2,
 * cond_fallback 1e6, limiter_cap 1, unit box, fully periodic). */
void lp_config_default(lp_config *cfg, int32_t dim);

/* Create / destroy a context.  lp_create validates cfg (LP_E_ARG on failure)
 * and selects the HIP device that is current on the calling thread. */
lp_status lp_create(const lp_config *cfg, struct lp_ctx **ctx);
lp_status lp_destroy(struct lp_ctx *ctx);

/* Neighbour search (Sec. 2.2, step 3): for each i < n,
 *   N(i) = { j != i : d2(i, j) < r[i]^2 },
 *   d2 = ((dx*dx) + (dy*dy)) + (dz*dz) in IEEE binary64 without contraction,
 *   dx = minimum-image displacement on periodic axes of the context's box,
 * ordered by (d2, j).  count[i] receives |N(i)| (the true count even when it
 * exceeds max_nb); idx[i * max_nb + c] receives the c-th member for
 * c < min(count[i], max_nb).  x, y, z, r: device arrays of n doubles (z is
 * ignored in 2D); count: n int32; idx: n * max_nb int32.  Returns
 * LP_E_CAPACITY (after a synchronisation) when a count exceeds max_nb.
 * Mirror walls are not applied. */
lp_status lp_neighbors(struct lp_ctx *ctx, void *stream, int64_t n, const double *x, const double *y,
                       const double *z, const double *r, int32_t *count, int32_t *idx);

/* Caller-owned workspace (the store/solver split of Sec. 2.2: the particle
 * store and the solver's scratch are separate objects).
 *
 * lp_workspace_bytes: the device bytes a time step (lp_step, lp_run or
 * lp_run_open; for lp_run_open, p->n is the capacity: every slot is counted)
 * of the particles p needs when every buffer comes from one caller block: the
 * radii, ghosts, cell tables of the grid planned for p (with lp_run's
 * headroom), cell-order copies, neighbour lists, derivatives and, per the
 * context's configuration, refinement, network and list-reuse buffers.
 * Runs the planning part of a step (radii, ghost count, grid; synchronises)
 * and writes the total, with 256 bytes of alignment slack, to *bytes (host).
 * The particles are only read.
 *
 * lp_set_workspace: every later buffer of the context is carved, 256-byte
 * aligned, from the caller's device block dev[0 .. bytes) instead of being
 * allocated; the context's own buffers are freed (the network's parameters
 * and optimiser moments move into the block).  dev stays the caller's (never
 * freed by the library) and must outlive the context or a later call; dev =
 * NULL returns to library-allocated buffers.  A step whose buffers no longer
 * fit -- more particles or ghosts, a finer grid, a buffer that grows (it is
 * carved again after the others) -- returns LP_E_CAPACITY before launching
 * anything; calling lp_set_workspace again (with the same or a larger
 * block) starts carving afresh.  Synchronises the stream.  LP_E_ARG for a
 * block that is not 256-byte aligned or smaller than 256 bytes. */
lp_status lp_workspace_bytes(struct lp_ctx *ctx, void *stream, const lp_particles *p, int64_t *bytes);
lp_status lp_set_workspace(struct lp_ctx *ctx, void *stream, void *dev, int64_t bytes);

/* lp_neighbors for callers that cannot allocate device memory (code under
 * HIP graph capture, serving loops, harnesses that forbid hipMalloc): the
 * same lists, bit for bit, computed in a static scratch block of
 * LP_NOALLOC_SCRATCH_BYTES that the library holds on each device it runs on
 * until the process ends.  No hipMalloc, hipFree or allocating library call
 * is made; the context's own workspace is left untouched.  The block must
 * hold the call's whole workspace (about 4 * max_nb + 100 bytes per particle
 * plus the cell tables: some 100,000 particles at max_nb 128); a larger call
 * returns LP_E_NOMEM with nothing written to count or idx (LP_E_CAPACITY
 * keeps lp_neighbors' meaning: a list longer than max_nb).  The context's
 * device must be current (LP_E_STATE otherwise).  Every call on a device
 * uses that device's one block: calls that overlap in time on one device
 * (other streams, other threads, other contexts) race and must be
 * serialised by the caller.  Synchronises like lp_neighbors. */
#define LP_NOALLOC_SCRATCH_BYTES (64u << 20)
lp_status lp_neighbors_noalloc(struct lp_ctx *ctx, void *stream, int64_t n, const double *x, const double *y,
                               const double *z, const double *r, int32_t *count, int32_t *idx);

/* Second-order GFD derivatives (Sec. 2.1): for each particle i, the
 * least-squares fit over its Lax-Wendroff stencil (neighbours within r[i],
 * octant round-robin order, first lw_cap) of
 *   f_j - f_i = sum_a d_a f dx_a + 1/2 sum_a d_aa f dx_a^2 + sum_{a<b} d_ab f dx_a dx_b.
 * f: host array of nf (1..5) device pointers to n doubles each.
 * deriv: device, nf * nu * n doubles, deriv[(f * nu + c) * n + i] with nu = 9
 * (3D: x, y, z, xx, yy, zz, xy, xz, yz) or 5 (2D: x, y, xx, yy, xy).
 * status: device, n bytes: 0 = second-order fit, 1 = rank deficient (linear
 * fit, second derivatives 0), 2 = fewer than dim usable neighbours (all 0).
 * x, y, z, r: device arrays of n doubles (z ignored in 2D); all arrays are
 * the caller's and are only read (deriv, status only written).  Always solved
 * in FP64.  Synchronises twice (to size the cell grid, and at the end).
 * Returns LP_E_ARG for n outside 1..2^30, nf outside 1..5 or a null pointer,
 * LP_E_CAPACITY when a neighbour count exceeds max_nb (the fits then use the
 * first max_nb neighbours), LP_E_NOMEM when the workspace cannot grow. */
lp_status lp_gfd(struct lp_ctx *ctx, void *stream, int64_t n, const double *x, const double *y,
                 const double *z, const double *r, int32_t nf, const double *const *f, double *deriv,
                 uint8_t *status);

/* Third-order GFD derivatives (Sec. 2.1, the Taylor system carried to the
 * cubic terms): for each particle i, the least-squares fit over the same
 * stencil as lp_gfd of
 *   f_j - f_i = (second-order terms of lp_gfd)
 *             + sum_{|alpha| = 3} d^alpha f dx^alpha / alpha!,
 * solved by Householder QR with column pivoting on coordinates scaled by r[i].
 * Arguments and layout as lp_gfd with nu = 19 (3D: x, y, z, xx, yy, zz, xy,
 * xz, yz, xxx, yyy, zzz, xxy, xxz, xyy, yyz, xzz, yzz, xyz; xyy is
 * d3f / dx dy dy) or 9 (2D: x, y, xx, yy, xy, xxx, yyy, xxy, xyy).
 * status: 0 = third-order fit; 1 = the cubic system has fewer rows than
 * unknowns or |R11|/|Rnn| above cond_max, and the values are lp_gfd's
 * second-order fit of the same stencil (third derivatives 0); 2 = that fit is
 * deficient too (linear fit); 3 = fewer than dim usable neighbours (all 0).
 * Always FP64; one wave per particle.  Synchronisation and errors as lp_gfd. */
lp_status lp_gfd3(struct lp_ctx *ctx, void *stream, int64_t n, const double *x, const double *y,
                  const double *z, const double *r, int32_t nf, const double *const *f, double *deriv,
                  uint8_t *status);

/* One time step (Sec. 2.2, steps 1-6) of the particle set p, in place:
 * dt > 0 is used as given, dt <= 0 selects cfl * min_i h_i / c_i.
 * Synchronises once (to size the cell grid).  Mass is never modified.  A
 * particle of zero mass is absent: it has no radius, no ghost and no
 * neighbours, is neither updated nor counted in dt, and is left as it is. */
lp_status lp_step(struct lp_ctx *ctx, void *stream, const lp_particles *p, double dt);

/* Advance p by nsteps CFL-limited steps or until the accumulated time reaches
 * t_end (t_end <= 0: no limit); the last step is shortened to end on t_end.
 * The first step plans the cell grid and the workspace (with headroom for
 * growth) and synchronises once; the following steps are one captured HIP
 * graph replayed on `stream`, with dt and t kept on the device.  Every 8
 * replays the call synchronises to stop at t_end and to re-plan (with a new
 * capture) when the particles outgrow the grid or the ghost capacity; a
 * replayed step that finds more mirror ghosts than the workspace holds is
 * skipped whole and redone after re-planning.  Results are identical to
 * nsteps calls of lp_step.  The run stops after the first step that reports
 * a capacity or numeric error (steps replayed after it are skipped whole and
 * change nothing); lp_check then reports the error, and an error still
 * pending from earlier steps stops the run before its first step.  The graph
 * is kept for the next call with the same particle arrays.  The caller must
 * not free or move the arrays while the call runs. */
lp_status lp_run(struct lp_ctx *ctx, void *stream, const lp_particles *p, int32_t nsteps, double t_end);

/* Totals in FP64: out[0] = sum m, out[1..3] = sum m u, out[4] = sum m (e + |u|^2/2),
 * e = P V / (gamma - 1).  out is a host array of 5 doubles.  Synchronises. */
lp_status lp_conservation(struct lp_ctx *ctx, void *stream, const lp_particles *p, double *out);

/* Open boundary, outflow (Sec. 2.2, step 1: outflow boundaries delete
 * particles): remove, in place, every particle with x_a < box_lo[a] for a bit
 * a of lo_mask or x_a >= box_hi[a] for a bit a of hi_mask; the others keep
 * their order.  Every array of p is compacted: x, u, V, P, m (the caller's
 * mass array, constant for the step, is written here) and phi, flags when not
 * NULL.  *n_kept (host) receives the new count; entries past it are left as
 * they were.  Synchronises once.  Call between steps, with a p->n of the new
 * count afterwards. */
lp_status lp_outflow(struct lp_ctx *ctx, void *stream, const lp_particles *p, uint32_t lo_mask, uint32_t hi_mask,
                     int64_t *n_kept);

/* Reservoir inflow state (Sec. 3.2): the state of particles entering through
 * the face of axis `axis` (side 0: box_lo, 1: box_hi) from a reservoir at rest
 * with pressure p_res and density rho_res.
 *   P_in:   mean pressure of the particles at distance 0 <= d < width inside
 *           the face (p_res when there are none);
 *   rho_in: equal entropy, p_res / rho_res^gamma = P_in / rho_in^gamma;
 *   u_in:   equal enthalpy with the reservoir at rest,
 *           u_in^2 / 2 + c_in^2 / (gamma - 1) = c_res^2 / (gamma - 1), c^2 = gamma P / rho
 *           (0 when the layer's pressure is at or above the reservoir's).
 * out (host, 4 doubles): P_in, rho_in, u_in (speed into the domain, normal to
 * the face), particles averaged.  LP_E_ARG for a bad face, width <= 0 or a
 * non-positive reservoir state.  Synchronises once.  Placing the particles
 * that enter (and their mass) is the caller's. */
lp_status lp_reservoir_inflow(struct lp_ctx *ctx, void *stream, const lp_particles *p, int32_t axis, int32_t side,
                              double width, double p_res, double rho_res, double *out);

/* Inflow layer (Sec. 2.2, step 1: inflow boundaries generate particles):
 * append one layer of particles on the square lattice of the given spacing,
 * in the plane at distance `depth` inside the face of axis `axis` (side 0:
 * box_lo, 1: box_hi).  Each other axis b holds box_lo[b] + (k + 1/2) spacing,
 * k = 0 .. floor((box_hi[b] - box_lo[b]) / spacing + 1e-9) - 1 (a cell short
 * of a whole one by rounding alone still counts), the first other axis running
 * fastest.  The new particles take V = 1 / rho, pressure p_in,
 * velocity u_n along the inward normal (0 in the other components) and mass
 * rho spacing^dim; phi = 1 and flags = 0 when those arrays are given.  A
 * reservoir face takes the state lp_reservoir_inflow returns.
 * p->n is the current count; every array of p (device) must hold cap entries,
 * and entries p->n .. *n_new - 1 are written (the mass array too).  *n_new
 * (host) receives the new count.  LP_E_ARG for a bad face, spacing <= 0,
 * depth < 0, rho <= 0, p_in <= 0, or cap < p->n; LP_E_CAPACITY (nothing
 * written) when the layer does not fit in cap.  Asynchronous on `stream`.
 * Call between steps, with a p->n of the new count afterwards. */
lp_status lp_inflow_layer(struct lp_ctx *ctx, void *stream, const lp_particles *p, int64_t cap, int32_t axis,
                          int32_t side, double spacing, double depth, double rho, double p_in, double u_n,
                          int64_t *n_new);

/* Open boundaries of lp_run_open (Sec. 2.2, step 1).  Outflow: after each
 * step, every particle with x_a < box_lo[a] for a bit a of out_lo_mask or
 * x_a >= box_hi[a] for a bit a of out_hi_mask leaves (as lp_outflow).
 * Inflow (in_every > 0): after every in_every-th step, and after the
 * outflow, one layer as lp_inflow_layer writes it on face (in_axis, in_side)
 * with the given spacing and depth; its state is rho, p_in, u_n when
 * res_width <= 0, else the reservoir state that lp_reservoir_inflow computes
 * at that moment for the layer of width res_width inside the face, from a
 * reservoir at rest with pressure res_p and density res_rho. */
typedef struct lp_open_bc {
    uint32_t out_lo_mask, out_hi_mask;  /* outflow faces, bit a: axis a */
    int32_t in_every;                   /* 0: no inflow */
    int32_t in_axis, in_side;           /* inflow face (side 0: box_lo, 1: box_hi) */
    double spacing, depth;              /* layer lattice spacing, distance of its plane inside the face */
    double rho, p_in, u_n;              /* fixed state of entering particles (res_width <= 0) */
    double res_width, res_p, res_rho;   /* reservoir (res_width > 0) */
} lp_open_bc;

/* lp_run with open boundaries inside the steps: each step as lp_run's (the
 * same captured graph replays, one capture for the whole run while the grid
 * and the ghost capacity serve), followed on the device by the outflow and,
 * on every in_every-th step, the inflow layer of *bc (host).  Deleted
 * particles are marked with zero mass and stay in their slots until the end
 * of the call; layers are appended after the last slot in use.  At the end
 * every array of p is compacted as lp_outflow does: the present particles
 * keep their order, the layers after the particles that were there before.
 * The result equals nsteps repetitions of lp_step, lp_outflow and, every
 * in_every-th time, lp_reservoir_inflow and lp_inflow_layer (the reservoir
 * pressure summed in another order: equal within rounding).
 * p->n (>= 1) is the current count; every array of p (device) must hold cap
 * entries (cap <= 2^30), and the mass array is written: entries p->n .. cap - 1
 * are set to zero first (those slots are absent until a layer fills them),
 * and a particle given with zero mass is absent and removed.  *n_out (host)
 * receives the final count (0 when every particle left; the run then stops).
 * LP_E_ARG for a bad count, cap, mask or inflow setting (nothing written).  A
 * layer that does not fit in cap is not written and stops the run as an
 * error of lp_run does; lp_check then reports LP_E_CAPACITY.  The arrays are
 * compacted, and *n_out set, also when the run itself returns an error. */
lp_status lp_run_open(struct lp_ctx *ctx, void *stream, const lp_particles *p, int64_t cap, const lp_open_bc *bc,
                      int32_t nsteps, double t_end, int64_t *n_out);

/* Synchronise and report kernel-side errors of all work since the last
 * check (LP_E_CAPACITY / LP_E_NUMERIC), then clear them. */
lp_status lp_check(struct lp_ctx *ctx, void *stream);

/* Synchronise and copy the diagnostics of the last step to *out (host). */
lp_status lp_get_info(struct lp_ctx *ctx, void *stream, lp_info *out);

/* Set the accumulated time (host value). */
lp_status lp_set_time(struct lp_ctx *ctx, void *stream, double t);

/* Kernel timing with HIP events recorded on the caller's stream around each
 * stage of lp_step / lp_run.  lp_profile(ctx, 1) starts recording (and clears
 * earlier records), lp_profile(ctx, 0) stops.  lp_profile_read synchronises
 * and writes, per stage, the summed milliseconds ms[q] and the number of
 * timed launches count[q] (host arrays of LP_NSTAGES entries), then clears.
 * Stages: 0 radii/dt/ghosts, 1 cell ordering, 2 neighbour search (+ work
 * queue), 3 second-order fits (fast path; in lp_gfd and lp_gfd3 their fit
 * kernels, fallback included), 4 half-ball fits + estimator +
 * update + mover, 5 FP64 pivoted-QR fallback, 6 whole step (also around each
 * graph replay of lp_run, whose inner stages are not timed), 7 estimator
 * network with the update it decides (LP_EST_MLP). */
#define LP_NSTAGES 8
#define LP_STAGE_STEP 6

/* Launch-shape parameters (results are identical for every setting; only the
 * speed changes).  Chosen by lp_autotune() or set explicitly: */
enum {
    LP_TUNE_SEARCH_MODE = 0,   /* 0: lane group per particle walking its cells, 1: LDS-staged tiles,
                                  2: lane group with pruned cells and candidates dealt evenly (default) */
    LP_TUNE_SEARCH_GROUP = 1,  /* lanes per particle of modes 0 and 2: 4, 8 (default), 16, 32 */
    LP_TUNE_SOLVE_BLOCK = 2,   /* threads per block of the fit and update kernels: 64, 128, 256 */
    LP_TUNE_SOLVE_MODE = 3,    /* 0: one thread per cell-order particle; 1: work queue regrouped by
                                  neighbour count within tiles of cell-order particles; 2: persistent
                                  launch over that queue */
    LP_TUNE_QUEUE_TILE = 4,    /* tile of the work queue of modes 1 and 2: 256, 512, 1024 */
    LP_TUNE_SEARCH_CAP = 5,    /* list slots per particle held in LDS by search mode 2 (longer lists
                                  are redone by an overflow kernel): 0 (default) = chosen by each
                                  planning step from the previous step's longest list, else a
                                  multiple of 8 in 8..128 */
    LP_TUNE_LIST_SKIN = 6,     /* neighbour-list reuse across time steps, in per mille of r: 0 = a full
                                  search every step; s > 0 (default 250) = a full search within
                                  (1 + s/1000) r only when the last one may miss a neighbour (checked on
                                  the device each step from the displacements since that search and
                                  the growth of r), and in between the exact test d2 < r_i^2 and the
                                  (d2, id) ranking over those candidates.  Used by lp_step / lp_run
                                  without mirror walls and with search mode 2; the lists are the full
                                  search's bit for bit.  Candidate lists must fit max_nb. */
    LP_TUNE_COUNT = 7
};
lp_status lp_set_tuning(struct lp_ctx *ctx, int32_t param, int32_t value);

/* Autotuner: time full steps of a private copy of p (p itself is not
 * modified) for every launch-shape setting in turn -- the solve mode, the
 * queue tile, the fit/update block size, the search mode and group (not the
 * list skin: a few steps cannot show how often a run rebuilds) -- keep the
 * fastest setting of each
 * (coordinate descent, `reps` timed steps per candidate after one warm-up),
 * and write the chosen values to best[LP_TUNE_COUNT] (host; may be NULL) and
 * the per-step milliseconds of the best setting to *ms (host; may be NULL).
 * Synchronises.  Allocates a copy of p's state for its duration.  The
 * context's device scalars (time, dt, step count, error bits) are restored
 * afterwards, also on failure; a candidate step's capacity or numeric error
 * is returned as LP_E_CAPACITY / LP_E_NUMERIC by lp_autotune itself. */
lp_status lp_autotune(struct lp_ctx *ctx, void *stream, const lp_particles *p, int32_t reps, int32_t *best,
                      double *ms);
lp_status lp_get_tuning(const struct lp_ctx *ctx, int32_t param, int32_t *value);
lp_status lp_profile(struct lp_ctx *ctx, int32_t enable);
lp_status lp_profile_read(struct lp_ctx *ctx, void *stream, double *ms, int64_t *count);

/* ---------------------------------------------------------------------------
 * Estimator network (not part of the paper's method): 16 -> 64 -> 64 -> 1 with
 * ReLU hidden layers and a sigmoid output, standing in for the state
 * estimator of the blended update (Sec. 2.1).  Inputs per particle, all
 * dimensionless: h d_a(rho)/rho (3), h d_a P/P (3), h div u / c, for V and P
 * on every axis the disagreement of the one-sided slopes that the quotient
 * estimator looks at (|log| of their quotient, at most 8; 8 for opposite signs;
 * 0 where the estimator ignores the pair) (6), log(V_max/V_min) and
 * log(P_max/P_min) over the half-ball members (2), h |grad u|_F / c.
 * Parameters (FP32, LP_MLP_NPARAM in this order): W1[64][16], b1[64],
 * W2[64][64], b2[64], w3[64], b3.  Inference and training run on BF16 matrix
 * instructions with FP32 accumulation.  As the estimator of a step the
 * network gives phi = min(1, 1.25 y), y its sigmoid output -- the limiter's
 * range -- so a network that imitates the quotient estimator is trained on
 * targets phi / 1.25.
 * ------------------------------------------------------------------------- */
#define LP_MLP_NIN 16
#define LP_MLP_NPARAM 5313

typedef struct lp_train_cfg {
    int32_t epochs;         /* passes over the samples */
    int32_t batch;          /* samples per Adam step */
    float lr, beta1, beta2, eps;   /* Adam */
    uint64_t seed;          /* order of the batches in every epoch */
    int32_t reserved[6];
} lp_train_cfg;

/* Defaults: 10 epochs, batch 4096, lr 2e-3, beta1 0.9, beta2 0.999, eps 1e-8, seed 1. */
void lp_train_cfg_default(lp_train_cfg *cfg);

/* Inputs and quotient-estimator phi of every particle of p at its current
 * state (Sec. 2.2 steps 1-5 as in lp_step, nothing advanced): feat (device,
 * n * 16 floats, particle i at feat[16 i]), phi (device, n floats), valid
 * (device, n bytes: 0 where phi = 0 is forced, for degenerate or vacuum
 * particles).  These are the training samples of the network.  The output
 * buffers are the caller's; valid may be NULL. */
lp_status lp_features(struct lp_ctx *ctx, void *stream, const lp_particles *p, float *feat, float *phi,
                      uint8_t *valid);

/* Network parameters: lp_mlp_init draws He-uniform weights (zero biases)
 * from seed; lp_mlp_set / lp_mlp_get copy all LP_MLP_NPARAM FP32 values from /
 * to a host array (count must be LP_MLP_NPARAM).  lp_step with LP_EST_MLP
 * returns LP_E_STATE until parameters are set. */
lp_status lp_mlp_init(struct lp_ctx *ctx, uint64_t seed);
lp_status lp_mlp_set(struct lp_ctx *ctx, const float *params, int64_t count);
lp_status lp_mlp_get(struct lp_ctx *ctx, float *params, int64_t count);

/* Network output for n samples: feat (device, n * 16), z (device, n) the
 * pre-sigmoid output and y (device, n) the sigmoid; z or y may be NULL. */
lp_status lp_mlp_forward(struct lp_ctx *ctx, void *stream, int64_t n, const float *feat, float *z, float *y);

/* Mean binary cross-entropy of the network output against target (device,
 * n floats in [0, 1]) and its gradient with respect to the parameters
 * (host, LP_MLP_NPARAM floats); *loss host.  Synchronises. */
lp_status lp_mlp_grad(struct lp_ctx *ctx, void *stream, int64_t n, const float *feat, const float *target,
                      float *grad, float *loss);

/* Adam on the mean binary cross-entropy over n samples (device feat, target),
 * from the current parameters; loss (host, cfg->epochs floats, may be NULL)
 * receives each epoch's mean batch loss.  Samples should come shuffled: the
 * batches are contiguous ranges, visited in a seeded order.  Synchronises. */
lp_status lp_mlp_train(struct lp_ctx *ctx, void *stream, int64_t n, const float *feat, const float *target,
                       const lp_train_cfg *cfg, float *loss);

const char *lp_status_str(lp_status s);
const char *lp_last_error(const struct lp_ctx *ctx);

#ifdef __cplusplus
}
#endif
#endif
