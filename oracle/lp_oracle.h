/*
 * lp_oracle.h -- interface of the FP64 CPU reference (test infrastructure only).
 * Used by the tests, the smoke check and the CPU-baseline leg of the benchmark;
 * never by the product library.  See lp_oracle.c for the paper mapping.
 */
#ifndef LP_ORACLE_H
#define LP_ORACLE_H
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

enum { LPO_OK = 0, LPO_E_ARG = 1, LPO_E_CAPACITY = 2, LPO_E_NUMERIC = 3, LPO_E_NOMEM = 5 };

enum {
    LPO_FLAG_LIMITED = 1,      /* phi < 1: blended towards upwind */
    LPO_FLAG_DEGENERATE = 2,   /* second-order fit rank deficient: linear fit, phi = 0 */
    LPO_FLAG_VACUUM = 4,       /* half-ball completed by vacuum ghosts, phi = 0 */
    LPO_FLAG_SUBSTITUTED = 8,  /* a half-ball fit failed: LW gradient used for that side */
    LPO_FLAG_NUMERIC = 32      /* non-positive V or P after the update */
};

typedef struct {
    int32_t dim;          /* 2 or 3 */
    int32_t lw_cap;       /* 0 -> 54 (3D) / 32 (2D) */
    int32_t uw_cap;       /* 0 -> 8, at most 64 */
    int32_t max_nb;       /* neighbour-list capacity */
    double gamma, cfl, kappa;
    double est_eps;       /* estimator activity threshold */
    double cond_max;      /* |R11|/|Rnn| above this: second-order fit rank deficient */
    double uw_cond_max;   /* |R11|/|Rnn| above this: half-ball fit unusable */
    double lo[3], hi[3];  /* box */
    int32_t periodic[3];
    int32_t wall_lo[3], wall_hi[3];
    int32_t vacuum;       /* free boundary: vacuum ghosts complete half-balls */
    double phi_fixed;     /* >= 0: every particle blends with this phi (1: pure Lax-Wendroff,
                             0: pure upwind) instead of the estimator's; < 0: the estimator */
    double limiter_cap;   /* > 0: phi = min(phi, limiter_cap); <= 0: the limiter as printed, whose
                             largest value is 1.25 at r = 1 */
} lpo_cfg;

int lpo_num_threads(void);
void lpo_set_num_threads(int n);   /* OpenMP threads of later calls (results do not depend on it) */
double lpo_limiter(double r);
double lpo_estimator_ratio(double sl, double sr);
double lpo_lstsq_qrp(int k, int n, int nrhs, double *A, double *B, double *X);
int lpo_lw_select(int dim, int k, const double *dxs, int cap, int *sel);
void lpo_lw_rates(int dim, double gamma, double dt, const double *st, const double *grad,
                  const double *hess, double *rate);
void lpo_uw_rates(int dim, double gamma, const double *st, const double *dl, const double *dr,
                  double *rate);
int lpo_neighbors(const lpo_cfg *c, int64_t n, const double *x, const double *y, const double *z,
                  const double *r, int32_t max_nb, int32_t *count, int32_t *idx);
int lpo_neighbors_subset(const lpo_cfg *c, int64_t n, const double *x, const double *y, const double *z,
                         const double *r, int32_t max_nb, int64_t nq, const int64_t *q, int32_t *count,
                         int32_t *idx);
int lpo_gfd(const lpo_cfg *c, int64_t n, const double *x, const double *y, const double *z,
            const double *r, int32_t nf, const double *const *f, double *deriv, uint8_t *status);
/* Third-order GFD derivatives: deriv[(f * nu + col) * n + i], nu = 19 (3D) or 9
 * (2D), columns as lp_gfd's followed by the cubic ones; status 0 = cubic fit,
 * 1 = quadratic, 2 = linear, 3 = none. */
int lpo_gfd3(const lpo_cfg *c, int64_t n, const double *x, const double *y, const double *z,
             const double *r, int32_t nf, const double *const *f, double *deriv, uint8_t *status);
/* Open boundaries: outflow deletion (in place, order kept) and the state of
 * particles entering from a reservoir at rest (out: P_in, rho_in, u_in, count). */
int lpo_outflow(const lpo_cfg *c, int64_t n, double *const *arrays, int narr, const double *const *x,
                uint32_t lo_mask, uint32_t hi_mask, int64_t *n_kept);
int lpo_reservoir_inflow(const lpo_cfg *c, int64_t n, const double *const *x, const double *P, int axis, int side,
                         double width, double p_res, double rho_res, double *out);
int lpo_inflow_layer(const lpo_cfg *c, int64_t n, int64_t cap, double *const *x, double *const *u, double *V,
                     double *P, double *m, int axis, int side, double spacing, double depth, double rho,
                     double p_in, double u_n, int64_t *n_new);
double lpo_timestep(const lpo_cfg *c, int64_t n, const double *V, const double *P, const double *m);
int lpo_step_subset(const lpo_cfg *c, int64_t n, const double *x, const double *y, const double *z,
                    const double *V, const double *u, const double *v, const double *w,
                    const double *P, const double *m, double dt_in, int64_t nsub, const int64_t *sub,
                    double *ox, double *oy, double *oz, double *oV, double *ou, double *ov,
                    double *ow, double *oP, double *ophi, uint8_t *oflags, double *dt_used,
                    int64_t *n_ghost, double *ofeat /* nsub x 16 or NULL: estimator-network inputs */);
int lpo_step(const lpo_cfg *c, int64_t n, double *x, double *y, double *z, double *V, double *u,
             double *v, double *w, double *P, const double *m, double dt_in, double *phi,
             uint8_t *flags, double *dt_used, int64_t *n_ghost);
void lpo_conservation(const lpo_cfg *c, int64_t n, const double *V, const double *u, const double *v,
                      const double *w, const double *P, const double *m, double *out);
#define LPO_MLP_NPARAM 5313
void lpo_mlp_forward(const double *theta, int64_t n, const double *feat, double *z, double *y);
double lpo_mlp_loss_grad(const double *theta, int64_t n, const double *feat, const double *target,
                         double *grad);
int lpo_particle_derivs(const lpo_cfg *c, int64_t n, const double *x, const double *y, const double *z,
                        const double *V, const double *u, const double *v, const double *w,
                        const double *P, int64_t i, const int32_t *list, int32_t k, double h, double s,
                        double *grad, double *hess, double *dl, double *dr, int32_t *valid, double *phi,
                        int32_t *flags);

#ifdef __cplusplus
}
#endif
#endif
