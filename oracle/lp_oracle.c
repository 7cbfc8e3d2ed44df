/*
 * lp_oracle.c -- slow, plain FP64 CPU reference of the Lagrangian particle (LP)
 * time step of Yuan, Zepeda Aguilar, Naitlho & Samulyak, "Massively-Parallel
 * Lagrangian Particle Code and Applications" (arXiv 2206.11998).
 *
 * TEST INFRASTRUCTURE ONLY.  Nothing in the product library links, loads or
 * calls this file; only the tests, the smoke check and the CPU-baseline leg of
 * the benchmark do.  It shares no code, header, table or constant with the GPU
 * path.
 *
 * Arithmetic: IEEE binary64, round-to-nearest, built with -ffp-contract=off and
 * no fast-math, so every expression below is evaluated exactly as written.
 * Particle-level loops are independent and run under OpenMP; results do not
 * depend on the thread count.
 *
 * Section map (paper numbering):
 *   Sec. 2.1, eqs. (mass)-(eos) ...... Lagrangian Euler system, ideal gas
 *   Sec. 2.1, upwind eqs ............. first-order upwind rates (1D printed;
 *                                       multi-D reading: sum over axes)
 *   Sec. 2.1, LW derivation .......... Cauchy-Kowalevski second derivatives
 *                                       (multi-D form derived from the same
 *                                       commutation rule; 1D typo in the
 *                                       printed u-update fixed to +gamma V u_x P_x)
 *   Sec. 2.1, GFD system + "QR with column pivoting"
 *   Sec. 2.1, blend, state estimator, limiter, particle mover
 *   Sec. 2.2, steps 1-6 of the time-step loop
 *
 * Parity unpinned: two readings here have no pin of their own -- their 1D or
 * special cases are pinned, their general form only by parity with the GPU
 * path and by the Sod and Yee trends: the multi-D upwind rate as the sum over
 * axes of the 1D characteristic form (lpo_uw_rates), and the state
 * estimator's aggregation over fields and axes, the largest quotient of the
 * active V and P pairs (the est_eps test in solve_particle).
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#include "lp_oracle.h"

#ifdef _OPENMP
#include <omp.h>
#endif

int lpo_num_threads(void)
{
#ifdef _OPENMP
    return omp_get_max_threads();
#else
    return 1;
#endif
}

void lpo_set_num_threads(int n)
{
#ifdef _OPENMP
    if (n > 0) omp_set_num_threads(n);
#else
    (void)n;
#endif
}

#define ORC_MAXN 9      /* unknowns of the 3D second-order fit */
#define ORC_MAXN3 19    /* unknowns of the 3D third-order fit */
#define ORC_MAXF 5      /* fields V, u1..uD, P */

/* ------------------------------------------------------------------------- */
/* Small helpers                                                              */
/* ------------------------------------------------------------------------- */

static int nfit2(int dim) { return dim == 3 ? 9 : 5; }           /* 2nd-order unknowns */
static int nfit3(int dim) { return dim == 3 ? 19 : 9; }          /* 3rd-order unknowns */
static int nsecond(int dim) { return dim == 3 ? 6 : 3; }         /* 2nd-derivative cols */

/* Minimum-image displacement along one axis (Sec. 2.2: periodic domains are
 * handled by the connectivity of the octree forest; here the same effect is
 * the minimum-image convention). */
static double min_image(const lpo_cfg *c, int a, double d)
{
    if (c->periodic[a]) {
        double L = c->hi[a] - c->lo[a];
        double half = 0.5 * L;
        if (d > half) d -= L;
        else if (d < -half) d += L;
    }
    return d;
}

/* Smoothing length h = (m V)^(1/D): the particle's volume share (Sec. 2.1: the
 * number density of particles is proportional to the mass density). */
static double smoothing_length(int dim, double m, double V)
{
    return dim == 3 ? cbrt(m * V) : sqrt(m * V);
}

/* ------------------------------------------------------------------------- */
/* Limiter and state estimator (Sec. 2.1, estimator and limiter formulas)    */
/* ------------------------------------------------------------------------- */

double lpo_limiter(double r)
{
    if (isinf(r)) return 0.0;
    double q = sqrt(r);
    if (r <= 1.5) return 1.25 * exp(1.0 - q);
    double t = q - 1.0;
    return 1.25 * exp(-4.5 * (t * t));
}

double lpo_estimator_ratio(double sl, double sr)
{
    if (sl * sr <= 0.0) return INFINITY;
    return 0.5 * (sr / sl + sl / sr);
}

/* ------------------------------------------------------------------------- */
/* Least squares by Householder QR with column pivoting (Sec. 2.1, GFD).      */
/* A is k x n row-major, B is k x nrhs row-major; both are overwritten.       */
/* X receives n x nrhs (row-major).  Column norms of the trailing block are   */
/* recomputed from scratch at every step.  Returns cond = |R11| / |Rnn|.      */
/* ------------------------------------------------------------------------- */

double lpo_lstsq_qrp(int k, int n, int nrhs, double *A, double *B, double *X)
{
    int perm[ORC_MAXN3 + 1];
    double Y[(ORC_MAXN3 + 1) * ORC_MAXF];
    for (int j = 0; j < n; ++j) perm[j] = j;
    int steps = k < n ? k : n;
    for (int p = 0; p < steps; ++p) {
        /* pivot: the remaining column of largest norm */
        int best = p;
        double bestnorm = -1.0;
        for (int j = p; j < n; ++j) {
            double s = 0.0;
            for (int r = p; r < k; ++r) s += A[r * n + j] * A[r * n + j];
            if (s > bestnorm) { bestnorm = s; best = j; }
        }
        if (best != p) {
            for (int r = 0; r < k; ++r) {
                double t = A[r * n + p];
                A[r * n + p] = A[r * n + best];
                A[r * n + best] = t;
            }
            int t = perm[p]; perm[p] = perm[best]; perm[best] = t;
        }
        /* Householder reflector H = I - tau v v^T that maps column p onto alpha e_p */
        double x0 = A[p * n + p];
        double sigma = 0.0;
        for (int r = p + 1; r < k; ++r) sigma += A[r * n + p] * A[r * n + p];
        double normx = sqrt(x0 * x0 + sigma);
        if (normx == 0.0) continue;
        double alpha = x0 >= 0.0 ? -normx : normx;
        double v0 = x0 - alpha;
        double tau = -1.0 / (alpha * v0);
        for (int j = p + 1; j < n; ++j) {
            double w = v0 * A[p * n + j];
            for (int r = p + 1; r < k; ++r) w += A[r * n + p] * A[r * n + j];
            w *= tau;
            A[p * n + j] -= w * v0;
            for (int r = p + 1; r < k; ++r) A[r * n + j] -= w * A[r * n + p];
        }
        for (int c = 0; c < nrhs; ++c) {
            double w = v0 * B[p * nrhs + c];
            for (int r = p + 1; r < k; ++r) w += A[r * n + p] * B[r * nrhs + c];
            w *= tau;
            B[p * nrhs + c] -= w * v0;
            for (int r = p + 1; r < k; ++r) B[r * nrhs + c] -= w * A[r * n + p];
        }
        A[p * n + p] = alpha;
        for (int r = p + 1; r < k; ++r) A[r * n + p] = 0.0;
    }
    if (k < n) {
        for (int i = 0; i < n * nrhs; ++i) X[i] = 0.0;
        return INFINITY;
    }
    double r11 = fabs(A[0]);
    double rnn = fabs(A[(n - 1) * n + (n - 1)]);
    double cond = rnn == 0.0 ? INFINITY : r11 / rnn;
    /* back substitution R y = Q^T b, then undo the column permutation */
    for (int c = 0; c < nrhs; ++c) {
        for (int p = n - 1; p >= 0; --p) {
            double y = B[p * nrhs + c];
            for (int j = p + 1; j < n; ++j) y -= A[p * n + j] * Y[j * nrhs + c];
            double d = A[p * n + p];
            Y[p * nrhs + c] = d == 0.0 ? 0.0 : y / d;
        }
    }
    for (int p = 0; p < n; ++p)
        for (int c = 0; c < nrhs; ++c) X[perm[p] * nrhs + c] = Y[p * nrhs + c];
    return cond;
}

/* ------------------------------------------------------------------------- */
/* Neighbour search (Sec. 2.2, step 3): N(i) = { j != i : d2(i,j) < r_i^2 },  */
/* d2 = ((dx*dx) + (dy*dy)) + (dz*dz) in FP64, ordered by (d2, id).            */
/* A uniform bucket grid of cell size >= max r only limits the candidates.    */
/* ------------------------------------------------------------------------- */

typedef struct { double d2; int32_t j; } nb_pair;

static int cmp_pair(const void *a, const void *b)
{
    const nb_pair *p = (const nb_pair *)a, *q = (const nb_pair *)b;
    if (p->d2 < q->d2) return -1;
    if (p->d2 > q->d2) return 1;
    return (p->j > q->j) - (p->j < q->j);
}

static double dist2(const lpo_cfg *c, const double *const X[3], int64_t i, int64_t j, double dx[3])
{
    dx[0] = dx[1] = dx[2] = 0.0;
    for (int a = 0; a < c->dim; ++a) dx[a] = min_image(c, a, X[a][j] - X[a][i]);
    double d2 = dx[0] * dx[0] + dx[1] * dx[1];
    if (c->dim == 3) d2 = d2 + dx[2] * dx[2];
    return d2;
}

/* Fills lists for the query particles q[0..nq) against all nall particles.
 * count[t] = true count; lists[t*cap + s] holds the first min(count,cap) ids. */
static int neighbor_lists(const lpo_cfg *c, int64_t nq, const int64_t *q, int64_t nall,
                          const double *const X[3], const double *r, int cap,
                          int32_t *count, int32_t *lists)
{
    int D = c->dim;
    /* Bucket size: at least the largest radius when radii are uniform; with
     * varying radii, the smallest radius (a query then scans
     * floor(r/cell) + 1 buckets on each side, which covers its ball). */
    double rmax = 0.0, rmin = INFINITY;
    for (int64_t t = 0; t < nq; ++t) {
        double v = r[q[t]];
        if (v > rmax) rmax = v;
        if (v < rmin) rmin = v;
    }
    if (!(rmax > 0.0)) rmax = 1.0;
    if (!(rmin > 0.0) || rmin > rmax) rmin = rmax;
    double target = (rmax <= 2.0 * rmin ? rmax : rmin) * 1.000001;
    double glo[3] = {0, 0, 0}, cs[3] = {1, 1, 1};
    int64_t nc[3] = {1, 1, 1};
    for (int a = 0; a < D; ++a) {
        double lo, ext;
        if (c->periodic[a]) { lo = c->lo[a]; ext = c->hi[a] - c->lo[a]; }
        else {
            double mn = INFINITY, mx = -INFINITY;
            for (int64_t j = 0; j < nall; ++j) { double v = X[a][j]; if (v < mn) mn = v; if (v > mx) mx = v; }
            lo = mn; ext = mx - mn; if (!(ext > 0.0)) ext = rmax;
        }
        int64_t n = (int64_t)floor(ext / target);
        if (n < 1) n = 1;
        if (n > 256) n = 256;
        glo[a] = lo; nc[a] = n; cs[a] = ext / (double)n;
    }
    int64_t ncell = nc[0] * nc[1] * nc[2];
    int64_t *cell_of = (int64_t *)malloc(sizeof(int64_t) * (size_t)(nall > 0 ? nall : 1));
    int64_t *start = (int64_t *)calloc((size_t)ncell + 1, sizeof(int64_t));
    int64_t *order = (int64_t *)malloc(sizeof(int64_t) * (size_t)(nall > 0 ? nall : 1));
    if (!cell_of || !start || !order) { free(cell_of); free(start); free(order); return LPO_E_NOMEM; }
    for (int64_t j = 0; j < nall; ++j) {
        int64_t ci[3] = {0, 0, 0};
        for (int a = 0; a < D; ++a) {
            int64_t v = (int64_t)floor((X[a][j] - glo[a]) / cs[a]);
            if (v < 0) v = 0;
            if (v >= nc[a]) v = nc[a] - 1;
            ci[a] = v;
        }
        cell_of[j] = (ci[2] * nc[1] + ci[1]) * nc[0] + ci[0];
        start[cell_of[j] + 1]++;
    }
    for (int64_t k = 0; k < ncell; ++k) start[k + 1] += start[k];
    {
        int64_t *fill = (int64_t *)malloc(sizeof(int64_t) * (size_t)ncell);
        if (!fill) { free(cell_of); free(start); free(order); return LPO_E_NOMEM; }
        memcpy(fill, start, sizeof(int64_t) * (size_t)ncell);
        for (int64_t j = 0; j < nall; ++j) order[fill[cell_of[j]]++] = j;
        free(fill);
    }
    int status = LPO_OK;
#pragma omp parallel
    {
        size_t bufcap = 256;
        nb_pair *buf = (nb_pair *)malloc(sizeof(nb_pair) * bufcap);
#pragma omp for schedule(dynamic, 16)
        for (int64_t t = 0; t < nq; ++t) {
            int64_t i = q[t];
            double ri2 = r[i] * r[i];
            int64_t ci[3] = {0, 0, 0};
            int64_t cid = cell_of[i];
            ci[0] = cid % nc[0]; ci[1] = (cid / nc[0]) % nc[1]; ci[2] = cid / (nc[0] * nc[1]);
            int64_t lo3[3], hi3[3];
            for (int a = 0; a < 3; ++a) {
                if (a >= D) { lo3[a] = hi3[a] = 0; continue; }
                int64_t R = (int64_t)floor(r[i] / cs[a]) + 1;
                if (c->periodic[a] && 2 * R + 1 >= nc[a]) { lo3[a] = 0; hi3[a] = nc[a] - 1; }
                else { lo3[a] = ci[a] - R; hi3[a] = ci[a] + R; }
            }
            size_t n = 0;
            for (int64_t z = lo3[2]; z <= hi3[2]; ++z)
                for (int64_t y = lo3[1]; y <= hi3[1]; ++y)
                    for (int64_t x = lo3[0]; x <= hi3[0]; ++x) {
                        int64_t cc[3] = {x, y, z};
                        int ok = 1;
                        for (int a = 0; a < D; ++a) {
                            if (c->periodic[a]) cc[a] = ((cc[a] % nc[a]) + nc[a]) % nc[a];
                            else if (cc[a] < 0 || cc[a] >= nc[a]) ok = 0;
                        }
                        if (!ok) continue;
                        int64_t cell = (cc[2] * nc[1] + cc[1]) * nc[0] + cc[0];
                        for (int64_t s = start[cell]; s < start[cell + 1]; ++s) {
                            int64_t j = order[s];
                            if (j == i) continue;
                            double dx[3];
                            double d2 = dist2(c, X, i, j, dx);
                            if (d2 < ri2) {
                                if (n == bufcap) { bufcap *= 2; buf = (nb_pair *)realloc(buf, sizeof(nb_pair) * bufcap); }
                                buf[n].d2 = d2; buf[n].j = (int32_t)j; ++n;
                            }
                        }
                    }
            qsort(buf, n, sizeof(nb_pair), cmp_pair);
            count[t] = (int32_t)n;
            size_t m = n < (size_t)cap ? n : (size_t)cap;
            for (size_t s = 0; s < m; ++s) lists[(size_t)t * (size_t)cap + s] = buf[s].j;
            if (n > (size_t)cap) {
#pragma omp atomic write
                status = LPO_E_CAPACITY;
            }
        }
        free(buf);
    }
    free(cell_of); free(start); free(order);
    return status;
}

int lpo_neighbors(const lpo_cfg *c, int64_t n, const double *x, const double *y, const double *z,
                  const double *r, int32_t max_nb, int32_t *count, int32_t *idx)
{
    const double *X[3] = {x, y, z ? z : x};
    int64_t *q = (int64_t *)malloc(sizeof(int64_t) * (size_t)(n > 0 ? n : 1));
    if (!q) return LPO_E_NOMEM;
    for (int64_t i = 0; i < n; ++i) q[i] = i;
    int st = neighbor_lists(c, n, q, n, X, r, max_nb, count, idx);
    free(q);
    return st;
}

/* The lists of the query particles q[0..nq) only, against all n particles. */
int lpo_neighbors_subset(const lpo_cfg *c, int64_t n, const double *x, const double *y, const double *z,
                         const double *r, int32_t max_nb, int64_t nq, const int64_t *q, int32_t *count,
                         int32_t *idx)
{
    const double *X[3] = {x, y, z ? z : x};
    return neighbor_lists(c, nq, q, n, X, r, max_nb, count, idx);
}

/* ------------------------------------------------------------------------- */
/* Stencils (Sec. 2.2, step 4; Sec. 2.1 "symmetric ... from all 8 octants",  */
/* "left and right semi-spheres").                                            */
/* ------------------------------------------------------------------------- */

/* Lax-Wendroff stencil: neighbours ordered so that the top of the list holds
 * members of every octant: key (rank within own octant, position in the
 * (d2,id)-ordered list).  Writes the selected list positions to sel. */
static int lw_select(int dim, int k, const double *dxs /* k x 3 */, int cap, int *sel)
{
    if (k <= cap) { for (int s = 0; s < k; ++s) sel[s] = s; return k; }
    int *rho = (int *)malloc(sizeof(int) * (size_t)k);
    int cnt[8] = {0, 0, 0, 0, 0, 0, 0, 0};
    for (int s = 0; s < k; ++s) {
        int o = 0;
        for (int a = 0; a < dim; ++a) if (dxs[s * 3 + a] >= 0.0) o |= 1 << a;
        rho[s] = cnt[o]++;
    }
    int m = 0;
    for (int level = 0; m < cap; ++level)
        for (int s = 0; s < k && m < cap; ++s)
            if (rho[s] == level) sel[m++] = s;
    free(rho);
    return m;
}

/* Upwind half-ball along axis a on side sgn (+1 right, -1 left): members with
 * sgn*dx_a > 0 in list order, at most cap. */
static int uw_select(int k, const double *dxs, int a, int sgn, int cap, int *sel)
{
    int m = 0;
    for (int s = 0; s < k && m < cap; ++s) {
        double d = dxs[s * 3 + a];
        if ((sgn > 0 && d > 0.0) || (sgn < 0 && d < 0.0)) sel[m++] = s;
    }
    return m;
}

/* ------------------------------------------------------------------------- */
/* GFD fits (Sec. 2.1, Taylor expansion and the system A x = b).             */
/* Coordinates are centred on the particle and divided by the stencil radius  */
/* s; the solution is unscaled afterwards (an exact reparametrisation).       */
/* ------------------------------------------------------------------------- */

static void second_order_row(int dim, const double *xi, double *row)
{
    for (int a = 0; a < dim; ++a) row[a] = xi[a];
    for (int a = 0; a < dim; ++a) row[dim + a] = 0.5 * xi[a] * xi[a];
    if (dim == 2) row[4] = xi[0] * xi[1];
    else { row[6] = xi[0] * xi[1]; row[7] = xi[0] * xi[2]; row[8] = xi[1] * xi[2]; }
}

/* Third-order row: the second-order row followed by the cubic Taylor terms
 * xi^alpha / alpha! (|alpha| = 3) in the order
 *   3D: xxx, yyy, zzz, xxy, xxz, xyy, yyz, xzz, yzz, xyz
 *   2D: xxx, yyy, xxy, xyy
 * (xyy is d3f / dx dy dy with the term xi_x xi_y^2 / 2). */
static void third_order_row(int dim, const double *xi, double *row)
{
    second_order_row(dim, xi, row);
    int o = nfit2(dim);
    double x = xi[0], y = xi[1];
    if (dim == 2) {
        row[o + 0] = x * x * x / 6.0;
        row[o + 1] = y * y * y / 6.0;
        row[o + 2] = 0.5 * x * x * y;
        row[o + 3] = 0.5 * x * y * y;
    } else {
        double z = xi[2];
        row[o + 0] = x * x * x / 6.0;
        row[o + 1] = y * y * y / 6.0;
        row[o + 2] = z * z * z / 6.0;
        row[o + 3] = 0.5 * x * x * y;
        row[o + 4] = 0.5 * x * x * z;
        row[o + 5] = 0.5 * x * y * y;
        row[o + 6] = 0.5 * y * y * z;
        row[o + 7] = 0.5 * x * z * z;
        row[o + 8] = 0.5 * y * z * z;
        row[o + 9] = x * y * z;
    }
}

/* Column index of the mixed second derivative d2/dx_a dx_b (a != b) */
static int mixed_col(int dim, int a, int b)
{
    if (a > b) { int t = a; a = b; b = t; }
    if (dim == 2) return 4;
    if (a == 0 && b == 1) return 6;
    if (a == 0 && b == 2) return 7;
    return 8;
}

/* ------------------------------------------------------------------------- */
/* Rates (Sec. 2.1).                                                          */
/* ------------------------------------------------------------------------- */

/* grad[f*3 + a]: d f / d x_a ; hess[f*6 + c]: second derivatives in column
 * order (11, 22, [33,] then mixed 12 [, 13, 23]) shifted by -dim, i.e.
 * hess[f*6 + (col - dim)].  Fields f: 0 = V, 1..dim = u, dim+1 = P. */
static double H(int dim, const double *hess, int f, int a, int b)
{
    int col = (a == b) ? dim + a : mixed_col(dim, a, b);
    return hess[f * 6 + (col - dim)];
}

void lpo_lw_rates(int dim, double gamma, double dt, const double *st /* V,u..,P */,
                  const double *grad, const double *hess, double *rate /* V,u..,P */)
{
    double V = st[0], P = st[dim + 1];
    int fP = dim + 1;
    double theta = 0.0, T = 0.0, gVgP = 0.0, lapP = 0.0;
    for (int a = 0; a < dim; ++a) theta += grad[(1 + a) * 3 + a];
    for (int i = 0; i < dim; ++i)
        for (int k = 0; k < dim; ++k) T += grad[(1 + k) * 3 + i] * grad[(1 + i) * 3 + k];
    for (int a = 0; a < dim; ++a) gVgP += grad[0 * 3 + a] * grad[fP * 3 + a];
    for (int a = 0; a < dim; ++a) lapP += H(dim, hess, fP, a, a);
    /* first material derivatives: mass, momentum and energy equations */
    double Vt = V * theta;
    double Pt = -gamma * P * theta;
    /* second material derivatives (Cauchy-Kowalevski, multi-D) */
    double Vtt = V * theta * theta - V * gVgP - V * V * lapP - V * T;
    double Ptt = gamma * gamma * P * theta * theta + gamma * P * gVgP + gamma * V * P * lapP + gamma * P * T;
    rate[0] = Vt + 0.5 * dt * Vtt;
    rate[fP] = Pt + 0.5 * dt * Ptt;
    for (int i = 0; i < dim; ++i) {
        double dPi = grad[fP * 3 + i];
        double dtheta_i = 0.0, uxP = 0.0;
        for (int k = 0; k < dim; ++k) {
            dtheta_i += H(dim, hess, 1 + k, i, k);
            uxP += grad[(1 + k) * 3 + i] * grad[fP * 3 + k];
        }
        double ut = -V * dPi;
        double utt = (gamma - 1.0) * V * theta * dPi + gamma * V * P * dtheta_i + V * uxP;
        rate[1 + i] = ut + 0.5 * dt * utt;
    }
}

/* one-sided derivatives along each axis a: dl/dr[a*3 + q], q = 0 (V), 1 (u_a), 2 (P) */
void lpo_uw_rates(int dim, double gamma, const double *st, const double *dl, const double *dr,
                  double *rate)
{
    double V = st[0], P = st[dim + 1];
    double c = sqrt(gamma * P * V);  /* V sqrt(K) with K = gamma P / V */
    double Vr = 0.0, Pr = 0.0;
    for (int a = 0; a < dim; ++a) {
        double ul = dl[a * 3 + 1], ur = dr[a * 3 + 1];
        double Pl = dl[a * 3 + 2], Prr = dr[a * 3 + 2];
        Vr += 0.5 * V * (ur + ul) - 0.5 * (V * V / c) * (Prr - Pl);
        rate[1 + a] = 0.5 * c * (ur - ul) - 0.5 * V * (Prr + Pl);
        Pr += -0.5 * gamma * P * (ur + ul) + 0.5 * c * (Prr - Pl);
    }
    rate[0] = Vr;
    rate[dim + 1] = Pr;
}

/* ------------------------------------------------------------------------- */
/* One particle: stencils, fits, estimator, blended update (Sec. 2.2 steps   */
/* 4-5 and Sec. 2.1).                                                        */
/* ------------------------------------------------------------------------- */

typedef struct {
    double grad[ORC_MAXF * 3];
    double hess[ORC_MAXF * 6];
    double dl[9], dr[9];       /* one-sided derivatives per axis (V, u_a, P) */
    int valid_l[3], valid_r[3];
    int lw_degenerate, vacuum_used, substituted, insufficient;
    double phi;
    double rate[ORC_MAXF];
    double vmin, vmax, pmin, pmax; /* V and P over the particle and its half-ball members */
} particle_result;

/* Fit the LW (second-order) polynomial for all fields over the selected rows.
 * Returns 0 = quadratic fit, 1 = degenerate -> linear fit, 2 = insufficient. */
static int lw_fit(const lpo_cfg *c, int k, const int *sel, const double *dxs, double s,
                  int nf, const double *fi, const double *fj /* k x nf, list order */,
                  double *grad, double *hess)
{
    int D = c->dim, n = nfit2(D);
    memset(grad, 0, sizeof(double) * (size_t)nf * 3);
    memset(hess, 0, sizeof(double) * (size_t)nf * 6);
    double *A = (double *)malloc(sizeof(double) * (size_t)(k > 0 ? k : 1) * ORC_MAXN);
    double *B = (double *)malloc(sizeof(double) * (size_t)(k > 0 ? k : 1) * ORC_MAXF);
    double X[ORC_MAXN * ORC_MAXF];
    int status = 0;
    double cond = INFINITY;
    if (k >= n) {
        for (int t = 0; t < k; ++t) {
            double xi[3] = {0.0, 0.0, 0.0};
            for (int a = 0; a < D; ++a) xi[a] = dxs[sel[t] * 3 + a] / s;
            second_order_row(D, xi, A + (size_t)t * n);
            for (int f = 0; f < nf; ++f) B[t * nf + f] = fj[sel[t] * nf + f] - fi[f];
        }
        cond = lpo_lstsq_qrp(k, n, nf, A, B, X);
    }
    if (k >= n && cond <= c->cond_max) {
        for (int f = 0; f < nf; ++f) {
            for (int a = 0; a < D; ++a) grad[f * 3 + a] = X[a * nf + f] / s;
            for (int q = 0; q < nsecond(D); ++q) hess[f * 6 + q] = X[(D + q) * nf + f] / (s * s);
        }
    } else {
        status = 1;
        if (k >= D) {
            for (int t = 0; t < k; ++t) {
                for (int a = 0; a < D; ++a) A[t * D + a] = dxs[sel[t] * 3 + a] / s;
                for (int f = 0; f < nf; ++f) B[t * nf + f] = fj[sel[t] * nf + f] - fi[f];
            }
            cond = lpo_lstsq_qrp(k, D, nf, A, B, X);
        } else cond = INFINITY;
        if (k >= D && cond <= c->cond_max) {
            for (int f = 0; f < nf; ++f)
                for (int a = 0; a < D; ++a) grad[f * 3 + a] = X[a * nf + f] / s;
        } else status = 2;
    }
    free(A); free(B);
    return status;
}

/* Linear one-sided fit of (V, u_a, P) on a half-ball's rows sel[].  Returns
 * 1 if valid and writes d[3]. */
static int uw_fit(const lpo_cfg *c, int m, const int *sel, const double *dxs, double s, int a,
                  const double *fi3, const double *fj3 /* k x 3 */, double *d)
{
    int D = c->dim;
    if (m < D) return 0;
    double A[64 * 3], B[64 * 3], X[9];
    for (int t = 0; t < m; ++t) {
        for (int b = 0; b < D; ++b) A[t * D + b] = dxs[sel[t] * 3 + b] / s;
        for (int q = 0; q < 3; ++q) B[t * 3 + q] = fj3[sel[t] * 3 + q] - fi3[q];
    }
    double cond = lpo_lstsq_qrp(m, D, 3, A, B, X);
    if (!(cond <= c->uw_cond_max)) return 0;
    for (int q = 0; q < 3; ++q) d[q] = X[a * 3 + q] / s;
    return 1;
}

/* Half-ball completed by vacuum ghosts: the m real members of the half-ball
 * and the mirror images, through the particle along axis a, of the mo members
 * of the opposite half-ball, which carry P = 0 and the particle's own V and u
 * (right-hand sides 0, 0, -P_i).  Returns 1 if valid and writes d[3]. */
static int uw_fit_completed(const lpo_cfg *c, int m, const int *sel, int mo, const int *selo, const double *dxs,
                            double s, int a, const double *fi3, const double *fj3, double Pi, double *d)
{
    int D = c->dim, rows = m + mo;
    if (rows < D) return 0;
    double A[128 * 3], B[128 * 3], X[9];
    for (int t = 0; t < rows; ++t) {
        int own = t < m;
        int j = own ? sel[t] : selo[t - m];
        for (int b = 0; b < D; ++b) {
            double v = dxs[j * 3 + b] / s;
            if (!own && b == a) v = -v;
            A[t * D + b] = v;
        }
        for (int q = 0; q < 3; ++q) B[t * 3 + q] = own ? fj3[j * 3 + q] - fi3[q] : (q == 2 ? -Pi : 0.0);
    }
    double cond = lpo_lstsq_qrp(rows, D, 3, A, B, X);
    if (!(cond <= c->uw_cond_max)) return 0;
    for (int q = 0; q < 3; ++q) d[q] = X[a * 3 + q] / s;
    return 1;
}

static void solve_particle(const lpo_cfg *c, int64_t i, const int32_t *list, int k,
                           const double *const X[3], const double *V, const double *const U[3],
                           const double *P, double h, double s, particle_result *res)
{
    int D = c->dim, nf = D + 2;
    memset(res, 0, sizeof(*res));
    double *dxs = (double *)malloc(sizeof(double) * 3 * (size_t)(k > 0 ? k : 1));
    double *fj = (double *)malloc(sizeof(double) * (size_t)nf * (size_t)(k > 0 ? k : 1));
    double *fj3 = (double *)malloc(sizeof(double) * 3 * (size_t)(k > 0 ? k : 1));
    int *sel = (int *)malloc(sizeof(int) * (size_t)(k > 0 ? k : 1));
    double fi[ORC_MAXF];
    fi[0] = V[i];
    for (int a = 0; a < D; ++a) fi[1 + a] = U[a][i];
    fi[D + 1] = P[i];
    for (int t = 0; t < k; ++t) {
        int64_t j = list[t];
        double dx[3];
        dist2(c, X, i, j, dx);
        for (int a = 0; a < 3; ++a) dxs[t * 3 + a] = dx[a];
        fj[t * nf + 0] = V[j];
        for (int a = 0; a < D; ++a) fj[t * nf + 1 + a] = U[a][j];
        fj[t * nf + D + 1] = P[j];
    }
    /* Lax-Wendroff fit on the symmetric stencil */
    int cap = c->lw_cap > 0 ? c->lw_cap : (D == 3 ? 54 : 32);
    int m = lw_select(D, k, dxs, cap, sel);
    int st = lw_fit(c, m, sel, dxs, s, nf, fi, fj, res->grad, res->hess);
    res->lw_degenerate = st != 0;
    res->insufficient = st == 2;
    /* upwind one-sided fits on half-balls */
    res->vmin = res->vmax = fi[0];
    res->pmin = res->pmax = fi[D + 1];
    int uwcap = c->uw_cap > 0 ? c->uw_cap : 8;
    int *self = (int *)malloc(sizeof(int) * (size_t)(uwcap > 0 ? uwcap : 1));
    int *selo = (int *)malloc(sizeof(int) * (size_t)(uwcap > 0 ? uwcap : 1));
    for (int a = 0; a < D; ++a) {
        double fi3[3] = {fi[0], fi[1 + a], fi[D + 1]};
        for (int t = 0; t < k; ++t) {
            fj3[t * 3 + 0] = fj[t * nf + 0];
            fj3[t * 3 + 1] = fj[t * nf + 1 + a];
            fj3[t * 3 + 2] = fj[t * nf + D + 1];
        }
        for (int side = 0; side < 2; ++side) {
            int sgn = side == 0 ? -1 : 1;
            double *d = side == 0 ? res->dl + a * 3 : res->dr + a * 3;
            int *valid = side == 0 ? &res->valid_l[a] : &res->valid_r[a];
            int ms = uw_select(k, dxs, a, sgn, uwcap, self);
            for (int t = 0; t < ms; ++t) {
                double vj = fj[self[t] * nf + 0], pj = fj[self[t] * nf + D + 1];
                if (vj < res->vmin) res->vmin = vj;
                if (vj > res->vmax) res->vmax = vj;
                if (pj < res->pmin) res->pmin = pj;
                if (pj > res->pmax) res->pmax = pj;
            }
            int ok = 0;
            if (c->vacuum && ms < uwcap) {
                /* free boundary (step 3): the direction holds fewer members
                 * than its list needs, so ghost particles complete it: the
                 * mirror images of the opposite half-ball's members, with
                 * P = 0 (vacuum) and the particle's own V and u, join the
                 * half-ball's real members in the fit */
                int mo = uw_select(k, dxs, a, -sgn, uwcap, selo);
                if (uw_fit_completed(c, ms, self, mo, selo, dxs, s, a, fi3, fj3, fi[D + 1], d)) {
                    res->vacuum_used = 1;
                    ok = 1;
                }
            } else {
                ok = uw_fit(c, ms, self, dxs, s, a, fi3, fj3, d);
                *valid = ok;
            }
            if (!ok) {
                d[0] = res->grad[0 * 3 + a];
                d[1] = res->grad[(1 + a) * 3 + a];
                d[2] = res->grad[(D + 1) * 3 + a];
                res->substituted = 1;
            }
        }
    }
    free(self); free(selo);
    /* state estimator: quotient of left and right derivatives of P and V */
    double r = 1.0;
    for (int a = 0; a < D; ++a) {
        if (!(res->valid_l[a] && res->valid_r[a])) continue;
        for (int q = 0; q < 3; q += 2) {  /* q = 0: V, q = 2: P */
            double sl = res->dl[a * 3 + q], sr = res->dr[a * 3 + q];
            double sv = q == 0 ? fi[0] : fi[D + 1];
            double big = fabs(sl) > fabs(sr) ? fabs(sl) : fabs(sr);
            if (big * h > c->est_eps * fabs(sv)) {
                double rr = lpo_estimator_ratio(sl, sr);
                if (rr > r) r = rr;
            }
        }
    }
    /* phi = limiter(r); with a cap (the default 1) the points the estimator
     * does not select advance with the pure Lax-Wendroff rate, without one the
     * printed limiter reaches 1.25 at r = 1 */
    double ph = lpo_limiter(r);
    res->phi = (c->limiter_cap > 0.0 && ph > c->limiter_cap) ? c->limiter_cap : ph;
    if (res->lw_degenerate || res->vacuum_used) res->phi = 0.0;
    /* a fixed phi isolates one side of the blend (Sec. 2.1) */
    if (c->phi_fixed >= 0.0) res->phi = c->phi_fixed;
    free(dxs); free(fj); free(fj3); free(sel);
}

/* ------------------------------------------------------------------------- */
/* Inputs of the learned state estimator.  The paper's estimator looks only   */
/* at the quotient of left and right one-sided derivatives; the network that  */
/* may stand in for it sees that quotient per field and axis together with    */
/* the local gradients it comes from.  All inputs are dimensionless.          */
/* ------------------------------------------------------------------------- */

/* Disagreement of the two one-sided slopes of a field along one axis: |log| of
 * their quotient, capped at 8, and 8 when they differ in sign; 0 where the
 * estimator ignores the pair (a side without a usable fit, or both slopes
 * below the activity threshold). */
static double slope_disagreement(const lpo_cfg *c, double sl, double sr, double s, double h, int valid)
{
    if (!valid) return 0.0;
    double big = fabs(sl) > fabs(sr) ? fabs(sl) : fabs(sr);
    if (!(big * h > c->est_eps * fabs(s))) return 0.0;
    if (!(sl * sr > 0.0)) return 8.0;
    double q = fabs(log(fabs(sr) / fabs(sl)));
    return q < 8.0 ? q : 8.0;
}

/* feat[0..2]  h d_a(rho) / rho = -h d_a V / V
 * feat[3..5]  h d_a P / P
 * feat[6]     h div u / c,  c = sqrt(gamma P V)
 * feat[7..9]  slope disagreement of V along each axis (that of rho is the same)
 * feat[10..12] slope disagreement of P along each axis
 * feat[13]    log(V_max / V_min) and feat[14] log(P_max / P_min) over the
 *             particle and its half-ball members
 * feat[15]    h |grad u|_F / c
 * Axes beyond the dimension give 0. */
static void particle_features(const lpo_cfg *c, const double *fi, const particle_result *res, double h,
                              double *feat)
{
    int D = c->dim;
    double V = fi[0], P = fi[D + 1];
    double cs = sqrt(c->gamma * P * V);
    double div = 0.0, gu2 = 0.0;
    for (int q = 0; q < 16; ++q) feat[q] = 0.0;
    for (int a = 0; a < D; ++a) {
        feat[a] = -h * res->grad[0 * 3 + a] / V;
        feat[3 + a] = h * res->grad[(D + 1) * 3 + a] / P;
        div += res->grad[(1 + a) * 3 + a];
        for (int b = 0; b < D; ++b) gu2 += res->grad[(1 + a) * 3 + b] * res->grad[(1 + a) * 3 + b];
        int valid = res->valid_l[a] && res->valid_r[a];
        feat[7 + a] = slope_disagreement(c, res->dl[a * 3 + 0], res->dr[a * 3 + 0], V, h, valid);
        feat[10 + a] = slope_disagreement(c, res->dl[a * 3 + 2], res->dr[a * 3 + 2], P, h, valid);
    }
    feat[6] = h * div / cs;
    feat[13] = log(res->vmax / res->vmin);
    feat[14] = log(res->pmax / res->pmin);
    feat[15] = h * sqrt(gu2) / cs;
}

/* ------------------------------------------------------------------------- */
/* The estimator network: 16 -> 64 (ReLU) -> 64 (ReLU) -> 1, output           */
/* y = 1 / (1 + exp(-z)).  Parameters packed as W1[64][16], b1[64],           */
/* W2[64][64], b2[64], w3[64], b3.  Loss: mean binary cross-entropy of y      */
/* against targets t in [0, 1].                                               */
/* ------------------------------------------------------------------------- */

#define MLP_IN 16
#define MLP_H 64
#define OFF_W1 0
#define OFF_B1 (OFF_W1 + MLP_H * MLP_IN)
#define OFF_W2 (OFF_B1 + MLP_H)
#define OFF_B2 (OFF_W2 + MLP_H * MLP_H)
#define OFF_W3 (OFF_B2 + MLP_H)
#define OFF_B3 (OFF_W3 + MLP_H)

static double mlp_one(const double *th, const double *x, double *a1, double *h1, double *a2, double *h2)
{
    for (int o = 0; o < MLP_H; ++o) {
        double s = th[OFF_B1 + o];
        for (int f = 0; f < MLP_IN; ++f) s += th[OFF_W1 + o * MLP_IN + f] * x[f];
        a1[o] = s;
        h1[o] = s > 0.0 ? s : 0.0;
    }
    for (int o = 0; o < MLP_H; ++o) {
        double s = th[OFF_B2 + o];
        for (int q = 0; q < MLP_H; ++q) s += th[OFF_W2 + o * MLP_H + q] * h1[q];
        a2[o] = s;
        h2[o] = s > 0.0 ? s : 0.0;
    }
    double z = th[OFF_B3];
    for (int o = 0; o < MLP_H; ++o) z += th[OFF_W3 + o] * h2[o];
    return z;
}

void lpo_mlp_forward(const double *theta, int64_t n, const double *feat, double *z, double *y)
{
#pragma omp parallel for schedule(static)
    for (int64_t i = 0; i < n; ++i) {
        double a1[MLP_H], h1[MLP_H], a2[MLP_H], h2[MLP_H];
        double zi = mlp_one(theta, feat + i * MLP_IN, a1, h1, a2, h2);
        if (z) z[i] = zi;
        if (y) y[i] = 1.0 / (1.0 + exp(-zi));
    }
}

/* Mean loss over n samples; grad (LPO_MLP_NPARAM entries) receives its
 * gradient by back-propagation through the three layers. */
double lpo_mlp_loss_grad(const double *theta, int64_t n, const double *feat, const double *target, double *grad)
{
    for (int q = 0; q < LPO_MLP_NPARAM; ++q) grad[q] = 0.0;
    double loss = 0.0;
    for (int64_t i = 0; i < n; ++i) {
        const double *x = feat + i * MLP_IN;
        double a1[MLP_H], h1[MLP_H], a2[MLP_H], h2[MLP_H];
        double z = mlp_one(theta, x, a1, h1, a2, h2);
        double t = target[i];
        /* -t log y - (1 - t) log(1 - y) = softplus(z) - t z */
        double sp = (z > 0.0 ? z : 0.0) + log1p(exp(-fabs(z)));
        loss += sp - t * z;
        double dz = (1.0 / (1.0 + exp(-z)) - t) / (double)n;
        grad[OFF_B3] += dz;
        double d2[MLP_H], d1[MLP_H];
        for (int o = 0; o < MLP_H; ++o) {
            grad[OFF_W3 + o] += dz * h2[o];
            d2[o] = a2[o] > 0.0 ? dz * theta[OFF_W3 + o] : 0.0;
            grad[OFF_B2 + o] += d2[o];
        }
        for (int q = 0; q < MLP_H; ++q) {
            double s = 0.0;
            for (int o = 0; o < MLP_H; ++o) {
                grad[OFF_W2 + o * MLP_H + q] += d2[o] * h1[q];
                s += theta[OFF_W2 + o * MLP_H + q] * d2[o];
            }
            d1[q] = a1[q] > 0.0 ? s : 0.0;
            grad[OFF_B1 + q] += d1[q];
        }
        for (int o = 0; o < MLP_H; ++o)
            for (int f = 0; f < MLP_IN; ++f) grad[OFF_W1 + o * MLP_IN + f] += d1[o] * x[f];
    }
    return loss / (double)n;
}

/* ------------------------------------------------------------------------- */
/* Derivative operator alone: lp_gfd's definition.                            */
/* ------------------------------------------------------------------------- */

int lpo_gfd(const lpo_cfg *c, int64_t n, const double *x, const double *y, const double *z,
            const double *r, int32_t nf, const double *const *f, double *deriv, uint8_t *status)
{
    int D = c->dim, nu = nfit2(D);
    const double *X[3] = {x, y, z ? z : x};
    int cap = c->max_nb;
    int32_t *count = (int32_t *)malloc(sizeof(int32_t) * (size_t)(n > 0 ? n : 1));
    int32_t *lists = (int32_t *)malloc(sizeof(int32_t) * (size_t)(n > 0 ? n : 1) * (size_t)cap);
    int64_t *q = (int64_t *)malloc(sizeof(int64_t) * (size_t)(n > 0 ? n : 1));
    if (!count || !lists || !q) { free(count); free(lists); free(q); return LPO_E_NOMEM; }
    for (int64_t i = 0; i < n; ++i) q[i] = i;
    int st = neighbor_lists(c, n, q, n, X, r, cap, count, lists);
    if (st == LPO_OK) {
#pragma omp parallel for schedule(dynamic, 16)
        for (int64_t i = 0; i < n; ++i) {
            int k = count[i];
            double *dxs = (double *)malloc(sizeof(double) * 3 * (size_t)(k > 0 ? k : 1));
            double *fj = (double *)malloc(sizeof(double) * (size_t)nf * (size_t)(k > 0 ? k : 1));
            double *fi = (double *)malloc(sizeof(double) * (size_t)nf);
            int *sel = (int *)malloc(sizeof(int) * (size_t)(k > 0 ? k : 1));
            double *grad = (double *)malloc(sizeof(double) * (size_t)nf * 3);
            double *hess = (double *)malloc(sizeof(double) * (size_t)nf * 6);
            for (int ff = 0; ff < nf; ++ff) fi[ff] = f[ff][i];
            for (int t = 0; t < k; ++t) {
                int64_t j = lists[(size_t)i * (size_t)cap + t];
                double dx[3];
                dist2(c, X, i, j, dx);
                for (int a = 0; a < 3; ++a) dxs[t * 3 + a] = dx[a];
                for (int ff = 0; ff < nf; ++ff) fj[t * nf + ff] = f[ff][j];
            }
            int lcap = c->lw_cap > 0 ? c->lw_cap : (D == 3 ? 54 : 32);
            int m = lw_select(D, k, dxs, lcap, sel);
            int s = nf <= ORC_MAXF ? lw_fit(c, m, sel, dxs, r[i], nf, fi, fj, grad, hess) : 2;
            status[i] = (uint8_t)s;
            for (int ff = 0; ff < nf; ++ff) {
                for (int a = 0; a < D; ++a) deriv[((size_t)ff * nu + a) * (size_t)n + i] = grad[ff * 3 + a];
                for (int qq = 0; qq < nsecond(D); ++qq)
                    deriv[((size_t)ff * nu + D + qq) * (size_t)n + i] = hess[ff * 6 + qq];
            }
            free(dxs); free(fj); free(fi); free(sel); free(grad); free(hess);
        }
    }
    free(count); free(lists); free(q);
    return st;
}

/* ------------------------------------------------------------------------- */
/* Third-order derivative operator: lp_gfd3's definition (Sec. 2.1: the GFD   */
/* system is the Taylor expansion truncated at second order; the same         */
/* construction one order further).                                           */
/* ------------------------------------------------------------------------- */

/* Fit over the selected rows; out[f * nu3 + col].  Returns 0 = cubic fit,
 * 1 = cubic deficient (fewer rows than unknowns or |R11|/|Rnn| > cond_max)
 * -> the second-order fit on the same rows, 2 = that one deficient too ->
 * linear fit, 3 = nothing usable (all 0). */
static int gfd3_fit(const lpo_cfg *c, int m, const int *sel, const double *dxs, double s, int nf,
                    const double *fi, const double *fj, double *out)
{
    int D = c->dim, n = nfit3(D), n2 = nfit2(D);
    memset(out, 0, sizeof(double) * (size_t)nf * (size_t)n);
    if (m >= n) {
        double *A = (double *)malloc(sizeof(double) * (size_t)m * ORC_MAXN3);
        double *B = (double *)malloc(sizeof(double) * (size_t)m * ORC_MAXF);
        double X[ORC_MAXN3 * ORC_MAXF];
        for (int t = 0; t < m; ++t) {
            double xi[3] = {0.0, 0.0, 0.0};
            for (int a = 0; a < D; ++a) xi[a] = dxs[sel[t] * 3 + a] / s;
            third_order_row(D, xi, A + (size_t)t * n);
            for (int f = 0; f < nf; ++f) B[t * nf + f] = fj[sel[t] * nf + f] - fi[f];
        }
        double cond = lpo_lstsq_qrp(m, n, nf, A, B, X);
        free(A); free(B);
        if (cond <= c->cond_max) {
            /* unscale: a column of degree p carries the derivative times s^p */
            for (int f = 0; f < nf; ++f)
                for (int q = 0; q < n; ++q) {
                    double sp = q < D ? s : (q < n2 ? s * s : s * s * s);
                    out[f * n + q] = X[q * nf + f] / sp;
                }
            return 0;
        }
    }
    double grad[ORC_MAXF * 3], hess[ORC_MAXF * 6];
    int st2 = lw_fit(c, m, sel, dxs, s, nf, fi, fj, grad, hess);
    for (int f = 0; f < nf; ++f) {
        for (int a = 0; a < D; ++a) out[f * n + a] = grad[f * 3 + a];
        for (int q = 0; q < nsecond(D); ++q) out[f * n + D + q] = hess[f * 6 + q];
    }
    return 1 + st2;
}

int lpo_gfd3(const lpo_cfg *c, int64_t n, const double *x, const double *y, const double *z,
             const double *r, int32_t nf, const double *const *f, double *deriv, uint8_t *status)
{
    int D = c->dim, nu = nfit3(D);
    if (nf < 1 || nf > ORC_MAXF) return LPO_E_ARG;
    const double *X[3] = {x, y, z ? z : x};
    int cap = c->max_nb;
    int32_t *count = (int32_t *)malloc(sizeof(int32_t) * (size_t)(n > 0 ? n : 1));
    int32_t *lists = (int32_t *)malloc(sizeof(int32_t) * (size_t)(n > 0 ? n : 1) * (size_t)cap);
    int64_t *q = (int64_t *)malloc(sizeof(int64_t) * (size_t)(n > 0 ? n : 1));
    if (!count || !lists || !q) { free(count); free(lists); free(q); return LPO_E_NOMEM; }
    for (int64_t i = 0; i < n; ++i) q[i] = i;
    int st = neighbor_lists(c, n, q, n, X, r, cap, count, lists);
    if (st == LPO_OK) {
#pragma omp parallel for schedule(dynamic, 16)
        for (int64_t i = 0; i < n; ++i) {
            int k = count[i];
            double *dxs = (double *)malloc(sizeof(double) * 3 * (size_t)(k > 0 ? k : 1));
            double *fj = (double *)malloc(sizeof(double) * (size_t)nf * (size_t)(k > 0 ? k : 1));
            int *sel = (int *)malloc(sizeof(int) * (size_t)(k > 0 ? k : 1));
            double fi[ORC_MAXF], out[ORC_MAXF * ORC_MAXN3];
            for (int ff = 0; ff < nf; ++ff) fi[ff] = f[ff][i];
            for (int t = 0; t < k; ++t) {
                int64_t j = lists[(size_t)i * (size_t)cap + t];
                double dx[3];
                dist2(c, X, i, j, dx);
                for (int a = 0; a < 3; ++a) dxs[t * 3 + a] = dx[a];
                for (int ff = 0; ff < nf; ++ff) fj[t * nf + ff] = f[ff][j];
            }
            int lcap = c->lw_cap > 0 ? c->lw_cap : (D == 3 ? 54 : 32);
            int m = lw_select(D, k, dxs, lcap, sel);
            status[i] = (uint8_t)gfd3_fit(c, m, sel, dxs, r[i], nf, fi, fj, out);
            for (int ff = 0; ff < nf; ++ff)
                for (int qq = 0; qq < nu; ++qq) deriv[((size_t)ff * nu + qq) * (size_t)n + i] = out[ff * nu + qq];
            free(dxs); free(fj); free(sel);
        }
    }
    free(count); free(lists); free(q);
    return st;
}

/* ------------------------------------------------------------------------- */
/* Open boundaries (Sec. 2.2, step 1: outflow by deleting particles, inflow   */
/* by generating them; Sec. 3.2: the state of particles entering from a       */
/* reservoir).                                                                */
/* ------------------------------------------------------------------------- */

/* Delete, in place, every particle past an outflow face: x_a < lo_a for a
 * bit a of lo_mask, x_a >= hi_a for a bit a of hi_mask.  The others keep their
 * order.  arrays[0..narr-1] are the per-particle FP64 arrays to compact. */
int lpo_outflow(const lpo_cfg *c, int64_t n, double *const *arrays, int narr, const double *const *x,
                uint32_t lo_mask, uint32_t hi_mask, int64_t *n_kept)
{
    int D = c->dim;
    int64_t k = 0;
    char *keep = (char *)malloc((size_t)(n > 0 ? n : 1));
    if (!keep) return LPO_E_NOMEM;
    for (int64_t i = 0; i < n; ++i) {
        int gone = 0;
        for (int a = 0; a < D; ++a) {
            if (((lo_mask >> a) & 1u) && x[a][i] < c->lo[a]) gone = 1;
            if (((hi_mask >> a) & 1u) && x[a][i] >= c->hi[a]) gone = 1;
        }
        keep[i] = (char)!gone;
    }
    for (int64_t i = 0; i < n; ++i) {
        if (!keep[i]) continue;
        for (int q = 0; q < narr; ++q) arrays[q][k] = arrays[q][i];
        ++k;
    }
    free(keep);
    *n_kept = k;
    return LPO_OK;
}

/* State of the particles entering through the face of axis `axis` (side 0:
 * box_lo, 1: box_hi) from a reservoir at rest with pressure p_res and
 * density rho_res:
 *   P_in   = mean pressure of the particles with distance 0 <= d < width
 *            from the face inside the box (p_res when there are none);
 *   rho_in from equal entropy, P_res / rho_res^gamma = P_in / rho_in^gamma;
 *   u_in   from equal enthalpy with the reservoir at rest,
 *            u_in^2 / 2 + c_in^2 / (gamma - 1) = c_res^2 / (gamma - 1),
 *            c^2 = gamma P / rho (0 when the right side is negative).
 * out[0] = P_in, out[1] = rho_in, out[2] = u_in, out[3] = particles averaged. */
int lpo_reservoir_inflow(const lpo_cfg *c, int64_t n, const double *const *x, const double *P, int axis, int side,
                         double width, double p_res, double rho_res, double *out)
{
    if (axis < 0 || axis >= c->dim || side < 0 || side > 1 || !(width > 0.0) || !(p_res > 0.0) ||
        !(rho_res > 0.0))
        return LPO_E_ARG;
    double sum = 0.0;
    int64_t cnt = 0;
    for (int64_t i = 0; i < n; ++i) {
        double d = side == 0 ? x[axis][i] - c->lo[axis] : c->hi[axis] - x[axis][i];
        if (d >= 0.0 && d < width) { sum += P[i]; ++cnt; }
    }
    double g = c->gamma;
    double p_in = cnt > 0 ? sum / (double)cnt : p_res;
    double rho_in = rho_res * pow(p_in / p_res, 1.0 / g);
    double c2_res = g * p_res / rho_res, c2_in = g * p_in / rho_in;
    double u2 = 2.0 * (c2_res - c2_in) / (g - 1.0);
    out[0] = p_in;
    out[1] = rho_in;
    out[2] = u2 > 0.0 ? sqrt(u2) : 0.0;
    out[3] = (double)cnt;
    return LPO_OK;
}

/* Inflow layer (Sec. 2.2, step 1: inflow boundaries generate particles):
 * particles on the square lattice of the given spacing over the face of axis
 * `axis` (side 0: lo, 1: hi), at distance `depth` inside it.  The other axes
 * b take box_lo[b] + (k + 1/2) spacing, k = 0 .. floor(extent_b / spacing + 1e-9) - 1
 * (a cell short of a whole one by rounding alone still counts),
 * the first other axis fastest.  State: V = 1/rho, pressure P, velocity u_n
 * along the inward normal, mass rho spacing^dim.  Writes entries n .. n +
 * count - 1 of the arrays (x[D], u[D], V, P, m) when n + count <= cap. */
int lpo_inflow_layer(const lpo_cfg *c, int64_t n, int64_t cap, double *const *x, double *const *u, double *V,
                     double *P, double *m, int axis, int side, double spacing, double depth, double rho,
                     double p_in, double u_n, int64_t *n_new)
{
    int D = c->dim;
    if (axis < 0 || axis >= D || side < 0 || side > 1 || !(spacing > 0.0) || !(depth >= 0.0) || !(rho > 0.0))
        return LPO_E_ARG;
    int other[2] = {0, 0}, no = 0;
    for (int b = 0; b < D; ++b)
        if (b != axis) other[no++] = b;
    int64_t cnt[2] = {1, 1};
    for (int q = 0; q < no; ++q) cnt[q] = (int64_t)floor((c->hi[other[q]] - c->lo[other[q]]) / spacing + 1e-9);
    int64_t count = cnt[0] * cnt[1];
    if (n + count > cap) return LPO_E_CAPACITY;
    double mass = rho;
    for (int a = 0; a < D; ++a) mass = mass * spacing;
    double xa = side == 0 ? c->lo[axis] + depth : c->hi[axis] - depth;
    double un = side == 0 ? u_n : -u_n;
    for (int64_t q = 0; q < count; ++q) {
        int64_t k[2] = {q % cnt[0], q / cnt[0]};
        int64_t i = n + q;
        for (int a = 0; a < D; ++a) u[a][i] = 0.0;
        x[axis][i] = xa;
        u[axis][i] = un;
        for (int t = 0; t < no; ++t) {
            double off = ((double)k[t] + 0.5) * spacing;
            x[other[t]][i] = c->lo[other[t]] + off;
        }
        V[i] = 1.0 / rho;
        P[i] = p_in;
        m[i] = mass;
    }
    *n_new = n + count;
    return LPO_OK;
}

/* ------------------------------------------------------------------------- */
/* Time step (Sec. 2.2, steps 1-6).                                           */
/* ------------------------------------------------------------------------- */

double lpo_timestep(const lpo_cfg *c, int64_t n, const double *V, const double *P, const double *m)
{
    double best = INFINITY;
    for (int64_t i = 0; i < n; ++i) {
        double h = smoothing_length(c->dim, m[i], V[i]);
        double cs = sqrt(c->gamma * P[i] * V[i]);
        double q = h / cs;
        if (q < best) best = q;
    }
    return c->cfl * best;
}

/* Mirror particles across solid walls (step 1): every particle closer than
 * r_max to a wall plane w gets an image at 2w - x with the normal velocity
 * reversed.  Ghost ids follow (source id, wall index) order. */
static int64_t mirror_ghosts(const lpo_cfg *c, int64_t n, const double *const X[3], double rmax,
                             int64_t *src, int *wall)
{
    int64_t g = 0;
    for (int64_t i = 0; i < n; ++i)
        for (int a = 0; a < c->dim; ++a) {
            if (c->wall_lo[a] && X[a][i] - c->lo[a] < rmax) { if (src) { src[g] = i; wall[g] = 2 * a; } ++g; }
            if (c->wall_hi[a] && c->hi[a] - X[a][i] < rmax) { if (src) { src[g] = i; wall[g] = 2 * a + 1; } ++g; }
        }
    return g;
}

int lpo_step_subset(const lpo_cfg *c, int64_t n, const double *x, const double *y, const double *z,
                    const double *V, const double *u, const double *v, const double *w,
                    const double *P, const double *m, double dt_in, int64_t nsub, const int64_t *sub,
                    double *ox, double *oy, double *oz, double *oV, double *ou, double *ov,
                    double *ow, double *oP, double *ophi, uint8_t *oflags, double *dt_used,
                    int64_t *n_ghost, double *ofeat)
{
    int D = c->dim;
    const double *X0[3] = {x, y, z ? z : x};
    const double *U0[3] = {u, v, w ? w : u};
    /* 1. time step from the CFL rule at t^n */
    double dt = dt_in > 0.0 ? dt_in : lpo_timestep(c, n, V, P, m);
    if (dt_used) *dt_used = dt;
    /* 2. radii r_i = kappa h_i */
    double *h = (double *)malloc(sizeof(double) * (size_t)n);
    double *r = (double *)malloc(sizeof(double) * (size_t)n);
    if (!h || !r) { free(h); free(r); return LPO_E_NOMEM; }
    double rmax = 0.0;
    for (int64_t i = 0; i < n; ++i) {
        h[i] = smoothing_length(D, m[i], V[i]);
        r[i] = c->kappa * h[i];
        if (r[i] > rmax) rmax = r[i];
    }
    /* 3. boundary particles */
    int64_t ng = mirror_ghosts(c, n, X0, rmax, NULL, NULL);
    if (n_ghost) *n_ghost = ng;
    int64_t nt = n + ng;
    double *ax[3], *au[3], *aV, *aP, *ar;
    for (int a = 0; a < 3; ++a) { ax[a] = (double *)malloc(sizeof(double) * (size_t)nt); au[a] = (double *)malloc(sizeof(double) * (size_t)nt); }
    aV = (double *)malloc(sizeof(double) * (size_t)nt);
    aP = (double *)malloc(sizeof(double) * (size_t)nt);
    ar = (double *)malloc(sizeof(double) * (size_t)nt);
    int64_t *src = (int64_t *)malloc(sizeof(int64_t) * (size_t)(ng > 0 ? ng : 1));
    int *wall = (int *)malloc(sizeof(int) * (size_t)(ng > 0 ? ng : 1));
    mirror_ghosts(c, n, X0, rmax, src, wall);
    for (int64_t i = 0; i < n; ++i) {
        for (int a = 0; a < 3; ++a) { ax[a][i] = a < D ? X0[a][i] : 0.0; au[a][i] = a < D ? U0[a][i] : 0.0; }
        aV[i] = V[i]; aP[i] = P[i]; ar[i] = r[i];
    }
    for (int64_t g = 0; g < ng; ++g) {
        int64_t i = src[g], j = n + g;
        int a = wall[g] / 2;
        double wpos = (wall[g] & 1) ? c->hi[a] : c->lo[a];
        for (int b = 0; b < 3; ++b) { ax[b][j] = ax[b][i]; au[b][j] = au[b][i]; }
        ax[a][j] = 2.0 * wpos - ax[a][i];
        au[a][j] = -au[a][i];
        aV[j] = V[i]; aP[j] = P[i]; ar[j] = r[i];
    }
    /* 4. neighbours of the requested particles over real + ghost particles */
    int cap = c->max_nb;
    int32_t *count = (int32_t *)malloc(sizeof(int32_t) * (size_t)(nsub > 0 ? nsub : 1));
    int32_t *lists = (int32_t *)malloc(sizeof(int32_t) * (size_t)(nsub > 0 ? nsub : 1) * (size_t)cap);
    const double *AX[3] = {ax[0], ax[1], ax[2]};
    const double *AU[3] = {au[0], au[1], au[2]};
    int st = neighbor_lists(c, nsub, sub, nt, AX, ar, cap, count, lists);
    if (st == LPO_OK) {
        int numeric_bad = 0;
#pragma omp parallel for schedule(dynamic, 16) reduction(| : numeric_bad)
        for (int64_t t = 0; t < nsub; ++t) {
            int64_t i = sub[t];
            particle_result res;
            /* 5. stencils, fits, estimator */
            solve_particle(c, i, lists + (size_t)t * (size_t)cap, count[t], AX, aV, AU, aP, h[i], r[i], &res);
            double stv[ORC_MAXF], lw[ORC_MAXF], uw[ORC_MAXF];
            stv[0] = aV[i];
            for (int a = 0; a < D; ++a) stv[1 + a] = AU[a][i];
            stv[D + 1] = aP[i];
            lpo_lw_rates(D, c->gamma, dt, stv, res.grad, res.hess, lw);
            lpo_uw_rates(D, c->gamma, stv, res.dl, res.dr, uw);
            /* blended update s^{n+1} = s^n + dt (UW - phi (UW - LW)) */
            double ns[ORC_MAXF];
            for (int f = 0; f < D + 2; ++f) ns[f] = stv[f] + dt * (uw[f] - res.phi * (uw[f] - lw[f]));
            /* 6. particle mover: x^{n+1} = x^n + dt/2 (u^n + u^{n+1}) */
            double nx[3] = {0.0, 0.0, 0.0};
            for (int a = 0; a < D; ++a) {
                double p = AX[a][i] + 0.5 * dt * (stv[1 + a] + ns[1 + a]);
                if (c->periodic[a]) {
                    double L = c->hi[a] - c->lo[a];
                    if (p >= c->hi[a]) p -= L;
                    else if (p < c->lo[a]) p += L;
                }
                nx[a] = p;
            }
            ox[t] = nx[0]; oy[t] = nx[1]; if (D == 3 && oz) oz[t] = nx[2];
            oV[t] = ns[0]; ou[t] = ns[1]; ov[t] = ns[2]; if (D == 3 && ow) ow[t] = ns[3];
            oP[t] = ns[D + 1];
            if (ophi) ophi[t] = res.phi;
            if (ofeat) particle_features(c, stv, &res, h[i], ofeat + (size_t)t * 16);
            uint8_t fl = 0;
            if (res.phi < 1.0) fl |= LPO_FLAG_LIMITED;
            if (res.lw_degenerate) fl |= LPO_FLAG_DEGENERATE;
            if (res.vacuum_used) fl |= LPO_FLAG_VACUUM;
            if (res.substituted) fl |= LPO_FLAG_SUBSTITUTED;
            if (!(ns[0] > 0.0) || !(ns[D + 1] > 0.0)) { fl |= LPO_FLAG_NUMERIC; numeric_bad = 1; }
            if (oflags) oflags[t] = fl;
        }
        if (numeric_bad) st = LPO_E_NUMERIC;
    }
    for (int a = 0; a < 3; ++a) { free(ax[a]); free(au[a]); }
    free(aV); free(aP); free(ar); free(src); free(wall); free(count); free(lists); free(h); free(r);
    return st;
}

int lpo_step(const lpo_cfg *c, int64_t n, double *x, double *y, double *z, double *V, double *u,
             double *v, double *w, double *P, const double *m, double dt_in, double *phi,
             uint8_t *flags, double *dt_used, int64_t *n_ghost)
{
    int D = c->dim;
    int64_t *sub = (int64_t *)malloc(sizeof(int64_t) * (size_t)(n > 0 ? n : 1));
    double *buf = (double *)malloc(sizeof(double) * (size_t)(n > 0 ? n : 1) * 8);
    if (!sub || !buf) { free(sub); free(buf); return LPO_E_NOMEM; }
    for (int64_t i = 0; i < n; ++i) sub[i] = i;
    double *o[8];
    for (int q = 0; q < 8; ++q) o[q] = buf + (size_t)q * (size_t)n;
    int st = lpo_step_subset(c, n, x, y, z, V, u, v, w, P, m, dt_in, n, sub, o[0], o[1], o[2], o[3],
                             o[4], o[5], o[6], o[7], phi, flags, dt_used, n_ghost, NULL);
    if (st == LPO_OK || st == LPO_E_NUMERIC) {
        memcpy(x, o[0], sizeof(double) * (size_t)n);
        memcpy(y, o[1], sizeof(double) * (size_t)n);
        if (D == 3 && z) memcpy(z, o[2], sizeof(double) * (size_t)n);
        memcpy(V, o[3], sizeof(double) * (size_t)n);
        memcpy(u, o[4], sizeof(double) * (size_t)n);
        memcpy(v, o[5], sizeof(double) * (size_t)n);
        if (D == 3 && w) memcpy(w, o[6], sizeof(double) * (size_t)n);
        memcpy(P, o[7], sizeof(double) * (size_t)n);
    }
    free(sub); free(buf);
    return st;
}

/* Total mass, momentum and energy, summed in id order (mass is carried by the
 * particles and is conserved exactly, Sec. 1). */
void lpo_conservation(const lpo_cfg *c, int64_t n, const double *V, const double *u, const double *v,
                      const double *w, const double *P, const double *m, double *out)
{
    int D = c->dim;
    double M = 0, px = 0, py = 0, pz = 0, E = 0;
    for (int64_t i = 0; i < n; ++i) {
        double ww = D == 3 ? w[i] : 0.0;
        double e = P[i] * V[i] / (c->gamma - 1.0);
        double ke = 0.5 * (u[i] * u[i] + v[i] * v[i] + ww * ww);
        M += m[i];
        px += m[i] * u[i];
        py += m[i] * v[i];
        pz += m[i] * ww;
        E += m[i] * (e + ke);
    }
    out[0] = M; out[1] = px; out[2] = py; out[3] = pz; out[4] = E;
}

/* Diagnostics for one particle, for the pins: LW derivatives, one-sided
 * derivatives, validity and phi, given an explicit neighbour list. */
int lpo_particle_derivs(const lpo_cfg *c, int64_t n, const double *x, const double *y, const double *z,
                        const double *V, const double *u, const double *v, const double *w,
                        const double *P, int64_t i, const int32_t *list, int32_t k, double h, double s,
                        double *grad, double *hess, double *dl, double *dr, int32_t *valid, double *phi,
                        int32_t *flags)
{
    (void)n;
    const double *X[3] = {x, y, z ? z : x};
    const double *U[3] = {u, v, w ? w : u};
    particle_result res;
    solve_particle(c, i, list, k, X, V, U, P, h, s, &res);
    memcpy(grad, res.grad, sizeof(res.grad));
    memcpy(hess, res.hess, sizeof(res.hess));
    memcpy(dl, res.dl, sizeof(res.dl));
    memcpy(dr, res.dr, sizeof(res.dr));
    for (int a = 0; a < 3; ++a) { valid[2 * a] = res.valid_l[a]; valid[2 * a + 1] = res.valid_r[a]; }
    *phi = res.phi;
    *flags = (res.lw_degenerate ? LPO_FLAG_DEGENERATE : 0) | (res.vacuum_used ? LPO_FLAG_VACUUM : 0) |
             (res.substituted ? LPO_FLAG_SUBSTITUTED : 0);
    return LPO_OK;
}

int lpo_lw_select(int dim, int k, const double *dxs, int cap, int *sel)
{
    return lw_select(dim, k, dxs, cap, sel);
}
