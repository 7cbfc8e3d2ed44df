/*
 * sanitize_driver.c -- exercises every entry point of the CPU oracle on small
 * synthetic particle sets, for a build with AddressSanitizer and
 * UndefinedBehaviorSanitizer (test infrastructure: run by
 * tests/test_oracle_sanitizers.py, never part of the product library).
 * Exit status 0 when every call returns the status expected of it.
 */
#include <math.h>
#include <stdint.h>
#include <stdio.h>
#include <stdlib.h>
#include <string.h>

#include "lp_oracle.h"

static uint64_t rng_state = 12345u;
static double urand(void)
{
    rng_state = rng_state * 6364136223846793005ull + 1442695040888963407ull;
    return (double)(rng_state >> 11) * (1.0 / 9007199254740992.0);
}

static lpo_cfg base(int dim, double kappa)
{
    lpo_cfg c;
    memset(&c, 0, sizeof c);
    c.dim = dim;
    c.max_nb = 128;
    c.gamma = 1.4;
    c.cfl = dim == 2 ? 0.5 : 0.2;
    c.kappa = kappa;
    c.est_eps = 1e-5;
    c.cond_max = 1e12;
    c.uw_cond_max = 1e2;
    for (int a = 0; a < 3; ++a) { c.lo[a] = 0.0; c.hi[a] = 1.0; }
    c.phi_fixed = -1.0;
    c.limiter_cap = 1.0;
    return c;
}

typedef struct {
    int64_t n;
    double *x[3], *u[3], *V, *P, *m;
} set;

static set lattice(int dim, int nside, double jitter, int cap_extra)
{
    set s;
    int64_t n = 1;
    for (int a = 0; a < dim; ++a) n *= nside;
    s.n = n;
    int64_t cap = n + cap_extra;
    for (int a = 0; a < 3; ++a) {
        s.x[a] = calloc((size_t)cap, sizeof(double));
        s.u[a] = calloc((size_t)cap, sizeof(double));
    }
    s.V = calloc((size_t)cap, sizeof(double));
    s.P = calloc((size_t)cap, sizeof(double));
    s.m = calloc((size_t)cap, sizeof(double));
    double h = 1.0 / nside;
    for (int64_t i = 0; i < n; ++i) {
        int64_t k = i;
        for (int a = 0; a < dim; ++a) {
            int64_t q = k % nside;
            k /= nside;
            s.x[a][i] = (q + 0.5 + jitter * (2.0 * urand() - 1.0)) * h;
        }
        double r2 = 0.0;
        for (int a = 0; a < dim; ++a) r2 += (s.x[a][i] - 0.5) * (s.x[a][i] - 0.5);
        s.V[i] = 1.0;
        s.P[i] = 1.0 + 0.1 * exp(-r2 / 0.01);
        s.u[0][i] = 0.01 * sin(6.0 * s.x[1][i]);
        s.m[i] = pow(h, dim);
    }
    return s;
}

static void release(set *s)
{
    for (int a = 0; a < 3; ++a) { free(s->x[a]); free(s->u[a]); }
    free(s->V); free(s->P); free(s->m);
}

static int fails = 0;
#define EXPECT(cond, what)                                              \
    do {                                                                \
        if (!(cond)) { fprintf(stderr, "FAILED: %s\n", what); ++fails; } \
    } while (0)

static void steps(const char *tag, lpo_cfg *c, set *s, int k)
{
    int64_t n = s->n;
    double *phi = malloc(sizeof(double) * (size_t)n);
    uint8_t *flags = malloc((size_t)n);
    for (int q = 0; q < k; ++q) {
        double dt = 0.0;
        int64_t ng = 0;
        int st = lpo_step(c, n, s->x[0], s->x[1], c->dim == 3 ? s->x[2] : NULL, s->V, s->u[0], s->u[1],
                          c->dim == 3 ? s->u[2] : NULL, s->P, s->m, 0.0, phi, flags, &dt, &ng);
        EXPECT(st == LPO_OK, tag);
    }
    double out[5];
    lpo_conservation(c, n, s->V, s->u[0], s->u[1], c->dim == 3 ? s->u[2] : NULL, s->P, s->m, out);
    EXPECT(out[0] > 0.0, "conservation");
    free(phi); free(flags);
}

int main(void)
{
    /* 2D periodic pulse with the estimator, then the printed limiter */
    {
        lpo_cfg c = base(2, 2.5);
        c.periodic[0] = c.periodic[1] = 1;
        set s = lattice(2, 20, 0.2, 0);
        steps("2D periodic", &c, &s, 2);
        c.limiter_cap = 0.0;
        steps("2D printed limiter", &c, &s, 1);
        c.phi_fixed = 1.0;
        steps("2D phi = 1", &c, &s, 1);
        release(&s);
    }
    /* 3D with mirror walls in x, periodic in y and z */
    {
        lpo_cfg c = base(3, 2.1);
        c.wall_lo[0] = c.wall_hi[0] = 1;
        c.periodic[1] = c.periodic[2] = 1;
        set s = lattice(3, 8, 0.2, 0);
        steps("3D walls", &c, &s, 2);
        /* derivative operators */
        int64_t n = s.n;
        double *r = malloc(sizeof(double) * (size_t)n);
        for (int64_t i = 0; i < n; ++i) r[i] = 2.1 * cbrt(s.m[i] * s.V[i]);
        const double *f[2] = {s.V, s.P};
        double *d2 = malloc(sizeof(double) * (size_t)n * 2 * 9);
        double *d3 = malloc(sizeof(double) * (size_t)n * 2 * 19);
        uint8_t *st2 = malloc((size_t)n), *st3 = malloc((size_t)n);
        lpo_cfg g = base(3, 2.1);
        g.periodic[0] = g.periodic[1] = g.periodic[2] = 1;
        EXPECT(lpo_gfd(&g, n, s.x[0], s.x[1], s.x[2], r, 2, f, d2, st2) == LPO_OK, "gfd");
        EXPECT(lpo_gfd3(&g, n, s.x[0], s.x[1], s.x[2], r, 2, f, d3, st3) == LPO_OK, "gfd3");
        /* neighbour lists, then a capacity too small for them */
        int32_t *cnt = malloc(sizeof(int32_t) * (size_t)n), *idx = malloc(sizeof(int32_t) * (size_t)n * 128);
        EXPECT(lpo_neighbors(&g, n, s.x[0], s.x[1], s.x[2], r, 128, cnt, idx) == LPO_OK, "neighbors");
        EXPECT(lpo_neighbors(&g, n, s.x[0], s.x[1], s.x[2], r, 4, cnt, idx) == LPO_E_CAPACITY, "neighbors cap");
        free(r); free(d2); free(d3); free(st2); free(st3); free(cnt); free(idx);
        release(&s);
    }
    /* free boundary: a small cloud in vacuum */
    {
        lpo_cfg c = base(3, 2.2);
        c.vacuum = 1;
        for (int a = 0; a < 3; ++a) { c.lo[a] = -2.0; c.hi[a] = 2.0; }
        set s = lattice(3, 9, 0.3, 0);
        steps("vacuum", &c, &s, 2);
        release(&s);
    }
    /* open boundaries: outflow, reservoir state, an inflow layer */
    {
        lpo_cfg c = base(2, 2.5);
        set s = lattice(2, 16, 0.2, 16 * 16);
        for (int64_t i = 0; i < s.n; ++i) s.x[0][i] += 0.3;
        double *arr[6] = {s.x[0], s.x[1], s.u[0], s.u[1], s.V, s.P};
        const double *xs[2] = {s.x[0], s.x[1]};
        int64_t kept = 0;
        EXPECT(lpo_outflow(&c, s.n, arr, 6, xs, 0u, 1u, &kept) == LPO_OK && kept < s.n, "outflow");
        double res[4];
        EXPECT(lpo_reservoir_inflow(&c, kept, xs, s.P, 0, 0, 0.1, 2.0, 1.5, res) == LPO_OK, "reservoir");
        double *xx[2] = {s.x[0], s.x[1]}, *uu[2] = {s.u[0], s.u[1]};
        int64_t nn = 0;
        EXPECT(lpo_inflow_layer(&c, kept, kept + 16, xx, uu, s.V, s.P, s.m, 0, 0, 1.0 / 16, 0.5 / 16, res[1],
                                res[0], res[2], &nn) == LPO_OK, "inflow layer");
        EXPECT(lpo_inflow_layer(&c, kept, kept + 3, xx, uu, s.V, s.P, s.m, 0, 0, 1.0 / 16, 0.5 / 16, 1.0, 1.0,
                                0.0, &nn) == LPO_E_CAPACITY, "inflow capacity");
        release(&s);
    }
    /* estimator network: forward and gradient */
    {
        double *th = malloc(sizeof(double) * LPO_MLP_NPARAM), *gr = malloc(sizeof(double) * LPO_MLP_NPARAM);
        double feat[16 * 8], tgt[8], z[8], y[8];
        for (int q = 0; q < LPO_MLP_NPARAM; ++q) th[q] = 0.1 * (2.0 * urand() - 1.0);
        for (int q = 0; q < 16 * 8; ++q) feat[q] = 2.0 * urand() - 1.0;
        for (int q = 0; q < 8; ++q) tgt[q] = urand();
        lpo_mlp_forward(th, 8, feat, z, y);
        double loss = lpo_mlp_loss_grad(th, 8, feat, tgt, gr);
        EXPECT(loss > 0.0 && isfinite(loss), "network loss");
        free(th); free(gr);
    }
    if (fails) return 1;
    printf("sanitized oracle run: all calls returned their expected status\n");
    return 0;
}
