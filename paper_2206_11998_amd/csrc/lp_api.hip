// lp_api.hip -- the C ABI of liblp (declared in include/lp.h): context,
// device workspace and the orchestration of one LP time step (Sec. 2.2,
// steps 1-6) as a sequence of kernels on the caller's stream.
#include <math.h>
#include <stdarg.h>
#include <stdio.h>
#include <string.h>

#include <string>
#include <vector>

#include <algorithm>
#include <mutex>

#include "lp_internal.h"

static double bits_to_double(unsigned long long b) {
    double d;
    memcpy(&d, &b, sizeof d);
    return d;
}

struct Buf {
    void *p = nullptr;
    size_t bytes = 0;
    bool owned = false;  // allocated by the library (else carved from a caller's or the scratch block)
};

struct lp_ctx {
    lp_config cfg;
    DevCfg dc;
    int device = 0;
    std::string err;
    // workspace
    Buf h, r, gcnt, scan_tmp, ghosts, key, slot, tables, sorted, srec, srecf, sid, nbr, count, queue, partials, consout,
        gfd_fields, hitd2, hitj, tflags, tlo, thi, prep_part, ovfq, der, lwst, wq, rq, rkeep,
        mfeat, mrates, mphi, mflag,                          // network-estimator staging
        theta, adam_m, adam_v, mgrad, mpart, mlosspart, mscal, // network parameters and training
        cand, ccount, xb, Rb, fovfq, octc,                   // neighbour-list reuse
        openres;                                             // lp_run_open: reservoir partial sums
    int search_mode = 2;            // 0: lane group walking its cells, 1: LDS-staged tiles, 2: balanced lane group
    int solve_block = 256;
    DevScalars *sc = nullptr;       // device scalars
    DevScalars *sc_host = nullptr;  // pinned copy
    int nwalls = 0;
    double S = 1.0;                 // cube side from the box (periodic extents are S / 2^j)
    double S_grid = 1.0;            // cube side used by the last grid
    int jper[3] = {0, 0, 0};        // periodic extent = S / 2^jper
    int search_group = 8;
    int search_cap = 0;             // LDS list slots per particle of the search: 0 = automatic
    int search_lcap = 0;            // automatic choice for steps (0: the kernel's maximum)
    int gfd_lcap = 0;               // the same for lp_gfd / lp_gfd3, from the last such call's longest list
    int64_t cap_real = 0, cap_total = 0, cap_ghost = 0;
    bool run_done = false;
    DevGrid grid;
    int last_levels[2] = {0, 0};
    // stage timing
    bool profiling = false;
    std::vector<hipEvent_t> ev_pool;
    size_t ev_used = 0;
    struct Rec { int stage; hipEvent_t a, b; };
    std::vector<Rec> recs;
    // lp_run graph
    hipGraphExec_t graph = nullptr;
    hipStream_t cap_stream = nullptr;  // private stream to capture on (the caller's may be the null stream)
    lp_particles graph_p;
    uint64_t graph_gen = 0;         // workspace generation the graph was captured against
    int64_t n_captures = 0;         // graphs captured so far
    const OpenDev *open = nullptr;  // set while lp_run_open runs: its boundary stage ends every step
    uint64_t gen = 1;               // bumped by every reallocation and grid change
    double grid_margin = 0.0;       // bounding-box margin of planned grids (lp_run plans with headroom)
    int solve_mode = 0;             // LP_TUNE_SOLVE_MODE
    bool mlp_ready = false;         // network parameters set
    bool want_stage = false;        // keep network-estimator staging allocated (lp_features)
    int queue_tile = 1024;          // LP_TUNE_QUEUE_TILE
    // neighbour-list reuse (LP_TUNE_LIST_SKIN): candidate radius (1 + skin/1000) r
    int list_skin = 250;
    uint64_t reuse_gen = 0;         // workspace generation the device candidate set belongs to
    lp_particles reuse_p;           // particle arrays it was built for
    int reuse_skin = -1;            // skin it was built with
    bool grid_set = false;          // a grid has been planned
    // while set, ensure() carves buffers out of this device block instead of
    // allocating: the caller's workspace (lp_set_workspace) or the scratch
    // block of lp_neighbors_noalloc; running out returns arena_status
    char *arena = nullptr;
    size_t arena_bytes = 0, arena_used = 0;
    lp_status arena_status = LP_E_NOMEM;
    bool caller_ws = false;         // arena is the caller's workspace
    // while set, ensure() only adds up the bytes it would carve (lp_workspace_bytes)
    bool measure = false;
    size_t measure_bytes = 0;
};

// every workspace buffer of a context, for swapping the whole set out and back
static Buf lp_ctx::*const kBufs[] = {
    &lp_ctx::h, &lp_ctx::r, &lp_ctx::gcnt, &lp_ctx::scan_tmp, &lp_ctx::ghosts, &lp_ctx::key, &lp_ctx::slot,
    &lp_ctx::tables, &lp_ctx::sorted, &lp_ctx::srec, &lp_ctx::srecf, &lp_ctx::sid, &lp_ctx::nbr, &lp_ctx::count,
    &lp_ctx::queue, &lp_ctx::partials, &lp_ctx::consout, &lp_ctx::gfd_fields, &lp_ctx::hitd2, &lp_ctx::hitj,
    &lp_ctx::tflags, &lp_ctx::tlo, &lp_ctx::thi, &lp_ctx::prep_part, &lp_ctx::ovfq, &lp_ctx::der, &lp_ctx::lwst,
    &lp_ctx::wq, &lp_ctx::rq, &lp_ctx::rkeep, &lp_ctx::mfeat, &lp_ctx::mrates, &lp_ctx::mphi, &lp_ctx::mflag,
    &lp_ctx::theta, &lp_ctx::adam_m, &lp_ctx::adam_v, &lp_ctx::mgrad, &lp_ctx::mpart, &lp_ctx::mlosspart,
    &lp_ctx::mscal, &lp_ctx::cand, &lp_ctx::ccount, &lp_ctx::xb, &lp_ctx::Rb, &lp_ctx::fovfq, &lp_ctx::octc,
    &lp_ctx::openres};
constexpr int kNumBufs = (int)(sizeof kBufs / sizeof kBufs[0]);

static lp_status fail(lp_ctx *c, lp_status s, const char *fmt, ...) {
    if (c) {
        char buf[512];
        va_list ap;
        va_start(ap, fmt);
        vsnprintf(buf, sizeof buf, fmt, ap);
        va_end(ap);
        c->err = buf;
    }
    return s;
}

#define HIPCHK(ctx, call)                                                                        \
    do {                                                                                         \
        hipError_t e_ = (call);                                                                  \
        if (e_ != hipSuccess) return fail(ctx, LP_E_DEVICE, "%s: %s", #call, hipGetErrorString(e_)); \
    } while (0)

static size_t align256(size_t b) { return (b + 255) & ~(size_t)255; }

static lp_status ensure(lp_ctx *c, Buf &b, size_t bytes) {
    if (c->measure) {
        c->measure_bytes += align256(bytes);
        return LP_OK;
    }
    if (b.bytes >= bytes) return LP_OK;
    ++c->gen;  // captured graphs hold the old address
    if (c->arena) {
        // a buffer that grows is carved anew after the others (its old region stays unused)
        size_t off = align256(c->arena_used);
        if (off > c->arena_bytes || bytes > c->arena_bytes - off)
            return fail(c, c->arena_status, "the workspace needs more than the %zu-byte %s", c->arena_bytes,
                        c->caller_ws ? "caller workspace" : "scratch block");
        if (b.p && b.owned) (void)hipFree(b.p);
        b.p = c->arena + off;
        b.bytes = bytes;
        b.owned = false;
        c->arena_used = off + bytes;
        return LP_OK;
    }
    if (b.p && b.owned) (void)hipFree(b.p);
    b.p = nullptr;
    b.bytes = 0;
    b.owned = false;
    size_t want = bytes + bytes / 8 + 256;
    if (hipMalloc(&b.p, want) != hipSuccess) {
        (void)hipGetLastError();
        return fail(c, LP_E_NOMEM, "device allocation of %zu bytes failed", want);
    }
    b.bytes = want;
    b.owned = true;
    return LP_OK;
}

static hipEvent_t next_event(lp_ctx *c) {
    if (c->ev_used == c->ev_pool.size()) {
        hipEvent_t e;
        if (hipEventCreate(&e) != hipSuccess) return nullptr;
        c->ev_pool.push_back(e);
    }
    return c->ev_pool[c->ev_used++];
}

// Mark the start (begin = true) or end of a timed stage on stream st.
static void stage_mark(lp_ctx *c, hipStream_t st, int stage, bool begin) {
    if (!c->profiling) return;
    hipEvent_t e = next_event(c);
    if (!e) return;
    (void)hipEventRecord(e, st);
    if (begin) {
        c->recs.push_back({stage, e, nullptr});
        return;
    }
    // stages nest (the whole step encloses its parts): close the latest open one
    for (size_t q = c->recs.size(); q-- > 0;)
        if (c->recs[q].stage == stage && !c->recs[q].b) {
            c->recs[q].b = e;
            return;
        }
}

#define ENSURE(ctx, buf, bytes)                        \
    do {                                               \
        lp_status s_ = ensure(ctx, buf, bytes);        \
        if (s_ != LP_OK) return s_;                    \
    } while (0)

// Scratch block of lp_neighbors_noalloc: one per device, held until the
// process ends.  In host code `scratch` names a host-side stand-in; the
// device address comes from hipGetSymbolAddress, once per device, in
// lp_create, and only that address is ever passed on.
#define LP_SCRATCH_MAX_DEVICES 64
static __device__ __align__(256) unsigned char scratch[LP_NOALLOC_SCRATCH_BYTES];
static std::mutex g_scratch_mu;
static void *g_scratch_ptr[LP_SCRATCH_MAX_DEVICES];
static hipError_t g_scratch_err[LP_SCRATCH_MAX_DEVICES];

static void scratch_setup(int device) {
    if (device < 0 || device >= LP_SCRATCH_MAX_DEVICES) return;
    std::lock_guard<std::mutex> lock(g_scratch_mu);
    if (g_scratch_ptr[device]) return;
    void *p = nullptr;
    hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e == hipSuccess && p) g_scratch_ptr[device] = p;
    else {
        g_scratch_err[device] = e == hipSuccess ? hipErrorInvalidSymbol : e;
        (void)hipGetLastError();
    }
}

static void *scratch_ptr(int device, hipError_t *err) {
    if (device < 0 || device >= LP_SCRATCH_MAX_DEVICES) { *err = hipErrorInvalidDevice; return nullptr; }
    std::lock_guard<std::mutex> lock(g_scratch_mu);
    *err = g_scratch_err[device];
    return g_scratch_ptr[device];
}

extern "C" void lp_config_default(lp_config *cfg, int32_t dim) {
    memset(cfg, 0, sizeof *cfg);
    cfg->dim = dim;
    cfg->precision = LP_FP64;
    cfg->estimator = LP_EST_PLAIN;
    cfg->max_nb = 128;
    cfg->refine = 1;
    cfg->gamma = 1.4;
    cfg->cfl = 0.5;
    cfg->kappa = dim == 2 ? 2.5 : 2.1;
    cfg->est_eps = 1e-5;
    cfg->cond_max = 1e12;
    cfg->uw_cond_max = 1e2;
    cfg->cond_fallback = 1e6;
    for (int a = 0; a < 3; ++a) { cfg->box_lo[a] = 0.0; cfg->box_hi[a] = 1.0; }
    cfg->periodic_mask = dim == 2 ? 3u : 7u;
    cfg->mlp_band = 0.05f;
    cfg->mlp_feat_max = 8.0f;
    cfg->limiter_cap = 1.0f;
}

extern "C" const char *lp_status_str(lp_status s) {
    switch (s) {
    case LP_OK: return "ok";
    case LP_E_ARG: return "invalid argument";
    case LP_E_CAPACITY: return "neighbour list capacity exceeded";
    case LP_E_NUMERIC: return "non-positive volume or pressure";
    case LP_E_DEVICE: return "HIP runtime error";
    case LP_E_NOMEM: return "out of device memory";
    case LP_E_STATE: return "invalid call sequence";
    default: return "unknown status";
    }
}

extern "C" const char *lp_last_error(const lp_ctx *c) { return c ? c->err.c_str() : "null context"; }

static bool is_pow2_ratio(double big, double small, int *j) {
    double q = big / small;
    int e = (int)llround(log2(q));
    if (e < 0 || e > 12) return false;
    if (fabs(ldexp(small, e) - big) > 1e-12 * big) return false;
    *j = e;
    return true;
}

extern "C" lp_status lp_create(const lp_config *cfg, lp_ctx **out) {
    if (!cfg || !out) return LP_E_ARG;
    *out = nullptr;
    lp_ctx *c = new lp_ctx();
    c->cfg = *cfg;
    const lp_config &k = *cfg;
    lp_status st = LP_OK;
    if (k.dim != 2 && k.dim != 3) st = fail(c, LP_E_ARG, "dim must be 2 or 3");
    else if (k.max_nb < 1 || k.max_nb > 256) st = fail(c, LP_E_ARG, "max_nb must be in 1..256");
    else if (k.lw_cap < 0 || k.lw_cap > 64) st = fail(c, LP_E_ARG, "lw_cap must be in 0..64");
    else if (k.uw_cap < 0 || k.uw_cap > 16) st = fail(c, LP_E_ARG, "uw_cap must be in 0..16");
    else if (k.precision != LP_FP64 && k.precision != LP_MIXED) st = fail(c, LP_E_ARG, "bad precision");
    else if (k.estimator != LP_EST_PLAIN && k.estimator != LP_EST_INJECTED && k.estimator != LP_EST_MLP)
        st = fail(c, LP_E_ARG, "unknown estimator mode");
    else if (!(k.mlp_band >= 0.0f && k.mlp_band <= 0.5f) || !(k.mlp_feat_max > 0.0f))
        st = fail(c, LP_E_ARG, "mlp_band must be in [0, 1/2], mlp_feat_max positive");
    else if (!(k.refine_cond >= 0.0f) || !(k.refine_cond < INFINITY))
        st = fail(c, LP_E_ARG, "refine_cond must be finite and non-negative");
    else if (!(k.limiter_cap >= 0.0f) || !(k.limiter_cap < INFINITY))
        st = fail(c, LP_E_ARG, "limiter_cap must be finite and non-negative");
    else if (!(k.gamma > 1.0) || !(k.kappa > 0.0) || !(k.cfl > 0.0)) st = fail(c, LP_E_ARG, "gamma, kappa, cfl");
    if (st == LP_OK) {
        double S = 0.0;
        for (int a = 0; a < k.dim; ++a) {
            double e = k.box_hi[a] - k.box_lo[a];
            if (!(e > 0.0)) { st = fail(c, LP_E_ARG, "empty box on axis %d", a); break; }
            if (e > S) S = e;
        }
        c->S = S;
        for (int a = 0; a < k.dim && st == LP_OK; ++a) {
            bool per = (k.periodic_mask >> a) & 1u;
            bool wall = ((k.wall_lo_mask | k.wall_hi_mask) >> a) & 1u;
            if (per && wall) st = fail(c, LP_E_ARG, "axis %d is both periodic and walled", a);
            if (per && !is_pow2_ratio(S, k.box_hi[a] - k.box_lo[a], &c->jper[a]))
                st = fail(c, LP_E_ARG, "periodic extent of axis %d must be the largest extent / 2^j", a);
        }
    }
    if (st != LP_OK) {
        fprintf(stderr, "lp_create: %s\n", c->err.c_str());
        delete c;
        return st;
    }
    DevCfg &d = c->dc;
    memset(&d, 0, sizeof d);
    d.D = k.dim;
    d.nu = k.dim == 3 ? 9 : 5;
    d.nf = k.dim + 2;
    d.lw_cap = k.lw_cap > 0 ? k.lw_cap : (k.dim == 3 ? 54 : 32);
    d.uw_cap = k.uw_cap > 0 ? k.uw_cap : 8;
    d.max_nb = k.max_nb;
    d.vacuum = k.vacuum;
    d.est_mode = k.estimator;
    d.precision = k.precision;
    d.refine = k.refine;
    d.refine_cond = k.refine_cond;
    d.gamma = k.gamma;
    d.kappa = k.kappa;
    d.cfl = k.cfl;
    d.est_eps = k.est_eps;
    d.cond_max = k.cond_max;
    d.uw_cond_max = k.uw_cond_max;
    d.cond_fb = k.cond_fallback;
    d.mlp_band = k.mlp_band;
    d.mlp_feat_max = k.mlp_feat_max;
    d.limiter_cap = k.limiter_cap;
    for (int a = 0; a < 3; ++a) {
        d.lo[a] = k.box_lo[a];
        d.hi[a] = k.box_hi[a];
        d.L[a] = k.box_hi[a] - k.box_lo[a];
        d.half[a] = 0.5 * d.L[a];
        d.periodic[a] = a < k.dim ? (int)((k.periodic_mask >> a) & 1u) : 0;
        d.wall_lo[a] = a < k.dim ? (int)((k.wall_lo_mask >> a) & 1u) : 0;
        d.wall_hi[a] = a < k.dim ? (int)((k.wall_hi_mask >> a) & 1u) : 0;
        c->nwalls += d.wall_lo[a] + d.wall_hi[a];
    }
    (void)hipGetDevice(&c->device);
    scratch_setup(c->device);
    if (hipMalloc((void **)&c->sc, sizeof(DevScalars)) != hipSuccess ||
        hipHostMalloc((void **)&c->sc_host, sizeof(DevScalars), hipHostMallocDefault) != hipSuccess) {
        (void)hipGetLastError();
        delete c;
        return LP_E_NOMEM;
    }
    memset(c->sc_host, 0, sizeof(DevScalars));
    if (hipMemcpy(c->sc, c->sc_host, sizeof(DevScalars), hipMemcpyHostToDevice) != hipSuccess) {
        delete c;
        return LP_E_DEVICE;
    }
    *out = c;
    return LP_OK;
}

extern "C" lp_status lp_destroy(lp_ctx *c) {
    if (!c) return LP_E_ARG;
    (void)hipDeviceSynchronize();
    if (c->graph) (void)hipGraphExecDestroy(c->graph);
    if (c->cap_stream) (void)hipStreamDestroy(c->cap_stream);
    for (hipEvent_t e : c->ev_pool) (void)hipEventDestroy(e);
    for (int q = 0; q < kNumBufs; ++q)
        if ((c->*kBufs[q]).p && (c->*kBufs[q]).owned) (void)hipFree((c->*kBufs[q]).p);
    if (c->sc) (void)hipFree(c->sc);
    if (c->sc_host) (void)hipHostFree(c->sc_host);
    delete c;
    return LP_OK;
}

// ---------------------------------------------------------------------------
// Grid levels from the radius range: the finest level has cells no larger
// than r_min (bounded by a table of 2^27 cells), the coarsest no larger than
// r_max; periodic axes need whole cells per period.
// ---------------------------------------------------------------------------
static double key_to_double(unsigned long long k) {
    unsigned long long b = (k >> 63) ? (k & 0x7fffffffffffffffull) : ~k;
    return bits_to_double(b);
}

// Grid cube: with any periodic axis, the box-derived side S (periodic
// extents are S / 2^j); otherwise the cube is fitted to the particles'
// bounding box read back with the radii (widened by margin * extent on every
// side), so no level is wasted on empty space.  Pure: writes only g and S.
static void plan_grid(const lp_ctx *c, double rmin, double rmax, double margin, DevGrid &g, double &S_out,
                      int levels[2]) {
    const int D = c->dc.D;
    const int Lmax = D == 3 ? 9 : 13;
    int jmin = 0;
    bool any_periodic = false;
    for (int a = 0; a < D; ++a) {
        if (c->dc.periodic[a]) any_periodic = true;
        if (c->dc.periodic[a] && c->jper[a] > jmin) jmin = c->jper[a];
    }
    double S = c->S;
    double glo[3] = {c->dc.lo[0], c->dc.lo[1], c->dc.lo[2]};
    if (!any_periodic) {
        double ext = 0.0;
        for (int a = 0; a < D; ++a) {
            double lo = key_to_double(c->sc_host->xlo[a]), hi = key_to_double(c->sc_host->xhi[a]);
            if (!(hi >= lo)) { lo = c->dc.lo[a]; hi = c->dc.hi[a]; }
            glo[a] = lo;
            if (hi - lo > ext) ext = hi - lo;
        }
        if (!(ext > 0.0)) ext = c->S;
        for (int a = 0; a < D; ++a) glo[a] -= margin * ext;
        S = ext * (1.0 + 2.0 * margin) * (1.0 + 1e-9) + 1e-300;
    }
    S_out = S;
    auto level_le = [&](double r) {
        int L = 0;
        while (L < Lmax && ldexp(S, -L) > r) ++L;
        return L;
    };
    int hi = level_le(rmin > 0 ? rmin : c->S);
    int lo = level_le(rmax > 0 ? rmax : c->S);
    if (hi < jmin) hi = jmin;
    if (lo < jmin) lo = jmin;
    if (lo > hi) lo = hi;
    if (hi - lo > 6) lo = hi - 6;
    memset(&g, 0, sizeof g);
    g.L_lo = lo;
    g.L_hi = hi;
    unsigned long long off = 0;
    for (int L = 0; L < LP_MAX_LEVEL; ++L) {
        g.s[L] = ldexp(S, -L);
        g.inv_s[L] = ldexp(1.0 / S, L);
        for (int a = 0; a < 3; ++a) {
            if (a >= D) { g.nc[L][a] = 1; continue; }
            int n = 1 << L;
            if (c->dc.periodic[a]) n = L >= c->jper[a] ? (1 << (L - c->jper[a])) : 1;
            g.nc[L][a] = n;
        }
        if (L >= lo && L <= hi) {
            g.off[L] = off;
            off += (1ull << (D * L)) + 1;
        }
    }
    for (int a = 0; a < 3; ++a) g.lo[a] = a < D ? glo[a] : 0.0;
    levels[0] = lo;
    levels[1] = hi;
}

static void choose_levels(lp_ctx *c, double rmin, double rmax) {
    DevGrid g;
    double S;
    int lv[2];
    plan_grid(c, rmin, rmax, c->grid_margin, g, S, lv);
    if (memcmp(&g, &c->grid, sizeof g) != 0) ++c->gen;
    c->grid = g;
    c->S_grid = S;
    c->last_levels[0] = lv[0];
    c->last_levels[1] = lv[1];
    c->grid_set = true;
}

// A graph-replayed step keeps the grid it was captured with.  That grid stays
// correct for any positions and radii (search boxes are clamped to the grid and
// outlying particles sit in its edge cells), but it is re-planned once the
// particles leave the cube or the radii need other levels.
static bool grid_outdated(const lp_ctx *c) {
    const DevScalars &h = *c->sc_host;
    bool any_periodic = false;
    for (int a = 0; a < c->dc.D; ++a) any_periodic |= c->dc.periodic[a] != 0;
    if (!any_periodic)
        for (int a = 0; a < c->dc.D; ++a) {
            double lo = key_to_double(h.xlo[a]), hi = key_to_double(h.xhi[a]);
            if (lo < c->grid.lo[a] || hi >= c->grid.lo[a] + c->S_grid) return true;
        }
    DevGrid g;
    double S;
    int lv[2];
    plan_grid(c, bits_to_double(h.rmin), bits_to_double(h.rmax), c->grid_margin, g, S, lv);
    // levels from the current cube side (the fitted side only grows between plans)
    return lv[1] > c->grid.L_hi + 1 || lv[0] < c->grid.L_lo - 1;
}

static uint64_t table_words(const lp_ctx *c) {
    const DevGrid &g = c->grid;
    uint64_t w = 0;
    for (int L = g.L_lo; L <= g.L_hi; ++L) w += (1ull << (c->dc.D * L)) + 1;
    return w;
}

// List slots per particle in the LDS of the search and filter kernels, from
// the longest list seen last (0: the kernels' maximum, 128).  Somewhat below
// that longest list: the few longer lists take the overflow kernel, and the
// smaller buffer lets another block share a CU (at 2M particles with
// lists of up to 76, 72 slots beat 96 by 0.3 ms a step).
static int lds_list_cap(int longest) {
    if (longest <= 0) return 0;
    const int cap = (longest * 15 / 16 + 7) / 8 * 8;
    return cap > 128 ? 0 : (cap < 16 ? 16 : cap);
}

// Allocate everything that depends on the particle counts and the grid.
// Arrays in cell order use the capacity cap_total as their stride.
// Neighbour lists reused between steps: a time step, no mirror walls (the
// ghost set would change with the positions), the balanced search, skin > 0.
static bool reuse_on(const lp_ctx *c) { return c->list_skin > 0 && c->nwalls == 0 && c->search_mode == 2; }
static double reuse_scale(const lp_ctx *c) { return 1.0 + c->list_skin / 1000.0; }

static lp_status ensure_capacity(lp_ctx *c, int64_t n_real, int64_t n_total, bool state, bool mixed) {
    const int D = c->dc.D;
    if (n_total > c->cap_total) c->cap_total = n_total;
    if (n_real > c->cap_real) c->cap_real = n_real;
    if (n_total - n_real > c->cap_ghost) c->cap_ghost = n_total - n_real;
    const int64_t nt = c->cap_total, nr = c->cap_real, ng = c->cap_ghost;
    ENSURE(c, c->h, sizeof(double) * nr);
    ENSURE(c, c->r, sizeof(double) * nr);
    ENSURE(c, c->gcnt, sizeof(uint32_t) * (nr + 1));
    uint64_t finest = 1ull << (D * c->grid.L_hi);
    uint64_t sw = scan_tmp_words(finest > (uint64_t)nr ? finest : (uint64_t)nr);
    ENSURE(c, c->scan_tmp, sizeof(uint32_t) * sw);
    if (ng > 0) ENSURE(c, c->ghosts, sizeof(double) * 10 * ng);
    ENSURE(c, c->key, sizeof(uint32_t) * nt);
    ENSURE(c, c->slot, sizeof(uint32_t) * nt);
    ENSURE(c, c->tables, sizeof(uint32_t) * table_words(c));
    ENSURE(c, c->sorted, sizeof(double) * (state ? 10 : 4) * nt);
    // FP64 gather records: the FP64 fits and update, and the refine-every-fit
    // mixed step (the FP32 fits read the FP32-field records; the few fits the
    // mixed step refines or sends to the FP64 fallback gather from the arrays)
    if (state && (!mixed || (c->dc.refine && !(c->dc.refine_cond > 0.0f))))
        ENSURE(c, c->srec, sizeof(double) * LP_REC * nt);
    if (state && c->dc.precision == LP_MIXED) ENSURE(c, c->srecf, (size_t)LP_RECF_BYTES * nt);
    ENSURE(c, c->sid, sizeof(int) * nt);
    ENSURE(c, c->nbr, sizeof(int) * (size_t)c->dc.max_nb * nt);
    ENSURE(c, c->count, sizeof(int) * nt);
    ENSURE(c, c->queue, sizeof(int) * nt);
    ENSURE(c, c->ovfq, sizeof(int) * nt);
    if (state && reuse_on(c)) {
        ENSURE(c, c->cand, sizeof(int) * (size_t)c->dc.max_nb * (size_t)((nt + 7) / 8 * 8));  // interleaved by 8
        ENSURE(c, c->ccount, sizeof(int) * nt);
        ENSURE(c, c->xb, sizeof(double) * 3 * nr);
        ENSURE(c, c->Rb, sizeof(double) * nr);
        ENSURE(c, c->fovfq, sizeof(int) * nt);
        ENSURE(c, c->octc, sizeof(unsigned long long) * nt);
    }
    if (state) {
        // the derivative array between the fit and the update kernels: FP64
        // fits and always-refined FP32 fits (the fused kernel keeps them in registers)
        if (!mixed || (c->dc.refine && !(c->dc.refine_cond > 0.0f)))
            ENSURE(c, c->der, sizeof(double) * (size_t)der_count(D) * nt);
        ENSURE(c, c->lwst, (size_t)nt);
        ENSURE(c, c->wq, sizeof(int) * nt);
        if (mixed && c->dc.refine && c->dc.refine_cond > 0.0f) {
            ENSURE(c, c->rq, sizeof(int) * 2 * nt);
            ENSURE(c, c->rkeep, sizeof(float) * (size_t)refine_keep_count(D) * nt);
        }
        if (c->dc.est_mode == LP_EST_MLP || c->want_stage) {
            ENSURE(c, c->mfeat, sizeof(float) * LP_MLP_NIN * nt);
            ENSURE(c, c->mrates, sizeof(double) * 2 * (D + 2) * nt);
            ENSURE(c, c->mphi, sizeof(double) * nt);
            ENSURE(c, c->mflag, (size_t)nt);
        }
    }
    if (c->search_mode == 1) {
        ENSURE(c, c->hitd2, sizeof(double) * (size_t)c->dc.max_nb * nt);
        ENSURE(c, c->hitj, sizeof(int) * (size_t)c->dc.max_nb * nt);
        ENSURE(c, c->tflags, sizeof(uint32_t) * (nt + 1));
        ENSURE(c, c->tlo, sizeof(int) * nt);
        ENSURE(c, c->thi, sizeof(int) * nt);
        uint64_t sw2 = scan_tmp_words((uint64_t)nt);
        if (sw2 > sw) ENSURE(c, c->scan_tmp, sizeof(uint32_t) * sw2);
    }
    return LP_OK;
}

// list stride convention of nb_at(): > 0 column-major, < 0 row-major
static int list_ldn(const lp_ctx *c) { return c->search_mode == 1 ? -c->dc.max_nb : (int)c->cap_total; }

static void run_search(lp_ctx *c, const Sorted &srt, int64_t n_total, int n_real, int lcap, hipStream_t st) {
    int ldn = (int)c->cap_total;
    if (c->search_mode == 1)
        launch_search_tiles(srt, &c->sc->n_total, (int)n_total, n_real, (const uint32_t *)c->tables.p, c->grid,
                            c->dc, (double *)c->hitd2.p, (int *)c->hitj.p, (int *)c->nbr.p, ldn, (int *)c->count.p,
                            c->sc, (const uint32_t *)c->key.p, (uint32_t *)c->tflags.p, (uint32_t *)c->scan_tmp.p,
                            (int *)c->tlo.p, (int *)c->thi.p, &c->sc->n_tiles, st);
    else
        launch_search(srt, &c->sc->n_total, (int)n_total, n_real, (const uint32_t *)c->tables.p, c->grid, c->dc,
                      (int *)c->nbr.p, ldn, (int *)c->count.p, c->sc, c->search_group, lcap, (int *)c->ovfq.p,
                      c->search_mode == 2, st);
}

static Sorted sorted_view(lp_ctx *c, bool state) {
    Sorted s;
    memset(&s, 0, sizeof s);
    double *b = (double *)c->sorted.p;
    size_t n = (size_t)c->cap_total;
    s.x[0] = b; s.x[1] = b + n; s.x[2] = b + 2 * n;
    s.r = b + 3 * n;
    if (state) {
        s.V = b + 4 * n; s.u[0] = b + 5 * n; s.u[1] = b + 6 * n; s.u[2] = b + 7 * n; s.P = b + 8 * n; s.h = b + 9 * n;
    }
    if (state && c->srec.p && c->srec.bytes >= sizeof(double) * LP_REC * n) s.rec = (double *)c->srec.p;
    if (state && c->dc.precision == LP_MIXED && c->srecf.p && c->srecf.bytes >= (size_t)LP_RECF_BYTES * n)
        s.recf = (float *)c->srecf.p;
    s.id = (int *)c->sid.p;
    return s;
}

static Ghosts ghost_view(lp_ctx *c) {
    Ghosts g;
    memset(&g, 0, sizeof g);
    int64_t ng = c->cap_ghost;
    if (ng <= 0 || !c->ghosts.p) return g;
    double *b = (double *)c->ghosts.p;
    size_t n = (size_t)ng;
    g.x[0] = b; g.x[1] = b + n; g.x[2] = b + 2 * n; g.V = b + 3 * n; g.u[0] = b + 4 * n; g.u[1] = b + 5 * n;
    g.u[2] = b + 6 * n; g.P = b + 7 * n; g.h = b + 8 * n; g.r = b + 9 * n;
    return g;
}

// Cell-order layout of n_total particles: keys, counting sort, level tables.
// gate (may be NULL): the cells are rebuilt only where *gate != 0 on the device
static void build_cells(lp_ctx *c, hipStream_t st, const double *const x[3], const double *const gx[3], int n_real,
                        int64_t n_total, const unsigned *gate = nullptr, const double *m = nullptr) {
    const int D = c->dc.D;
    const DevGrid &g = c->grid;
    uint32_t *tabs = (uint32_t *)c->tables.p;
    uint32_t *finest = tabs + g.off[g.L_hi];
    uint64_t nfin = 1ull << (D * g.L_hi);
    launch_fill_u32(finest, nfin + 1, 0u, st, gate);
    // the sort reads every real slot and ghost (n_in); absent particles (zero
    // mass, m given) are left out of the cell order
    launch_keys(x, gx, n_real, &c->sc->n_in, (int)n_total, g, D, (uint32_t *)c->key.p, (uint32_t *)c->slot.p,
                finest, st, gate, m);
    launch_scan_u32(finest, nfin, (uint32_t *)c->scan_tmp.p, nullptr, st, gate);
}

// Output buffers of lp_features (caller order, device).
struct lp_features_out {
    float *feat, *phi;
    uint8_t *valid;
};

static lp_status check_particles(lp_ctx *c, const lp_particles *p) {
    if (!p || p->n <= 0 || p->n > (1ll << 30)) return fail(c, LP_E_ARG, "particle count must be in 1..2^30");
    for (int a = 0; a < c->dc.D; ++a)
        if (!p->x[a] || !p->u[a]) return fail(c, LP_E_ARG, "null position/velocity array");
    if (!p->V || !p->P || !p->m) return fail(c, LP_E_ARG, "null V, P or m");
    if (c->dc.est_mode == LP_EST_INJECTED && !p->phi) return fail(c, LP_E_ARG, "injected estimator needs phi");
    if (c->dc.est_mode == LP_EST_MLP && !c->mlp_ready)
        return fail(c, LP_E_STATE, "estimator network has no parameters (lp_mlp_init / lp_mlp_set)");
    return LP_OK;
}

static Soa soa_of(const lp_particles *p) {
    Soa s;
    memset(&s, 0, sizeof s);
    for (int a = 0; a < 3; ++a) { s.x[a] = p->x[a]; s.u[a] = p->u[a]; }
    if (!s.x[2]) s.x[2] = s.x[0];
    if (!s.u[2]) s.u[2] = s.u[0];
    s.V = p->V; s.P = p->P; s.m = p->m; s.phi = p->phi; s.flags = p->flags;
    s.n = (int)p->n;
    return s;
}

// One step.  sync_levels: read r_min / r_max / ghost count back to size the
// grid and the workspace (lp_step, and the planning steps of lp_run);
// otherwise the current grid and capacities are used as they are (the step
// captured for graph replay: no host synchronisation, no allocation, kernels
// sized to the capacities and bounded by the device-side counts).
static lp_status step_impl(lp_ctx *c, hipStream_t st, const lp_particles *p, double dt_in, bool sync_levels,
                           int clip_t_end, const lp_features_out *harvest = nullptr) {
    const int D = c->dc.D;
    const int n = (int)p->n;
    const bool mixed = c->dc.precision == LP_MIXED;
    Soa soa = soa_of(p);
    if (sync_levels) {
        ENSURE(c, c->h, sizeof(double) * n);
        ENSURE(c, c->r, sizeof(double) * n);
        ENSURE(c, c->gcnt, sizeof(uint32_t) * (n + 1));
        ENSURE(c, c->scan_tmp, sizeof(uint32_t) * scan_tmp_words(n));
        ENSURE(c, c->prep_part, sizeof(double) * prep_partial_words(n));
    }
    stage_mark(c, st, 0, true);
    launch_reset_scalars(c->sc, dt_in, n, sync_levels ? 1 : 0, st);
    {
        // the list-reuse check rides on the radii pass, where the last build's
        // positions and radii cover these particles (else the step rebuilds)
        const bool chk = reuse_on(c) && c->xb.p && c->Rb.p && c->cap_real >= n;
        double *xbp[3] = {(double *)c->xb.p, (double *)c->xb.p + c->cap_real, (double *)c->xb.p + 2 * c->cap_real};
        launch_prep(soa, c->dc, c->sc, (double *)c->h.p, (double *)c->r.p, (double *)c->prep_part.p, st,
                    chk ? xbp : nullptr, chk ? (const double *)c->Rb.p : nullptr);
    }
    launch_dt(c->dc, c->sc, clip_t_end, st);
    if (c->nwalls) {
        launch_ghost_count(soa, c->dc, c->sc, (uint32_t *)c->gcnt.p, st);
        launch_scan_u32((uint32_t *)c->gcnt.p, n, (uint32_t *)c->scan_tmp.p, &c->sc->n_ghost, st);
    }
    int64_t n_total;
    if (sync_levels) {
        stage_mark(c, st, 0, false);
        HIPCHK(c, hipMemcpyAsync(c->sc_host, c->sc, sizeof(DevScalars), hipMemcpyDeviceToHost, st));
        HIPCHK(c, hipStreamSynchronize(st));
        if (clip_t_end && c->sc_host->done) {
            c->run_done = true;
            return LP_OK;
        }
        n_total = n + c->sc_host->n_ghost;
        // a planning step of lp_run keeps the grid a captured graph was made
        // with while it still covers the particles and their radii
        const bool keep = c->grid_set && c->grid_margin > 0.0 &&
                          ((c->graph && c->graph_gen == c->gen) || reuse_on(c)) && !grid_outdated(c);
        if (!keep) choose_levels(c, bits_to_double(c->sc_host->rmin), bits_to_double(c->sc_host->rmax));
        int64_t want = n_total;
        if (c->nwalls && c->grid_margin > 0.0) {
            // planning for graph replays: room for the ghost count to grow
            int64_t ng = c->sc_host->n_ghost;
            want = n + ng + ng / 4 + 1024;
        }
        lp_status s = ensure_capacity(c, n, want, true, mixed);
        if (s != LP_OK) return s;
        // search list slots in LDS from the last step's largest list
        const int lcap = lds_list_cap(c->sc_host->prev_max_count);
        if (lcap != c->search_lcap) {
            c->search_lcap = lcap;
            ++c->gen;  // a captured step holds the old buffer size
        }
    } else {
        n_total = c->cap_total;
    }
    // ghosts admitted: what both the ghost arrays and the cell-order arrays hold
    const int64_t gcap = c->nwalls ? std::min<int64_t>(c->cap_ghost, c->cap_total - n) : 0;
    launch_gate(c->sc, n, gcap, clip_t_end, st);  // lp_run's steps stop at a reported error
    // neighbour-list reuse: the device decides per step whether the
    // candidate lists of the last rebuild still cover every neighbour; a
    // rebuild is forced when the workspace, the grid, the particle arrays or
    // the skin changed since they were built (host state, so only eager and
    // planning steps can force one: a captured step is replayed on the same)
    const bool reuse = reuse_on(c);
    const unsigned *gate = nullptr;
    if (reuse) {
        const bool same = c->reuse_gen == c->gen && c->reuse_skin == c->list_skin &&
                          memcmp(&c->reuse_p, p, sizeof *p) == 0;
        double *xb[3] = {(double *)c->xb.p, (double *)c->xb.p + c->cap_real, (double *)c->xb.p + 2 * c->cap_real};
        launch_reuse(soa, c->dc, (const double *)c->r.p, xb, (double *)c->Rb.p, n, reuse_scale(c), same ? 0 : 1,
                     c->sc, st);
        c->reuse_gen = c->gen;
        c->reuse_skin = c->list_skin;
        c->reuse_p = *p;
        gate = &c->sc->rebuild;
    }
    Ghosts gh = ghost_view(c);
    stage_mark(c, st, 1, true);
    if (c->nwalls)
        launch_ghost_write(soa, c->dc, c->sc, (const uint32_t *)c->gcnt.p, (const double *)c->h.p,
                           (const double *)c->r.p, gh, c->cap_ghost, st);
    const double *gx[3] = {gh.x[0], gh.x[1], gh.x[2]};
    const double *x[3] = {p->x[0], p->x[1], D == 3 ? p->x[2] : p->x[1]};
    build_cells(c, st, x, gx, n, n_total, gate, p->m);
    Sorted srt = sorted_view(c, true);
    ScatterArgs sa;
    memset(&sa, 0, sizeof sa);
    const double *src[10] = {soa.x[0], soa.x[1], soa.x[2], (const double *)c->r.p, soa.V, soa.u[0], soa.u[1],
                             soa.u[2], soa.P, (const double *)c->h.p};
    const double *gsrc[10] = {gh.x[0], gh.x[1], gh.x[2], gh.r, gh.V, gh.u[0], gh.u[1], gh.u[2], gh.P, gh.h};
    double *dst[10] = {srt.x[0], srt.x[1], srt.x[2], srt.r, srt.V, srt.u[0], srt.u[1], srt.u[2], srt.P, srt.h};
    sa.nd = 10;
    for (int q = 0; q < 10; ++q) { sa.src[q] = src[q]; sa.gsrc[q] = gsrc[q]; sa.dst[q] = dst[q]; }
    if (D == 2) { sa.src[2] = soa.x[0]; sa.src[7] = soa.u[0]; }
    // gather records: x_0..x_{D-1}, V, u_0..u_{D-1}, P (value indices above)
    sa.rec = srt.rec;
    sa.recf = srt.recf;
    sa.dim = D;
    sa.m = p->m;
    {
        const int r3[LP_REC] = {0, 1, 2, 4, 5, 6, 7, 8}, r2[LP_REC] = {0, 1, 4, 5, 6, 8, -1, -1};
        for (int q = 0; q < LP_REC; ++q) sa.rec_src[q] = D == 3 ? r3[q] : r2[q];
    }
    const uint32_t *start = (const uint32_t *)c->tables.p + c->grid.off[c->grid.L_hi];
    launch_scatter(sa, n, &c->sc->n_in, (int)n_total, (const uint32_t *)c->key.p, (const uint32_t *)c->slot.p, start,
                   srt.id, st);
    launch_coarsen((uint32_t *)c->tables.p, c->grid, D, &c->sc->n_total, st, gate);
    stage_mark(c, st, 1, false);
    int ldn = list_ldn(c);
    stage_mark(c, st, 2, true);
    if (reuse) {
        // rebuild steps: the candidates within (1 + skin) r; every step: the exact lists from them
        // (candidate lists interleaved by eight particles: list stride 0)
        launch_search_cand(srt, &c->sc->n_total, (int)n_total, n, (const uint32_t *)c->tables.p, c->grid, c->dc,
                           (int *)c->cand.p, (int *)c->ccount.p, c->sc, c->search_group, reuse_scale(c), gate,
                           &c->sc->max_cand, st);
        launch_filter(srt, &c->sc->n_total, (int)n_total, n, c->dc, (const int *)c->cand.p, 0,
                      (const int *)c->ccount.p, (int *)c->nbr.p, ldn, (int *)c->count.p,
                      (const uint32_t *)c->tables.p, c->grid, c->sc, 8 /* lanes per particle: measured best */,
                      c->search_cap ? c->search_cap : c->search_lcap, (int *)c->fovfq.p,
                      (unsigned long long *)c->octc.p, st);
    } else {
        run_search(c, srt, n_total, n, c->search_cap ? c->search_cap : c->search_lcap, st);
    }
    if (c->solve_mode != 0)
        launch_bin_tiles((const int *)c->count.p, srt.id, &c->sc->n_total, (int)n_total, n, c->dc.max_nb,
                         c->queue_tile, (int *)c->wq.p, st);
    stage_mark(c, st, 2, false);
    stage_mark(c, st, 3, true);
    struct Between { lp_ctx *c; hipStream_t st; } bt{c, st};
    auto between = [](void *arg) {
        Between *b = (Between *)arg;
        stage_mark(b->c, b->st, 3, false);
        stage_mark(b->c, b->st, 4, true);
    };
    SolveArgs sv;
    memset(&sv, 0, sizeof sv);
    sv.srt = srt;
    sv.p = soa;
    sv.nbr = (const int *)c->nbr.p;
    sv.ldn = ldn;
    sv.count = (const int *)c->count.p;
    sv.n_total_dev = &c->sc->n_total;
    sv.n_real = n;
    sv.cfg = c->dc;
    sv.sc = c->sc;
    sv.queue = (int *)c->queue.p;
    sv.octc = reuse ? (const unsigned long long *)c->octc.p : nullptr;
    sv.der = (double *)c->der.p;
    sv.ld = c->cap_total;
    sv.lwst = (uint8_t *)c->lwst.p;
    sv.wq = c->solve_mode != 0 ? (const int *)c->wq.p : nullptr;
    sv.rq = (int *)c->rq.p;
    sv.rkeep = (float *)c->rkeep.p;
    // the network estimator (or a harvest of its inputs) stages the update
    const bool staged = harvest || c->dc.est_mode == LP_EST_MLP;
    if (staged) {
        sv.ms.feat = (float *)c->mfeat.p;
        sv.ms.rates = (double *)c->mrates.p;
        sv.ms.phi_plain = (double *)c->mphi.p;
        sv.ms.mflag = (uint8_t *)c->mflag.p;
        sv.ms.ld = c->cap_total;
        // a step (not a harvest) with the network: the fused kernel applies it where it can
        if (!harvest) sv.ms.theta = (const float *)c->theta.p;
    }
    const bool net_fused = solve_fuses_network(sv, c->solve_mode);
    launch_solve(sv, (int)n_total, c->solve_block, c->solve_mode, +between, &bt, st);
    stage_mark(c, st, 4, false);
    stage_mark(c, st, 5, true);
    launch_solve_fallback(srt, soa, (const int *)c->nbr.p, ldn, (const int *)c->count.p, n, c->dc, c->sc,
                          (const int *)c->queue.p, n, sv.ms, st);
    stage_mark(c, st, 5, false);
    if (harvest) {
        launch_features_out(srt, sv.ms, &c->sc->n_total, n_total, n, harvest->feat, harvest->phi, harvest->valid, st);
        HIPCHK(c, hipGetLastError());
        return LP_OK;  // nothing advanced
    }
    if (staged) {
        stage_mark(c, st, 7, true);
        launch_mlp_apply((const float *)c->theta.p, srt, soa, c->dc, c->sc, n_total, n, sv.ms, net_fused ? 1 : 0,
                         (const int *)c->queue.p, (const int *)c->rq.p, st);
        stage_mark(c, st, 7, false);
    }
    if (c->open) launch_open_end(soa, c->dc, *c->open, c->sc, st);  // lp_run_open: outflow, inflow
    launch_advance_time(c->sc, st);
    HIPCHK(c, hipGetLastError());
    return LP_OK;
}

extern "C" lp_status lp_step(lp_ctx *c, void *stream, const lp_particles *p, double dt) {
    if (!c) return LP_E_ARG;
    lp_status s = check_particles(c, p);
    if (s != LP_OK) return s;
    HIPCHK(c, hipSetDevice(c->device));
    hipStream_t st = (hipStream_t)stream;
    // with reused lists, eager steps also plan the grid with headroom and
    // keep it while it serves (a new grid means new cells and candidates)
    c->grid_margin = reuse_on(c) ? 0.125 : 0.0;
    stage_mark(c, st, LP_STAGE_STEP, true);
    s = step_impl(c, st, p, dt, true, 0);
    stage_mark(c, st, LP_STAGE_STEP, false);
    return s;
}

static lp_status read_scalars(lp_ctx *c, hipStream_t st) {
    HIPCHK(c, hipMemcpyAsync(c->sc_host, c->sc, sizeof(DevScalars), hipMemcpyDeviceToHost, st));
    HIPCHK(c, hipStreamSynchronize(st));
    return LP_OK;
}

// Capture one step of p with the current plan into c->graph (unless the
// graph of the same particle arrays and workspace generation exists).
static lp_status graph_prepare(lp_ctx *c, const lp_particles *p) {
    if (c->graph && c->graph_gen == c->gen && memcmp(&c->graph_p, p, sizeof *p) == 0) return LP_OK;
    if (c->graph) {
        (void)hipGraphExecDestroy(c->graph);
        c->graph = nullptr;
    }
    if (!c->cap_stream) HIPCHK(c, hipStreamCreateWithFlags(&c->cap_stream, hipStreamNonBlocking));
    const bool prof = c->profiling;
    c->profiling = false;  // no event nodes in the graph
    const uint64_t gen0 = c->gen;
    HIPCHK(c, hipStreamBeginCapture(c->cap_stream, hipStreamCaptureModeRelaxed));
    lp_status s = step_impl(c, c->cap_stream, p, 0.0, false, 1);
    hipGraph_t g = nullptr;
    hipError_t e = hipStreamEndCapture(c->cap_stream, &g);
    c->profiling = prof;
    if (s != LP_OK) {
        if (g) (void)hipGraphDestroy(g);
        return s;
    }
    if (e != hipSuccess || !g) return fail(c, LP_E_DEVICE, "graph capture failed: %s", hipGetErrorString(e));
    if (c->gen != gen0) {
        (void)hipGraphDestroy(g);
        return fail(c, LP_E_STATE, "workspace changed during graph capture");
    }
    e = hipGraphInstantiate(&c->graph, g, nullptr, nullptr, 0);
    (void)hipGraphDestroy(g);
    if (e != hipSuccess) {
        c->graph = nullptr;
        return fail(c, LP_E_DEVICE, "hipGraphInstantiate: %s", hipGetErrorString(e));
    }
    c->graph_gen = c->gen;
    c->graph_p = *p;
    ++c->n_captures;
    return LP_OK;
}

#define LP_GRAPH_CHUNK 8

extern "C" lp_status lp_run(lp_ctx *c, void *stream, const lp_particles *p, int32_t nsteps, double t_end) {
    if (!c) return LP_E_ARG;
    lp_status s = check_particles(c, p);
    if (s != LP_OK) return s;
    if (nsteps < 0) return fail(c, LP_E_ARG, "nsteps < 0");
    HIPCHK(c, hipSetDevice(c->device));
    hipStream_t st = (hipStream_t)stream;
    // t_end is kept on the device; each step shortens its dt to land on it
    if ((s = read_scalars(c, st)) != LP_OK) return s;
    c->sc_host->t_end = t_end;
    c->sc_host->done = 0u;
    c->sc_host->halt = 0u;
    HIPCHK(c, hipMemcpyAsync(c->sc, c->sc_host, sizeof(DevScalars), hipMemcpyHostToDevice, st));
    c->run_done = false;
    int64_t steps = 0;
    while (steps < nsteps && !c->run_done) {
        // planning step: sizes the grid (with headroom) and the workspace
        c->grid_margin = 0.125;
        stage_mark(c, st, LP_STAGE_STEP, true);
        s = step_impl(c, st, p, 0.0, true, 1);
        stage_mark(c, st, LP_STAGE_STEP, false);
        if (s != LP_OK) return s;
        if (c->run_done) break;
        if ((s = read_scalars(c, st)) != LP_OK) return s;
        if (c->sc_host->error_bits) break;  // reported by lp_check; later steps would be skipped
        ++steps;
        if (steps >= nsteps) break;
        if ((s = graph_prepare(c, p)) != LP_OK) return s;
        if ((s = read_scalars(c, st)) != LP_OK) return s;
        // replays of the captured step, checked every LP_GRAPH_CHUNK steps
        for (;;) {
            const unsigned long long before = c->sc_host->steps;
            int64_t chunk = nsteps - steps < LP_GRAPH_CHUNK ? nsteps - steps : LP_GRAPH_CHUNK;
            for (int64_t q = 0; q < chunk; ++q) {
                stage_mark(c, st, LP_STAGE_STEP, true);
                HIPCHK(c, hipGraphLaunch(c->graph, st));
                stage_mark(c, st, LP_STAGE_STEP, false);
            }
            if ((s = read_scalars(c, st)) != LP_OK) return s;
            steps += (int64_t)(c->sc_host->steps - before);
            if (c->sc_host->done || (t_end > 0.0 && c->sc_host->t >= t_end)) {
                c->run_done = true;
                break;
            }
            if (c->sc_host->error_bits) {
                c->run_done = true;  // the steps after the failing one were skipped
                break;
            }
            if (steps >= nsteps || c->sc_host->halt || grid_outdated(c)) break;
        }
    }
    c->grid_margin = 0.0;
    return LP_OK;
}

extern "C" lp_status lp_neighbors(lp_ctx *c, void *stream, int64_t n, const double *x, const double *y,
                                  const double *z, const double *r, int32_t *count, int32_t *idx) {
    if (!c) return LP_E_ARG;
    if (n <= 0 || n > (1ll << 30) || !x || !y || (c->dc.D == 3 && !z) || !r || !count || !idx)
        return fail(c, LP_E_ARG, "lp_neighbors: bad arguments");
    HIPCHK(c, hipSetDevice(c->device));
    hipStream_t st = (hipStream_t)stream;
    const int D = c->dc.D;
    ++c->gen;  // the cell arrays are rebuilt here: a step's reused lists and captured graph are outdated
    launch_reset_scalars(c->sc, 0.0, (int)n, 1, st);
    {
        const double *xs[3] = {x, y, c->dc.D == 3 ? z : y};
        launch_rminmax(r, xs, c->dc.D, (int)n, c->sc, st);
    }
    HIPCHK(c, hipMemcpyAsync(c->sc_host, c->sc, sizeof(DevScalars), hipMemcpyDeviceToHost, st));
    HIPCHK(c, hipStreamSynchronize(st));
    choose_levels(c, bits_to_double(c->sc_host->rmin), bits_to_double(c->sc_host->rmax));
    lp_status s = ensure_capacity(c, n, n, false, false);
    if (s != LP_OK) return s;
    const double *xs[3] = {x, y, D == 3 ? z : y};
    const double *gx[3] = {nullptr, nullptr, nullptr};
    build_cells(c, st, xs, gx, (int)n, n);
    Sorted srt = sorted_view(c, false);
    ScatterArgs sa;
    memset(&sa, 0, sizeof sa);
    sa.nd = 4;
    sa.src[0] = x; sa.src[1] = y; sa.src[2] = D == 3 ? z : y; sa.src[3] = r;
    sa.dst[0] = srt.x[0]; sa.dst[1] = srt.x[1]; sa.dst[2] = srt.x[2]; sa.dst[3] = srt.r;
    const uint32_t *start = (const uint32_t *)c->tables.p + c->grid.off[c->grid.L_hi];
    launch_scatter(sa, (int)n, &c->sc->n_in, (int)n, (const uint32_t *)c->key.p, (const uint32_t *)c->slot.p, start,
                   srt.id, st);
    launch_coarsen((uint32_t *)c->tables.p, c->grid, D, &c->sc->n_total, st);
    int ldn = list_ldn(c);
    run_search(c, srt, n, (int)n, c->search_cap, st);
    launch_lists_out(srt.id, (const int *)c->nbr.p, ldn, (const int *)c->count.p, (int)n, c->dc.max_nb, count, idx, st);
    HIPCHK(c, hipGetLastError());
    HIPCHK(c, hipMemcpyAsync(c->sc_host, c->sc, sizeof(DevScalars), hipMemcpyDeviceToHost, st));
    HIPCHK(c, hipStreamSynchronize(st));
    if (c->sc_host->max_count > c->dc.max_nb) return fail(c, LP_E_CAPACITY, "neighbour count %d exceeds max_nb %d",
                                                          c->sc_host->max_count, c->dc.max_nb);
    return LP_OK;
}

extern "C" lp_status lp_neighbors_noalloc(lp_ctx *c, void *stream, int64_t n, const double *x, const double *y,
                                          const double *z, const double *r, int32_t *count, int32_t *idx) {
    if (!c) return LP_E_ARG;
    if (n <= 0 || n > (1ll << 30) || !x || !y || (c->dc.D == 3 && !z) || !r || !count || !idx)
        return fail(c, LP_E_ARG, "lp_neighbors_noalloc: bad arguments");
    int dev = -1;
    HIPCHK(c, hipGetDevice(&dev));
    if (dev != c->device)
        return fail(c, LP_E_STATE, "lp_neighbors_noalloc: device %d is current, the context's is %d", dev, c->device);
    hipError_t serr = hipSuccess;
    void *block = scratch_ptr(c->device, &serr);
    if (!block)
        return fail(c, LP_E_DEVICE, "lp_neighbors_noalloc: no scratch block on device %d (%s)", c->device,
                    hipGetErrorString(serr));
    // swap every workspace buffer out, run lp_neighbors on buffers carved
    // from the scratch block, then put the context's own buffers back
    Buf saved[kNumBufs];
    for (int q = 0; q < kNumBufs; ++q) {
        saved[q] = c->*kBufs[q];
        c->*kBufs[q] = Buf{};
    }
    const int64_t cr = c->cap_real, ct = c->cap_total, cg = c->cap_ghost;
    const DevGrid grid = c->grid;
    const double S_grid = c->S_grid;
    const bool prof = c->profiling;
    char *const arena0 = c->arena;
    const size_t arena_bytes0 = c->arena_bytes, arena_used0 = c->arena_used;
    const lp_status arena_status0 = c->arena_status;
    const bool caller_ws0 = c->caller_ws;
    c->cap_real = c->cap_total = c->cap_ghost = 0;
    c->profiling = false;
    c->arena = (char *)block;
    c->arena_bytes = LP_NOALLOC_SCRATCH_BYTES;
    c->arena_used = 0;
    c->arena_status = LP_E_NOMEM;
    c->caller_ws = false;
    lp_status s = lp_neighbors(c, stream, n, x, y, z, r, count, idx);
    if (s != LP_OK) (void)hipStreamSynchronize((hipStream_t)stream);
    c->arena = arena0;
    c->arena_bytes = arena_bytes0;
    c->arena_used = arena_used0;
    c->arena_status = arena_status0;
    c->caller_ws = caller_ws0;
    for (int q = 0; q < kNumBufs; ++q) c->*kBufs[q] = saved[q];
    c->cap_real = cr;
    c->cap_total = ct;
    c->cap_ghost = cg;
    c->grid = grid;
    c->S_grid = S_grid;
    c->profiling = prof;
    ++c->gen;
    return s;
}

// lp_gfd (order 2) and lp_gfd3 (order 3): cells, search and the fit of the
// given order over the caller's positions and fields
static lp_status gfd_run(lp_ctx *c, void *stream, int64_t n, const double *x, const double *y, const double *z,
                         const double *r, int32_t nf, const double *const *f, double *deriv, uint8_t *status,
                         int order) {
    const char *name = order == 3 ? "lp_gfd3" : "lp_gfd";
    if (!c) return LP_E_ARG;
    if (n <= 0 || n > (1ll << 30) || !x || !y || (c->dc.D == 3 && !z) || !r || !f || nf < 1 || nf > 5 || !deriv ||
        !status)
        return fail(c, LP_E_ARG, "%s: bad arguments", name);
    for (int q = 0; q < nf; ++q)
        if (!f[q]) return fail(c, LP_E_ARG, "%s: null field", name);
    HIPCHK(c, hipSetDevice(c->device));
    hipStream_t st = (hipStream_t)stream;
    const int D = c->dc.D;
    ++c->gen;  // the cell arrays are rebuilt here: a step's reused lists and captured graph are outdated
    launch_reset_scalars(c->sc, 0.0, (int)n, 1, st);
    {
        const double *xs[3] = {x, y, c->dc.D == 3 ? z : y};
        launch_rminmax(r, xs, c->dc.D, (int)n, c->sc, st);
    }
    HIPCHK(c, hipMemcpyAsync(c->sc_host, c->sc, sizeof(DevScalars), hipMemcpyDeviceToHost, st));
    HIPCHK(c, hipStreamSynchronize(st));
    choose_levels(c, bits_to_double(c->sc_host->rmin), bits_to_double(c->sc_host->rmax));
    lp_status s = ensure_capacity(c, n, n, false, false);
    if (s != LP_OK) return s;
    ENSURE(c, c->gfd_fields, sizeof(double) * nf * n);
    const double *xs[3] = {x, y, D == 3 ? z : y};
    const double *gx[3] = {nullptr, nullptr, nullptr};
    stage_mark(c, st, 1, true);
    build_cells(c, st, xs, gx, (int)n, n);
    Sorted srt = sorted_view(c, false);
    ScatterArgs sa;
    memset(&sa, 0, sizeof sa);
    sa.nd = 4 + nf;
    sa.src[0] = x; sa.src[1] = y; sa.src[2] = D == 3 ? z : y; sa.src[3] = r;
    sa.dst[0] = srt.x[0]; sa.dst[1] = srt.x[1]; sa.dst[2] = srt.x[2]; sa.dst[3] = srt.r;
    const double *fs[5];
    for (int q = 0; q < nf; ++q) {
        double *dq = (double *)c->gfd_fields.p + (size_t)q * n;
        sa.src[4 + q] = f[q];
        sa.dst[4 + q] = dq;
        fs[q] = dq;
    }
    if (order == 2 && nf <= D + 2) {
        // gather records for the fit: positions, then the caller's fields
        ENSURE(c, c->srec, sizeof(double) * LP_REC * n);
        srt.rec = (double *)c->srec.p;
        sa.rec = srt.rec;
        const int r3[LP_REC] = {0, 1, 2, 4, 5, 6, 7, 8}, r2[LP_REC] = {0, 1, 4, 5, 6, 7, -1, -1};
        for (int q = 0; q < LP_REC; ++q) {
            const int v = D == 3 ? r3[q] : r2[q];
            sa.rec_src[q] = v < 4 + nf ? v : -1;
        }
    }
    const uint32_t *start = (const uint32_t *)c->tables.p + c->grid.off[c->grid.L_hi];
    launch_scatter(sa, (int)n, &c->sc->n_in, (int)n, (const uint32_t *)c->key.p, (const uint32_t *)c->slot.p, start,
                   srt.id, st);
    launch_coarsen((uint32_t *)c->tables.p, c->grid, D, &c->sc->n_total, st);
    stage_mark(c, st, 1, false);
    int ldn = list_ldn(c);
    stage_mark(c, st, 2, true);
    // list slots in LDS sized from the last call's longest list (a longer
    // list takes the overflow kernel, so the lists are the same either way)
    run_search(c, srt, n, (int)n, c->search_cap ? c->search_cap : c->gfd_lcap, st);
    stage_mark(c, st, 2, false);
    stage_mark(c, st, 3, true);
    if (order == 3) {
        launch_gfd3(srt, fs, nf, (const int *)c->nbr.p, ldn, (const int *)c->count.p, (int)n, c->dc, c->sc,
                    (int *)c->queue.p, deriv, status, st);
    } else {
        launch_gfd(srt, fs, nf, (const int *)c->nbr.p, ldn, (const int *)c->count.p, (int)n, c->dc, c->sc,
                   (int *)c->queue.p, deriv, status, st);
        launch_gfd_fallback(srt, fs, nf, (const int *)c->nbr.p, ldn, (const int *)c->count.p, (int)n, c->dc, c->sc,
                            (const int *)c->queue.p, (int)n, deriv, status, st);
    }
    stage_mark(c, st, 3, false);
    HIPCHK(c, hipGetLastError());
    HIPCHK(c, hipMemcpyAsync(c->sc_host, c->sc, sizeof(DevScalars), hipMemcpyDeviceToHost, st));
    HIPCHK(c, hipStreamSynchronize(st));
    {
        c->gfd_lcap = lds_list_cap(c->sc_host->max_count);
    }
    if (c->sc_host->max_count > c->dc.max_nb) return fail(c, LP_E_CAPACITY, "neighbour count %d exceeds max_nb %d",
                                                          c->sc_host->max_count, c->dc.max_nb);
    return LP_OK;
}

extern "C" lp_status lp_gfd(lp_ctx *c, void *stream, int64_t n, const double *x, const double *y, const double *z,
                            const double *r, int32_t nf, const double *const *f, double *deriv, uint8_t *status) {
    return gfd_run(c, stream, n, x, y, z, r, nf, f, deriv, status, 2);
}

extern "C" lp_status lp_gfd3(lp_ctx *c, void *stream, int64_t n, const double *x, const double *y, const double *z,
                             const double *r, int32_t nf, const double *const *f, double *deriv, uint8_t *status) {
    return gfd_run(c, stream, n, x, y, z, r, nf, f, deriv, status, 3);
}

extern "C" lp_status lp_conservation(lp_ctx *c, void *stream, const lp_particles *p, double *out) {
    if (!c || !out) return LP_E_ARG;
    lp_status s = check_particles(c, p);
    if (s != LP_OK) return s;
    HIPCHK(c, hipSetDevice(c->device));
    hipStream_t st = (hipStream_t)stream;
    const int nblocks = 1024;
    ENSURE(c, c->partials, sizeof(double) * 5 * nblocks);
    ENSURE(c, c->consout, sizeof(double) * 5);
    launch_conservation(soa_of(p), c->dc, (double *)c->partials.p, nblocks, (double *)c->consout.p, st);
    HIPCHK(c, hipMemcpyAsync(out, c->consout.p, sizeof(double) * 5, hipMemcpyDeviceToHost, st));
    HIPCHK(c, hipStreamSynchronize(st));
    return LP_OK;
}

extern "C" lp_status lp_outflow(lp_ctx *c, void *stream, const lp_particles *p, uint32_t lo_mask,
                                uint32_t hi_mask, int64_t *n_kept) {
    if (!c || !n_kept) return LP_E_ARG;
    lp_status s = check_particles(c, p);
    if (s != LP_OK) return s;
    HIPCHK(c, hipSetDevice(c->device));
    hipStream_t st = (hipStream_t)stream;
    const int64_t n = p->n;
    const int D = c->dc.D;
    ENSURE(c, c->gcnt, sizeof(uint32_t) * (n + 1));
    ENSURE(c, c->scan_tmp, sizeof(uint32_t) * scan_tmp_words((uint64_t)n));
    ENSURE(c, c->gfd_fields, out_stage_bytes(D, n));
    uint32_t *pos = (uint32_t *)c->gcnt.p;
    launch_out_keep(soa_of(p), c->dc, lo_mask, hi_mask, pos, st);
    launch_scan_u32(pos, (uint64_t)n, (uint32_t *)c->scan_tmp.p, nullptr, st);
    uint32_t kept = 0;
    HIPCHK(c, hipMemcpyAsync(&kept, pos + n, sizeof(uint32_t), hipMemcpyDeviceToHost, st));
    HIPCHK(c, hipStreamSynchronize(st));
    if ((int64_t)kept < n) {
        // every array through the staging area, then back into the caller's arrays (the mass array
        // too: constant for the step, compacted here)
        launch_out_compact(soa_of(p), D, pos, kept, (double *)c->gfd_fields.p, st);
        HIPCHK(c, hipGetLastError());
    }
    *n_kept = kept;
    return LP_OK;
}

extern "C" lp_status lp_reservoir_inflow(lp_ctx *c, void *stream, const lp_particles *p, int32_t axis, int32_t side,
                                         double width, double p_res, double rho_res, double *out) {
    if (!c || !out) return LP_E_ARG;
    lp_status s = check_particles(c, p);
    if (s != LP_OK) return s;
    if (axis < 0 || axis >= c->dc.D || side < 0 || side > 1 || !(width > 0.0) || !(p_res > 0.0) || !(rho_res > 0.0))
        return fail(c, LP_E_ARG, "lp_reservoir_inflow: bad face, width or reservoir state");
    HIPCHK(c, hipSetDevice(c->device));
    hipStream_t st = (hipStream_t)stream;
    const int nblocks = 256;
    ENSURE(c, c->partials, sizeof(double) * 2 * nblocks);
    ENSURE(c, c->consout, sizeof(double) * 5);
    const double face = side == 0 ? c->dc.lo[axis] : c->dc.hi[axis];
    launch_reservoir(p->x[axis], p->P, (int)p->n, side, face, width, p_res, rho_res, c->dc.gamma,
                     (double *)c->partials.p, nblocks, (double *)c->consout.p, st);
    HIPCHK(c, hipMemcpyAsync(out, c->consout.p, sizeof(double) * 4, hipMemcpyDeviceToHost, st));
    HIPCHK(c, hipStreamSynchronize(st));
    return LP_OK;
}

// Lattice of an inflow layer on the face of `axis`: the other axes oth[0..D-2]
// and the points along each (whole cells of the box, a cell short by rounding
// alone counted; 1 for an absent second axis in 2D).  False when too many.
static bool inflow_lattice(const lp_ctx *c, int axis, double spacing, int oth[2], int64_t cnt[2], int64_t *count) {
    const int D = c->dc.D;
    int no = 0;
    oth[0] = oth[1] = 0;
    cnt[0] = cnt[1] = 1;
    for (int b = 0; b < D; ++b)
        if (b != axis) oth[no++] = b;
    for (int t = 0; t < no; ++t) {
        const double k = floor((c->dc.hi[oth[t]] - c->dc.lo[oth[t]]) / spacing + 1e-9);
        if (!(k <= (double)((int64_t)1 << 30))) return false;
        cnt[t] = (int64_t)k;
    }
    *count = cnt[0] * cnt[1];
    return *count <= ((int64_t)1 << 30);
}

extern "C" lp_status lp_inflow_layer(lp_ctx *c, void *stream, const lp_particles *p, int64_t cap, int32_t axis,
                                     int32_t side, double spacing, double depth, double rho, double p_in, double u_n,
                                     int64_t *n_new) {
    if (!c || !p || !n_new) return LP_E_ARG;
    const int D = c->dc.D;
    if (axis < 0 || axis >= D || side < 0 || side > 1 || !(spacing > 0.0) || !(depth >= 0.0) || !(rho > 0.0) ||
        !(p_in > 0.0) || !isfinite(u_n))
        return fail(c, LP_E_ARG, "lp_inflow_layer: bad face, spacing, depth or state");
    if (p->n < 0 || cap < p->n || cap > ((int64_t)1 << 30)) return fail(c, LP_E_ARG, "lp_inflow_layer: bad n or cap");
    for (int a = 0; a < D; ++a)
        if (!p->x[a] || !p->u[a]) return fail(c, LP_E_ARG, "lp_inflow_layer: null array");
    if (!p->V || !p->P || !p->m) return fail(c, LP_E_ARG, "lp_inflow_layer: null array");
    int oth[2];
    int64_t cnt[2], count;
    if (!inflow_lattice(c, axis, spacing, oth, cnt, &count))
        return fail(c, LP_E_ARG, "lp_inflow_layer: spacing too small");
    if (p->n + count > cap)
        return fail(c, LP_E_CAPACITY, "lp_inflow_layer: %lld particles after the layer, capacity %lld",
                    (long long)(p->n + count), (long long)cap);
    *n_new = p->n + count;
    if (count == 0) return LP_OK;
    HIPCHK(c, hipSetDevice(c->device));
    double mass = rho;
    for (int a = 0; a < D; ++a) mass = mass * spacing;
    const double xa = side == 0 ? c->dc.lo[axis] + depth : c->dc.hi[axis] - depth;
    launch_inflow_layer(soa_of(p), c->dc, p->n, count, cnt[0], axis, oth[0], oth[1], spacing, xa,
                        side == 0 ? u_n : -u_n, 1.0 / rho, p_in, mass, (hipStream_t)stream);
    HIPCHK(c, hipGetLastError());
    return LP_OK;
}

extern "C" lp_status lp_run_open(lp_ctx *c, void *stream, const lp_particles *p, int64_t cap, const lp_open_bc *bc,
                                 int32_t nsteps, double t_end, int64_t *n_out) {
    if (!c || !p || !bc || !n_out) return LP_E_ARG;
    const int D = c->dc.D;
    if (p->n < 1 || cap < p->n || cap > ((int64_t)1 << 30)) return fail(c, LP_E_ARG, "lp_run_open: bad n or cap");
    if (nsteps < 0) return fail(c, LP_E_ARG, "nsteps < 0");
    const uint32_t faces = (1u << D) - 1u;
    if ((bc->out_lo_mask & ~faces) || (bc->out_hi_mask & ~faces))
        return fail(c, LP_E_ARG, "lp_run_open: outflow mask names an axis past the dimension");
    lp_particles q = *p;
    q.n = cap;
    lp_status s = check_particles(c, &q);
    if (s != LP_OK) return s;
    OpenDev o;
    memset(&o, 0, sizeof o);
    o.lo_mask = bc->out_lo_mask;
    o.hi_mask = bc->out_hi_mask;
    o.cap = cap;
    o.res_blocks = 256;
    if (bc->in_every > 0) {
        const bool res = bc->res_width > 0.0;
        if (bc->in_axis < 0 || bc->in_axis >= D || bc->in_side < 0 || bc->in_side > 1 || !(bc->spacing > 0.0) ||
            !(bc->depth >= 0.0) ||
            (res ? !(bc->res_p > 0.0) || !(bc->res_rho > 0.0)
                 : !(bc->rho > 0.0) || !(bc->p_in > 0.0) || !isfinite(bc->u_n)))
            return fail(c, LP_E_ARG, "lp_run_open: bad inflow face, spacing, depth or state");
        int oth[2];
        int64_t cnt[2];
        if (!inflow_lattice(c, bc->in_axis, bc->spacing, oth, cnt, &o.count))
            return fail(c, LP_E_ARG, "lp_run_open: spacing too small");
        o.in_every = bc->in_every;
        o.axis = bc->in_axis;
        o.side = bc->in_side;
        o.o0 = oth[0];
        o.o1 = oth[1];
        o.cnt0 = cnt[0];
        o.spacing = bc->spacing;
        o.xa = bc->in_side == 0 ? c->dc.lo[o.axis] + bc->depth : c->dc.hi[o.axis] - bc->depth;
        if (res) {
            o.res_width = bc->res_width;
            o.res_face = bc->in_side == 0 ? c->dc.lo[o.axis] : c->dc.hi[o.axis];
            o.res_p = bc->res_p;
            o.res_rho = bc->res_rho;
            o.gamma = c->dc.gamma;
        } else {
            // as lp_inflow_layer rounds them
            o.un = bc->in_side == 0 ? bc->u_n : -bc->u_n;
            o.V = 1.0 / bc->rho;
            o.P = bc->p_in;
            double mass = bc->rho;
            for (int a = 0; a < D; ++a) mass = mass * bc->spacing;
            o.mass = mass;
        }
    }
    HIPCHK(c, hipSetDevice(c->device));
    hipStream_t st = (hipStream_t)stream;
    if (o.res_width > 0.0) {
        ENSURE(c, c->openres, sizeof(double) * (2 * o.res_blocks + 4));
        o.res_part = (double *)c->openres.p;
    }
    // the slots past p->n are absent until a layer fills them
    if (cap > p->n) launch_fill_u32((uint32_t *)(p->m + p->n), 2 * (uint64_t)(cap - p->n), 0u, st);
    if ((s = read_scalars(c, st)) != LP_OK) return s;
    c->sc_host->n_hw = (int)p->n;
    c->sc_host->open_k = 0ull;
    c->sc_host->insert_now = 0u;
    c->sc_host->pop_changed = 1u;  // lists built for other particles do not serve
    HIPCHK(c, hipMemcpyAsync(c->sc, c->sc_host, sizeof(DevScalars), hipMemcpyHostToDevice, st));
    // a graph of plain steps must not serve, nor this one outlive the call
    ++c->gen;
    c->open = &o;
    const lp_status s_run = lp_run(c, stream, &q, nsteps, t_end);
    c->open = nullptr;
    ++c->gen;
    // compaction of the slots in use (also after a failed run): present
    // particles keep their order
    if ((s = read_scalars(c, st)) != LP_OK) return s_run != LP_OK ? s_run : s;
    const int64_t n = c->sc_host->n_hw;
    ENSURE(c, c->gcnt, sizeof(uint32_t) * (n + 1));
    ENSURE(c, c->scan_tmp, sizeof(uint32_t) * scan_tmp_words((uint64_t)n));
    // staging of the compaction: the cell-order arrays, which every step
    // refills from the caller's arrays, when the run left them large enough
    double *stage = nullptr;
    if (c->sorted.p && c->sorted.bytes >= out_stage_bytes(D, n)) {
        stage = (double *)c->sorted.p;
    } else {
        ENSURE(c, c->gfd_fields, out_stage_bytes(D, n));
        stage = (double *)c->gfd_fields.p;
    }
    lp_particles r = q;
    r.n = n;
    uint32_t *pos = (uint32_t *)c->gcnt.p;
    launch_alive_keep(soa_of(&r), pos, st);
    launch_scan_u32(pos, (uint64_t)n, (uint32_t *)c->scan_tmp.p, nullptr, st);
    uint32_t kept = 0;
    HIPCHK(c, hipMemcpyAsync(&kept, pos + n, sizeof(uint32_t), hipMemcpyDeviceToHost, st));
    HIPCHK(c, hipStreamSynchronize(st));
    if ((int64_t)kept < n) {
        launch_out_compact(soa_of(&r), D, pos, kept, stage, st);
        HIPCHK(c, hipGetLastError());
    }
    *n_out = kept;
    return s_run;
}

extern "C" lp_status lp_check(lp_ctx *c, void *stream) {
    if (!c) return LP_E_ARG;
    HIPCHK(c, hipSetDevice(c->device));
    hipStream_t st = (hipStream_t)stream;
    HIPCHK(c, hipStreamSynchronize(st));
    HIPCHK(c, hipGetLastError());
    HIPCHK(c, hipMemcpy(c->sc_host, c->sc, sizeof(DevScalars), hipMemcpyDeviceToHost));
    unsigned bits = c->sc_host->error_bits;
    if (bits) {
        c->sc_host->error_bits = 0;
        HIPCHK(c, hipMemcpy(&c->sc->error_bits, &c->sc_host->error_bits, sizeof(unsigned), hipMemcpyHostToDevice));
    }
    if (bits & 1u) return fail(c, LP_E_CAPACITY, "a neighbour list exceeded max_nb = %d", c->dc.max_nb);
    if (bits & 2u) return fail(c, LP_E_NUMERIC, "non-positive V or P after an update");
    if (bits & 4u) return fail(c, LP_E_CAPACITY, "lp_run_open: an inflow layer did not fit in cap");
    return LP_OK;
}

extern "C" lp_status lp_get_info(lp_ctx *c, void *stream, lp_info *out) {
    if (!c || !out) return LP_E_ARG;
    HIPCHK(c, hipSetDevice(c->device));
    hipStream_t st = (hipStream_t)stream;
    HIPCHK(c, hipMemcpyAsync(c->sc_host, c->sc, sizeof(DevScalars), hipMemcpyDeviceToHost, st));
    HIPCHK(c, hipStreamSynchronize(st));
    memset(out, 0, sizeof *out);
    out->t = c->sc_host->t;
    out->dt = c->sc_host->dt;
    out->n_ghost = c->sc_host->n_ghost;
    out->max_count = c->sc_host->max_count;
    out->n_fallback = c->sc_host->n_fallback;
    out->n_limited = (int64_t)c->sc_host->n_limited;
    out->error_bits = c->sc_host->error_bits;
    out->levels[0] = c->last_levels[0];
    out->levels[1] = c->last_levels[1];
    out->n_mlp = (int64_t)c->sc_host->n_mlp;
    out->n_mlp_plain = (int64_t)c->sc_host->n_mlp_plain;
    out->n_refined = c->sc_host->n_refine;
    out->n_list_builds = (int64_t)c->sc_host->n_builds;
    out->n_captures = c->n_captures;
    return LP_OK;
}

extern "C" lp_status lp_set_time(lp_ctx *c, void *stream, double t) {
    if (!c) return LP_E_ARG;
    HIPCHK(c, hipSetDevice(c->device));
    hipStream_t st = (hipStream_t)stream;
    HIPCHK(c, hipMemcpyAsync(c->sc_host, c->sc, sizeof(DevScalars), hipMemcpyDeviceToHost, st));
    HIPCHK(c, hipStreamSynchronize(st));
    c->sc_host->t = t;
    HIPCHK(c, hipMemcpyAsync(c->sc, c->sc_host, sizeof(DevScalars), hipMemcpyHostToDevice, st));
    HIPCHK(c, hipStreamSynchronize(st));
    return LP_OK;
}

extern "C" lp_status lp_profile(lp_ctx *c, int32_t enable) {
    if (!c) return LP_E_ARG;
    c->profiling = enable != 0;
    if (c->profiling) {
        c->recs.clear();
        c->ev_used = 0;
    }
    return LP_OK;
}

extern "C" lp_status lp_profile_read(lp_ctx *c, void *stream, double *ms, int64_t *count) {
    if (!c || !ms || !count) return LP_E_ARG;
    HIPCHK(c, hipSetDevice(c->device));
    HIPCHK(c, hipStreamSynchronize((hipStream_t)stream));
    for (int q = 0; q < LP_NSTAGES; ++q) { ms[q] = 0.0; count[q] = 0; }
    for (const auto &r : c->recs) {
        if (!r.b || r.stage < 0 || r.stage >= LP_NSTAGES) continue;
        float t = 0.f;
        if (hipEventElapsedTime(&t, r.a, r.b) == hipSuccess) {
            ms[r.stage] += t;
            count[r.stage] += 1;
        }
    }
    c->recs.clear();
    c->ev_used = 0;
    return LP_OK;
}

extern "C" lp_status lp_set_tuning(lp_ctx *c, int32_t param, int32_t value) {
    if (!c) return LP_E_ARG;
    int *field = nullptr;
    switch (param) {
    case LP_TUNE_SEARCH_MODE:
        if (value < 0 || value > 2) return fail(c, LP_E_ARG, "search mode must be 0, 1 or 2");
        field = &c->search_mode;
        break;
    case LP_TUNE_SEARCH_GROUP:
        if (value != 4 && value != 8 && value != 16 && value != 32) return fail(c, LP_E_ARG, "group must be 4..32");
        field = &c->search_group;
        break;
    case LP_TUNE_SOLVE_BLOCK:
        if (value != 64 && value != 128 && value != 256) return fail(c, LP_E_ARG, "solve block must be 64..256");
        field = &c->solve_block;
        break;
    case LP_TUNE_SOLVE_MODE:
        if (value < 0 || value > 2) return fail(c, LP_E_ARG, "solve mode must be 0, 1 or 2");
        field = &c->solve_mode;
        break;
    case LP_TUNE_QUEUE_TILE:
        if (value != 256 && value != 512 && value != 1024) return fail(c, LP_E_ARG, "queue tile must be 256, 512 or 1024");
        field = &c->queue_tile;
        break;
    case LP_TUNE_SEARCH_CAP:
        if (value != 0 && (value < 8 || value > 128 || value % 8 != 0))
            return fail(c, LP_E_ARG, "search cap must be 0 or a multiple of 8 in 8..128");
        field = &c->search_cap;
        break;
    case LP_TUNE_LIST_SKIN:
        if (value < 0 || value > 1000) return fail(c, LP_E_ARG, "list skin must be in 0..1000 (per mille of r)");
        field = &c->list_skin;
        break;
    default:
        return fail(c, LP_E_ARG, "unknown tuning parameter %d", param);
    }
    if (*field != value) {
        *field = value;
        ++c->gen;  // a captured step holds the old launch shapes
    }
    return LP_OK;
}

extern "C" lp_status lp_get_tuning(const lp_ctx *c, int32_t param, int32_t *value) {
    if (!c || !value) return LP_E_ARG;
    switch (param) {
    case LP_TUNE_SEARCH_MODE: *value = c->search_mode; return LP_OK;
    case LP_TUNE_SEARCH_GROUP: *value = c->search_group; return LP_OK;
    case LP_TUNE_SOLVE_BLOCK: *value = c->solve_block; return LP_OK;
    case LP_TUNE_SOLVE_MODE: *value = c->solve_mode; return LP_OK;
    case LP_TUNE_LIST_SKIN: *value = c->list_skin; return LP_OK;
    case LP_TUNE_QUEUE_TILE: *value = c->queue_tile; return LP_OK;
    case LP_TUNE_SEARCH_CAP: *value = c->search_cap; return LP_OK;
    default: return LP_E_ARG;
    }
}

// ---------------------------------------------------------------------------
// Autotuner: coordinate descent over the launch-shape parameters, each
// candidate timed on full steps of a private copy of the particle state.
// ---------------------------------------------------------------------------
extern "C" lp_status lp_autotune(lp_ctx *c, void *stream, const lp_particles *p, int32_t reps, int32_t *best,
                                 double *ms_out) {
    if (!c) return LP_E_ARG;
    lp_status s = check_particles(c, p);
    if (s != LP_OK) return s;
    if (reps < 1) reps = 3;
    HIPCHK(c, hipSetDevice(c->device));
    hipStream_t st = (hipStream_t)stream;
    const int D = c->dc.D;
    const int64_t n = p->n;
    const int narr = 2 * D + 2;
    double *buf = nullptr;
    if (hipMalloc(&buf, sizeof(double) * narr * n) != hipSuccess) {
        (void)hipGetLastError();
        return fail(c, LP_E_NOMEM, "autotune: no room for a copy of the state");
    }
    lp_particles q = *p;
    const double *src[8];
    double *dst[8];
    int k = 0;
    for (int a = 0; a < D; ++a) { q.x[a] = buf + (int64_t)k * n; src[k] = p->x[a]; dst[k++] = q.x[a]; }
    for (int a = 0; a < D; ++a) { q.u[a] = buf + (int64_t)k * n; src[k] = p->u[a]; dst[k++] = q.u[a]; }
    q.V = buf + (int64_t)k * n; src[k] = p->V; dst[k++] = q.V;
    q.P = buf + (int64_t)k * n; src[k] = p->P; dst[k++] = q.P;
    q.phi = c->dc.est_mode == LP_EST_INJECTED ? p->phi : nullptr;
    q.flags = nullptr;
    hipEvent_t e0 = nullptr, e1 = nullptr;
    const bool prof = c->profiling;
    c->profiling = false;
    // the candidate steps run on a private copy of the particles but through
    // the context's device scalars (clock, dt, counters, sticky error bits):
    // all of them are put back afterwards, on success and on failure alike
    DevScalars saved;
    bool have_saved = false;
    auto cleanup = [&]() {
        if (e0) (void)hipEventDestroy(e0);
        if (e1) (void)hipEventDestroy(e1);
        (void)hipStreamSynchronize(st);
        if (have_saved) {
            *c->sc_host = saved;
            (void)hipMemcpyAsync(c->sc, c->sc_host, sizeof(DevScalars), hipMemcpyHostToDevice, st);
            (void)hipStreamSynchronize(st);
        }
        (void)hipFree(buf);
        c->profiling = prof;
    };
    auto run_candidate = [&](double &ms) -> lp_status {
        // the grid policy of lp_step (headroom, kept while it serves, when lists are reused)
        c->grid_margin = reuse_on(c) ? 0.125 : 0.0;
        for (int a = 0; a < narr; ++a)
            HIPCHK(c, hipMemcpyAsync(dst[a], src[a], sizeof(double) * n, hipMemcpyDeviceToDevice, st));
        lp_status r = step_impl(c, st, &q, 0.0, true, 0);  // warm-up (plans and allocates)
        if (r != LP_OK) return r;
        HIPCHK(c, hipEventRecord(e0, st));
        for (int i = 0; i < reps; ++i) {
            r = step_impl(c, st, &q, 0.0, true, 0);
            if (r != LP_OK) return r;
        }
        HIPCHK(c, hipEventRecord(e1, st));
        HIPCHK(c, hipEventSynchronize(e1));
        float t = 0.f;
        HIPCHK(c, hipEventElapsedTime(&t, e0, e1));
        ms = (double)t / reps;
        // a candidate's capacity or numeric error is autotune's own failure
        r = read_scalars(c, st);
        if (r != LP_OK) return r;
        if (c->sc_host->error_bits & 1u)
            return fail(c, LP_E_CAPACITY, "lp_autotune: a candidate step exceeded max_nb = %d", c->dc.max_nb);
        if (c->sc_host->error_bits & 2u)
            return fail(c, LP_E_NUMERIC, "lp_autotune: a candidate step left a non-positive V or P");
        return LP_OK;
    };
    auto body = [&]() -> lp_status {
        HIPCHK(c, hipEventCreate(&e0));
        HIPCHK(c, hipEventCreate(&e1));
        lp_status r = read_scalars(c, st);
        if (r != LP_OK) return r;
        saved = *c->sc_host;
        have_saved = true;
        c->grid_margin = 0.0;
        struct Param { int id; std::vector<int> values; };
        // (not the list skin: a few steps from one state cannot see how often a run rebuilds)
        std::vector<Param> params = {{LP_TUNE_SOLVE_MODE, {0, 1, 2}},
                                     {LP_TUNE_QUEUE_TILE, {256, 512, 1024}},
                                     {LP_TUNE_SOLVE_BLOCK, {64, 128, 256}},
                                     {LP_TUNE_SEARCH_MODE, {0, 1, 2}},
                                     {LP_TUNE_SEARCH_GROUP, {4, 8, 16, 32}}};
        double best_ms = 0.0;
        r = run_candidate(best_ms);
        if (r != LP_OK) return r;
        for (const Param &pr : params) {
            int32_t cur = 0;
            (void)lp_get_tuning(c, pr.id, &cur);
            int chosen = cur;
            for (int v : pr.values) {
                if (v == cur) continue;
                if (pr.id == LP_TUNE_SEARCH_GROUP && c->search_mode == 1) continue;
                if (pr.id == LP_TUNE_QUEUE_TILE && c->solve_mode == 0) continue;
                r = lp_set_tuning(c, pr.id, v);
                if (r != LP_OK) return r;
                double ms = 0.0;
                r = run_candidate(ms);
                if (r != LP_OK) return r;
                if (ms < best_ms) { best_ms = ms; chosen = v; }
            }
            r = lp_set_tuning(c, pr.id, chosen);
            if (r != LP_OK) return r;
        }
        if (best)
            for (int id = 0; id < LP_TUNE_COUNT; ++id) (void)lp_get_tuning(c, id, &best[id]);
        if (ms_out) *ms_out = best_ms;
        return LP_OK;
    };
    s = body();
    cleanup();
    return s;
}

// ---------------------------------------------------------------------------
// Estimator network
// ---------------------------------------------------------------------------
extern "C" void lp_train_cfg_default(lp_train_cfg *cfg) {
    memset(cfg, 0, sizeof *cfg);
    cfg->epochs = 10;
    cfg->batch = 4096;
    cfg->lr = 2e-3f;
    cfg->beta1 = 0.9f;
    cfg->beta2 = 0.999f;
    cfg->eps = 1e-8f;
    cfg->seed = 1;
}

extern "C" lp_status lp_features(lp_ctx *c, void *stream, const lp_particles *p, float *feat, float *phi,
                                 uint8_t *valid) {
    if (!c) return LP_E_ARG;
    if (!p || p->n <= 0 || p->n > (1ll << 30) || !feat || !phi) return fail(c, LP_E_ARG, "lp_features: bad arguments");
    for (int a = 0; a < c->dc.D; ++a)
        if (!p->x[a] || !p->u[a]) return fail(c, LP_E_ARG, "null position/velocity array");
    if (!p->V || !p->P || !p->m) return fail(c, LP_E_ARG, "null V, P or m");
    HIPCHK(c, hipSetDevice(c->device));
    c->want_stage = true;
    c->grid_margin = 0.0;
    lp_features_out out{feat, phi, valid};
    lp_particles q = *p;
    q.phi = nullptr;  // nothing is written to the particles
    q.flags = nullptr;
    return step_impl(c, (hipStream_t)stream, &q, 0.0, true, 0, &out);
}

// splitmix64: a counter-based generator for the initial weights
static uint64_t splitmix64(uint64_t &x) {
    uint64_t z = (x += 0x9e3779b97f4a7c15ull);
    z = (z ^ (z >> 30)) * 0xbf58476d1ce4e5b9ull;
    z = (z ^ (z >> 27)) * 0x94d049bb133111ebull;
    return z ^ (z >> 31);
}

static lp_status mlp_alloc(lp_ctx *c) {
    ENSURE(c, c->theta, sizeof(float) * LP_MLP_NPARAM);
    ENSURE(c, c->adam_m, sizeof(float) * LP_MLP_NPARAM);
    ENSURE(c, c->adam_v, sizeof(float) * LP_MLP_NPARAM);
    ENSURE(c, c->mgrad, sizeof(float) * LP_MLP_NPARAM);
    return LP_OK;
}

// ---------------------------------------------------------------------------
// Caller-owned workspace
// ---------------------------------------------------------------------------
extern "C" lp_status lp_workspace_bytes(lp_ctx *c, void *stream, const lp_particles *p, int64_t *bytes) {
    if (!c || !bytes) return LP_E_ARG;
    lp_status s = check_particles(c, p);
    if (s != LP_OK) return s;
    HIPCHK(c, hipSetDevice(c->device));
    hipStream_t st = (hipStream_t)stream;
    const int n = (int)p->n;
    const bool mixed = c->dc.precision == LP_MIXED;
    // the planning part of a step: radii, time-step bound, ghost count, grid
    ENSURE(c, c->h, sizeof(double) * n);
    ENSURE(c, c->r, sizeof(double) * n);
    ENSURE(c, c->gcnt, sizeof(uint32_t) * (n + 1));
    ENSURE(c, c->scan_tmp, sizeof(uint32_t) * scan_tmp_words(n));
    ENSURE(c, c->prep_part, sizeof(double) * prep_partial_words(n));
    Soa soa = soa_of(p);
    launch_reset_scalars(c->sc, 0.0, n, 1, st);
    launch_prep(soa, c->dc, c->sc, (double *)c->h.p, (double *)c->r.p, (double *)c->prep_part.p, st);
    if (c->nwalls) {
        launch_ghost_count(soa, c->dc, c->sc, (uint32_t *)c->gcnt.p, st);
        launch_scan_u32((uint32_t *)c->gcnt.p, n, (uint32_t *)c->scan_tmp.p, &c->sc->n_ghost, st);
    }
    HIPCHK(c, hipGetLastError());
    if ((s = read_scalars(c, st)) != LP_OK) return s;
    const double margin0 = c->grid_margin;
    c->grid_margin = 0.125;  // lp_run's headroom
    choose_levels(c, bits_to_double(c->sc_host->rmin), bits_to_double(c->sc_host->rmax));
    c->grid_margin = margin0;
    const int64_t ng = c->sc_host->n_ghost;
    const int64_t want = c->nwalls ? n + ng + ng / 4 + 1024 : n;
    // every buffer a step (eager or replayed) of these particles carves, from an empty workspace
    const int64_t cr = c->cap_real, ct = c->cap_total, cg = c->cap_ghost;
    c->cap_real = c->cap_total = c->cap_ghost = 0;
    c->measure = true;
    c->measure_bytes = 0;
    (void)ensure(c, c->h, sizeof(double) * n);
    (void)ensure(c, c->r, sizeof(double) * n);
    (void)ensure(c, c->gcnt, sizeof(uint32_t) * (n + 1));
    (void)ensure(c, c->scan_tmp, sizeof(uint32_t) * scan_tmp_words(n));
    (void)ensure(c, c->prep_part, sizeof(double) * prep_partial_words(n));
    (void)ensure_capacity(c, n, want, true, mixed);
    if (c->mlp_ready || c->dc.est_mode == LP_EST_MLP) (void)mlp_alloc(c);
    (void)ensure(c, c->openres, sizeof(double) * (2 * 256 + 4));  // lp_run_open's reservoir sums
    c->measure = false;
    c->cap_real = cr;
    c->cap_total = ct;
    c->cap_ghost = cg;
    *bytes = (int64_t)c->measure_bytes + 256;
    return LP_OK;
}

extern "C" lp_status lp_set_workspace(lp_ctx *c, void *stream, void *dev, int64_t bytes) {
    if (!c) return LP_E_ARG;
    if (dev && (bytes < 256 || ((uintptr_t)dev & 255u) != 0))
        return fail(c, LP_E_ARG, "lp_set_workspace: the block must be 256-byte aligned and at least 256 bytes");
    HIPCHK(c, hipSetDevice(c->device));
    HIPCHK(c, hipStreamSynchronize((hipStream_t)stream));
    // the network's parameters and optimiser moments outlive the move
    std::vector<float> keep;
    const bool have = c->mlp_ready && c->theta.p && c->adam_m.p && c->adam_v.p;
    if (have) {
        keep.resize(3 * (size_t)LP_MLP_NPARAM);
        HIPCHK(c, hipMemcpy(keep.data(), c->theta.p, sizeof(float) * LP_MLP_NPARAM, hipMemcpyDeviceToHost));
        HIPCHK(c, hipMemcpy(keep.data() + LP_MLP_NPARAM, c->adam_m.p, sizeof(float) * LP_MLP_NPARAM,
                            hipMemcpyDeviceToHost));
        HIPCHK(c, hipMemcpy(keep.data() + 2 * LP_MLP_NPARAM, c->adam_v.p, sizeof(float) * LP_MLP_NPARAM,
                            hipMemcpyDeviceToHost));
    }
    for (int q = 0; q < kNumBufs; ++q) {
        Buf &b = c->*kBufs[q];
        if (b.p && b.owned) (void)hipFree(b.p);
        b = Buf{};
    }
    c->cap_real = c->cap_total = c->cap_ghost = 0;
    c->arena = (char *)dev;
    c->arena_bytes = dev ? (size_t)bytes : 0;
    c->arena_used = 0;
    c->arena_status = LP_E_CAPACITY;
    c->caller_ws = dev != nullptr;
    ++c->gen;
    if (have) {
        lp_status s = mlp_alloc(c);
        if (s != LP_OK) return s;
        HIPCHK(c, hipMemcpy(c->theta.p, keep.data(), sizeof(float) * LP_MLP_NPARAM, hipMemcpyHostToDevice));
        HIPCHK(c, hipMemcpy(c->adam_m.p, keep.data() + LP_MLP_NPARAM, sizeof(float) * LP_MLP_NPARAM,
                            hipMemcpyHostToDevice));
        HIPCHK(c, hipMemcpy(c->adam_v.p, keep.data() + 2 * LP_MLP_NPARAM, sizeof(float) * LP_MLP_NPARAM,
                            hipMemcpyHostToDevice));
    }
    return LP_OK;
}

extern "C" lp_status lp_mlp_set(lp_ctx *c, const float *params, int64_t count) {
    if (!c) return LP_E_ARG;
    if (!params || count != LP_MLP_NPARAM) return fail(c, LP_E_ARG, "lp_mlp_set: need %d parameters", LP_MLP_NPARAM);
    HIPCHK(c, hipSetDevice(c->device));
    lp_status s = mlp_alloc(c);
    if (s != LP_OK) return s;
    HIPCHK(c, hipMemcpy(c->theta.p, params, sizeof(float) * LP_MLP_NPARAM, hipMemcpyHostToDevice));
    c->mlp_ready = true;
    return LP_OK;
}

extern "C" lp_status lp_mlp_get(lp_ctx *c, float *params, int64_t count) {
    if (!c) return LP_E_ARG;
    if (!params || count != LP_MLP_NPARAM) return fail(c, LP_E_ARG, "lp_mlp_get: need %d parameters", LP_MLP_NPARAM);
    if (!c->mlp_ready) return fail(c, LP_E_STATE, "estimator network has no parameters");
    HIPCHK(c, hipSetDevice(c->device));
    HIPCHK(c, hipDeviceSynchronize());
    HIPCHK(c, hipMemcpy(params, c->theta.p, sizeof(float) * LP_MLP_NPARAM, hipMemcpyDeviceToHost));
    return LP_OK;
}

extern "C" lp_status lp_mlp_init(lp_ctx *c, uint64_t seed) {
    if (!c) return LP_E_ARG;
    std::vector<float> th(LP_MLP_NPARAM, 0.0f);
    uint64_t state = seed;
    auto uniform = [&](double bound) {
        double u = (double)(splitmix64(state) >> 11) * (1.0 / 9007199254740992.0);  // [0, 1)
        return (float)((2.0 * u - 1.0) * bound);
    };
    const int nin = LP_MLP_NIN, nh = 64;
    const int off_w1 = 0, off_w2 = nh * nin + nh, off_w3 = off_w2 + nh * nh + nh;
    for (int q = 0; q < nh * nin; ++q) th[off_w1 + q] = uniform(sqrt(6.0 / nin));
    for (int q = 0; q < nh * nh; ++q) th[off_w2 + q] = uniform(sqrt(6.0 / nh));
    for (int q = 0; q < nh; ++q) th[off_w3 + q] = uniform(sqrt(6.0 / nh));
    return lp_mlp_set(c, th.data(), LP_MLP_NPARAM);
}

extern "C" lp_status lp_mlp_forward(lp_ctx *c, void *stream, int64_t n, const float *feat, float *z, float *y) {
    if (!c) return LP_E_ARG;
    if (n < 0 || (n > 0 && !feat)) return fail(c, LP_E_ARG, "lp_mlp_forward: bad arguments");
    if (!c->mlp_ready) return fail(c, LP_E_STATE, "estimator network has no parameters");
    if (n == 0) return LP_OK;
    HIPCHK(c, hipSetDevice(c->device));
    launch_mlp_forward((const float *)c->theta.p, n, feat, z, y, (hipStream_t)stream);
    HIPCHK(c, hipGetLastError());
    return LP_OK;
}

static lp_status mlp_train_buffers(lp_ctx *c, int64_t batch, int epochs) {
    lp_status s = mlp_alloc(c);
    if (s != LP_OK) return s;
    ENSURE(c, c->mpart, sizeof(float) * (size_t)mlp_grad_blocks(batch) * LP_MLP_NPARAM);
    ENSURE(c, c->mlosspart, sizeof(float) * (size_t)mlp_grad_blocks(batch));
    ENSURE(c, c->mscal, sizeof(float) * (size_t)(2 + (epochs > 0 ? epochs : 0)));
    return LP_OK;
}

extern "C" lp_status lp_mlp_grad(lp_ctx *c, void *stream, int64_t n, const float *feat, const float *target,
                                 float *grad, float *loss) {
    if (!c) return LP_E_ARG;
    if (n <= 0 || !feat || !target || !grad) return fail(c, LP_E_ARG, "lp_mlp_grad: bad arguments");
    if (!c->mlp_ready) return fail(c, LP_E_STATE, "estimator network has no parameters");
    HIPCHK(c, hipSetDevice(c->device));
    hipStream_t st = (hipStream_t)stream;
    lp_status s = mlp_train_buffers(c, n, 0);
    if (s != LP_OK) return s;
    float *scal = (float *)c->mscal.p;
    launch_mlp_grad((const float *)c->theta.p, 0, n, feat, target, (float *)c->mpart.p, (float *)c->mlosspart.p,
                    (float *)c->mgrad.p, scal, st);
    HIPCHK(c, hipGetLastError());
    HIPCHK(c, hipMemcpyAsync(grad, c->mgrad.p, sizeof(float) * LP_MLP_NPARAM, hipMemcpyDeviceToHost, st));
    float l = 0.f;
    HIPCHK(c, hipMemcpyAsync(&l, scal, sizeof(float), hipMemcpyDeviceToHost, st));
    HIPCHK(c, hipStreamSynchronize(st));
    if (loss) *loss = l;
    return LP_OK;
}

extern "C" lp_status lp_mlp_train(lp_ctx *c, void *stream, int64_t n, const float *feat, const float *target,
                                  const lp_train_cfg *cfg, float *loss) {
    if (!c) return LP_E_ARG;
    if (n <= 0 || !feat || !target || !cfg) return fail(c, LP_E_ARG, "lp_mlp_train: bad arguments");
    if (cfg->epochs < 0 || cfg->batch < 16 || !(cfg->lr > 0.f) || !(cfg->beta1 >= 0.f && cfg->beta1 < 1.f) ||
        !(cfg->beta2 >= 0.f && cfg->beta2 < 1.f) || !(cfg->eps > 0.f))
        return fail(c, LP_E_ARG, "lp_mlp_train: bad training configuration");
    if (!c->mlp_ready) return fail(c, LP_E_STATE, "estimator network has no parameters");
    HIPCHK(c, hipSetDevice(c->device));
    hipStream_t st = (hipStream_t)stream;
    const int64_t batch = cfg->batch < n ? cfg->batch : n;
    lp_status s = mlp_train_buffers(c, batch, cfg->epochs);
    if (s != LP_OK) return s;
    float *scal = (float *)c->mscal.p;  // [0] batch loss, [1] unused, [2 + e] summed batch losses of epoch e
    launch_fill_f32((float *)c->adam_m.p, LP_MLP_NPARAM, 0.f, st);
    launch_fill_f32((float *)c->adam_v.p, LP_MLP_NPARAM, 0.f, st);
    launch_fill_f32(scal, 2 + cfg->epochs, 0.f, st);
    const int64_t nbatch = (n + batch - 1) / batch;
    std::vector<int64_t> order((size_t)nbatch);
    uint64_t rng = cfg->seed;
    int t = 0;
    for (int e = 0; e < cfg->epochs; ++e) {
        for (int64_t b = 0; b < nbatch; ++b) order[(size_t)b] = b;
        for (int64_t b = nbatch - 1; b > 0; --b) {  // Fisher-Yates
            int64_t q = (int64_t)(splitmix64(rng) % (uint64_t)(b + 1));
            std::swap(order[(size_t)b], order[(size_t)q]);
        }
        for (int64_t b = 0; b < nbatch; ++b) {
            const int64_t b0 = order[(size_t)b] * batch;
            const int64_t nb = n - b0 < batch ? n - b0 : batch;
            launch_mlp_grad((const float *)c->theta.p, b0, nb, feat, target, (float *)c->mpart.p,
                            (float *)c->mlosspart.p, (float *)c->mgrad.p, scal, st);
            launch_mlp_adam((float *)c->theta.p, (float *)c->adam_m.p, (float *)c->adam_v.p,
                            (const float *)c->mgrad.p, cfg->lr, cfg->beta1, cfg->beta2, cfg->eps, ++t, scal,
                            scal + 2 + e, st);
        }
    }
    HIPCHK(c, hipGetLastError());
    if (loss && cfg->epochs > 0) {
        std::vector<float> acc((size_t)cfg->epochs);
        HIPCHK(c, hipMemcpyAsync(acc.data(), scal + 2, sizeof(float) * cfg->epochs, hipMemcpyDeviceToHost, st));
        HIPCHK(c, hipStreamSynchronize(st));
        for (int e = 0; e < cfg->epochs; ++e) loss[e] = acc[(size_t)e] / (float)nbatch;
    }
    HIPCHK(c, hipStreamSynchronize(st));
    return LP_OK;
}
