// lp_solve.hip -- the fused per-particle solver of the LP step on gfx950:
// stencils (Sec. 2.2, step 4), GFD fits (Sec. 2.1), state estimator and
// limiter, blended upwind / Lax-Wendroff update, EOS and particle mover
// (Sec. 2.1; Sec. 2.2 steps 5-6).
//
// Fast path (k_lw_fit + k_finish): one thread per particle.  The second-order fit is solved
// through the R factor of its QR decomposition obtained from the Cholesky
// factor of the normal matrix (R^T R = A^T A) -- the rows of the scaled
// stencil matrix stream through registers once, so the whole fit costs one
// pass over the neighbour list, with no cross-lane traffic and no scratch
// memory.  A condition estimate ||R||_F^2 ||R^-1||_F^2 of the normal matrix
// routes every stencil for which this is not accurate to the FP64
// pivoted-Householder path.  The fit writes its derivatives to a SoA array and
// a second kernel (k_finish) does the half-ball fits, the estimator and the
// update; splitting keeps each kernel's register count low enough for two to
// four waves per SIMD.
//
// Fallback (k_solve_fallback): one wave per particle, one stencil row per lane;
// Householder QR with column pivoting (the paper's solver) with all column
// norms and reflector products formed by wave-wide butterfly reductions.
// It applies the same rank-deficiency rule as the definition (|R11|/|Rnn|).
#include "lp_mlp.h"

// Multiply-adds are fused only inside one source expression, never across
// statements, so that every kernel instantiating the same fit code rounds it
// the same way (the adaptive refinement relies on the FP32 fit of one kernel
// reproducing the other's bit for bit).
#pragma clang fp contract(on)

template <int D> struct Dim;
template <> struct Dim<3> { static constexpr int NU = 9, NF = 5, NS = 6, NG = 45; };
template <> struct Dim<2> { static constexpr int NU = 5, NF = 4, NS = 3, NG = 15; };
// what an FP32 fit queued for refinement keeps per queue slot: the factor R
// (packed), 1/diag R and the FP32 coefficients
template <int D> struct RefineKeep { static constexpr int N = Dim<D>::NG + Dim<D>::NU + Dim<D>::NF * Dim<D>::NU; };

__host__ __device__ constexpr int tri(int p, int q, int n) { return p * n - p * (p - 1) / 2 + (q - p); }

// ---------------------------------------------------------------------------
// Stencil rows
// ---------------------------------------------------------------------------
template <int D, typename T>
__device__ __forceinline__ void second_order_row(const T xi[3], T row[Dim<D>::NU]) {
#pragma unroll
    for (int a = 0; a < D; ++a) row[a] = xi[a];
#pragma unroll
    for (int a = 0; a < D; ++a) row[D + a] = T(0.5) * xi[a] * xi[a];
    if (D == 2) {
        row[4] = xi[0] * xi[1];
    } else {
        row[6] = xi[0] * xi[1];
        row[7] = xi[0] * xi[2];
        row[8] = xi[1] * xi[2];
    }
}

template <int D>
__device__ __forceinline__ void displacement(const Sorted &srt, const DevCfg &cfg, int j, const double xi[3],
                                             double dx[3]) {
    if (srt.rec) {
        double p[3];
        rec_pos<D>(srt.rec, j, p);
        disp_of<D>(cfg, p, xi, dx);
    } else {
        disp_to<D>(cfg, srt.x, j, xi, dx);
    }
}

// Position of cell-order particle j: from its gather record when there is one.
template <int D>
__device__ __forceinline__ void position_of(const Sorted &srt, int j, double p[3]) {
    if (srt.rec) {
        rec_pos<D>(srt.rec, j, p);
    } else {
        p[0] = srt.x[0][j];
        p[1] = srt.x[1][j];
        p[2] = D == 3 ? srt.x[2][j] : 0.0;
    }
}

// A list longer than the cap keeps its members of octant rank below Rstar
// and the first rem members (in list order) of rank Rstar: from the octant
// counts of the whole list, Rstar is the largest number of rounds (one
// member per non-empty octant each) that fit under the cap.  The counts come
// from octc (8 bits per octant, as the list filter recorded them) unless it
// is NULL or ~0; otherwise a walk counts them, keeping the next position and
// the index after it in flight (k >= 2 here).
template <int D>
__device__ __forceinline__ void lw_round_limit(const Sorted &srt, const DevCfg &cfg, const int *nbr, int ldn, int s,
                                               int k, const double xi[3], int cap, const unsigned long long *octc,
                                               int &Rstar, int &rem) {
    int cnt[8];
    const unsigned long long known = octc ? octc[s] : ~0ull;
    if (known != ~0ull) {
        for (int o = 0; o < 8; ++o) cnt[o] = (int)((known >> (8 * o)) & 0xff);
    } else {
        unsigned long long c03 = 0, c47 = 0;  // octant counts, 16 bits each
        double pn[3];
        position_of<D>(srt, nb_at(nbr, ldn, s, 0), pn);
        int jn = nb_at(nbr, ldn, s, 1);
        for (int t = 0; t < k; ++t) {
            const double pc[3] = {pn[0], pn[1], pn[2]};
            position_of<D>(srt, jn, pn);
            jn = nb_at(nbr, ldn, s, t + 2 < k ? t + 2 : k - 1);
            double dx[3];
            disp_of<D>(cfg, pc, xi, dx);
            const int o = octant<D>(dx);
            if (o < 4) c03 += 1ull << (16 * o); else c47 += 1ull << (16 * (o - 4));
        }
        for (int o = 0; o < 4; ++o) cnt[o] = (int)((c03 >> (16 * o)) & 0xffff);
        for (int o = 0; o < 4; ++o) cnt[4 + o] = (int)((c47 >> (16 * o)) & 0xffff);
    }
    int R = 0, taken = 0;
    for (;;) {
        int next = 0;
        for (int o = 0; o < 8; ++o) next += cnt[o] < R + 1 ? cnt[o] : R + 1;
        if (next > cap) break;
        taken = next;
        ++R;
    }
    Rstar = R;
    rem = cap - taken;
}

// Visit the Lax-Wendroff stencil: all neighbours when they fit under the cap,
// otherwise the first `cap` in the order (rank within own octant, list
// position), i.e. the top of the list holds members of every octant.
template <int D, typename F>
__device__ __forceinline__ void for_lw_stencil(const Sorted &srt, const DevCfg &cfg, const int *nbr, int ldn, int s,
                                               int k, const double xi[3], F &&body,
                                               const unsigned long long *octc = nullptr) {
    const int cap = cfg.lw_cap;
    int Rstar = 1 << 30, rem = 0;
    if (k > cap) lw_round_limit<D>(srt, cfg, nbr, ldn, s, k, xi, cap, octc, Rstar, rem);
    unsigned long long s03 = 0, s47 = 0;
    int takenR = 0;
    // the next member's index is loaded one iteration ahead, so the gathers
    // of a member wait for one memory round trip instead of two
    int jn = k > 0 ? nb_at(nbr, ldn, s, 0) : 0;
    for (int t = 0; t < k; ++t) {
        const int j = jn;
        if (t + 1 < k) jn = nb_at(nbr, ldn, s, t + 1);
        double dx[3];
        displacement<D>(srt, cfg, j, xi, dx);
        if (k > cap) {
            int o = octant<D>(dx);
            int rho;
            if (o < 4) { rho = (int)((s03 >> (16 * o)) & 0xffff); s03 += 1ull << (16 * o); }
            else { rho = (int)((s47 >> (16 * (o - 4))) & 0xffff); s47 += 1ull << (16 * (o - 4)); }
            bool take = rho < Rstar || (rho == Rstar && takenR < rem);
            if (rho == Rstar && take) ++takenR;
            if (!take) continue;
        }
        body(j, dx);
    }
}

// for_lw_stencil with the positions and fields of the next PF entries in
// flight (and the index after them): for the latency-bound refinement of a
// few particles, whose lanes have registers to spare.  body(j, dx, f) gets the
// member's V, u_0..u_{D-1}, P.  The loop is unrolled PF times, so that the
// prefetched entries rotate without copies.
template <int D, int PF, bool PER = true, typename F>
__device__ __forceinline__ void for_lw_stencil_deep(const Sorted &srt, const DevCfg &cfg, const int *nbr, int ldn,
                                                    int s, int k, const double xi[3], F &&body,
                                                    const unsigned long long *octc = nullptr) {
    const int cap = cfg.lw_cap;
    int Rstar = 1 << 30, rem = 0;
    if (k > cap) lw_round_limit<D>(srt, cfg, nbr, ldn, s, k, xi, cap, octc, Rstar, rem);
    if (k <= 0) return;
    unsigned long long s03 = 0, s47 = 0;
    int takenR = 0;
    double rp[PF][3], rf[PF][D + 2];
    int rj[PF];
#pragma unroll
    for (int q = 0; q < PF; ++q) {
        rj[q] = nb_at(nbr, ldn, s, q < k ? q : k - 1);
        position_of<D>(srt, rj[q], rp[q]);
        gather_fields<D>(srt, rj[q], rf[q]);
    }
    int jn = nb_at(nbr, ldn, s, PF < k ? PF : k - 1);  // index of entry t + PF
    for (int t0 = 0; t0 < k; t0 += PF) {
#pragma unroll
        for (int u = 0; u < PF; ++u) {
            const int t = t0 + u;
            if (t < k) {
                const int j = rj[u];
                double p[3], f[D + 2];
#pragma unroll
                for (int q = 0; q < 3; ++q) p[q] = rp[u][q];
#pragma unroll
                for (int q = 0; q < D + 2; ++q) f[q] = rf[u][q];
                rj[u] = jn;
                position_of<D>(srt, jn, rp[u]);
                gather_fields<D>(srt, jn, rf[u]);
                jn = nb_at(nbr, ldn, s, t + PF + 1 < k ? t + PF + 1 : k - 1);
                double dx[3];
                disp_of<D, PER>(cfg, p, xi, dx);
                bool take = true;
                if (k > cap) {
                    int o = octant<D>(dx);
                    int rho;
                    if (o < 4) { rho = (int)((s03 >> (16 * o)) & 0xffff); s03 += 1ull << (16 * o); }
                    else { rho = (int)((s47 >> (16 * (o - 4))) & 0xffff); s47 += 1ull << (16 * (o - 4)); }
                    take = rho < Rstar || (rho == Rstar && takenR < rem);
                    if (rho == Rstar && take) ++takenR;
                }
                if (take) body(j, dx, f);
            }
        }
    }
}

// Raw gather record of a neighbour as loaded: four 16-byte words of the FP64
// record, or the three (2D: two) of the FP32-field record.
template <bool F32REC> struct RecRaw;
template <> struct RecRaw<false> { double2 q[4]; };
template <> struct RecRaw<true> { uint4 q[3]; };

template <int D, bool F32REC>
__device__ __forceinline__ void load_rec(const Sorted &srt, int j, RecRaw<F32REC> &r) {
    if constexpr (F32REC) {
        const uint4 *p = reinterpret_cast<const uint4 *>(reinterpret_cast<const char *>(srt.recf) +
                                                         (int64_t)LP_RECF_BYTES * j);
        r.q[0] = p[0];
        r.q[1] = p[1];
        if constexpr (D == 3) r.q[2] = p[2];
    } else {
        const double2 *p = reinterpret_cast<const double2 *>(srt.rec + (int64_t)LP_REC * j);
#pragma unroll
        for (int q = 0; q < 4; ++q) r.q[q] = p[q];
    }
}

// position p and fields V, u_0 .. u_{D-1}, P of a loaded record
template <int D, bool F32REC>
__device__ __forceinline__ void unpack_rec(const RecRaw<F32REC> &r, double p[3], double f[D + 2]) {
    if constexpr (F32REC) {
        p[0] = __hiloint2double((int)r.q[0].y, (int)r.q[0].x);
        p[1] = __hiloint2double((int)r.q[0].w, (int)r.q[0].z);
        if constexpr (D == 3) {
            p[2] = __hiloint2double((int)r.q[1].y, (int)r.q[1].x);
            f[0] = __uint_as_float(r.q[1].z);
            f[1] = __uint_as_float(r.q[1].w);
            f[2] = __uint_as_float(r.q[2].x);
            f[3] = __uint_as_float(r.q[2].y);
            f[4] = __uint_as_float(r.q[2].z);
        } else {
            p[2] = 0.0;
            f[0] = __uint_as_float(r.q[1].x);
            f[1] = __uint_as_float(r.q[1].y);
            f[2] = __uint_as_float(r.q[1].z);
            f[3] = __uint_as_float(r.q[1].w);
        }
    } else {
        p[0] = r.q[0].x;
        p[1] = r.q[0].y;
        if constexpr (D == 3) {
            p[2] = r.q[1].x;
            f[0] = r.q[1].y; f[1] = r.q[2].x; f[2] = r.q[2].y; f[3] = r.q[3].x; f[4] = r.q[3].y;
        } else {
            p[2] = 0.0;
            f[0] = r.q[1].x; f[1] = r.q[1].y; f[2] = r.q[2].x; f[3] = r.q[2].y;
        }
    }
}

// The same stencil walk over the gather records, two entries deep: while
// entry t is processed, the record of entry t + 1 and the index of entry
// t + 2 are in flight (every load is unconditional, with the index clamped
// to the list, so that no load result passes through a branch).  body(j, dx,
// f) gets the member's V, u_0..u_{D-1}, P.  Needs srt.rec.
template <int D, bool F32REC = false, bool PER = true, typename F>
__device__ __forceinline__ void for_lw_stencil_rec(const Sorted &srt, const DevCfg &cfg, const int *nbr, int ldn,
                                                   int s, int k, const double xi[3], F &&body,
                                                   const unsigned long long *octc = nullptr) {
    const int cap = cfg.lw_cap;
    int Rstar = 1 << 30, rem = 0;
    if (k > cap) lw_round_limit<D>(srt, cfg, nbr, ldn, s, k, xi, cap, octc, Rstar, rem);
    if (k <= 0) return;
    unsigned long long s03 = 0, s47 = 0;
    int takenR = 0;
    int jc = nb_at(nbr, ldn, s, 0);                  // entry t
    int jn = nb_at(nbr, ldn, s, k > 1 ? 1 : 0);      // entry t + 1
    RecRaw<F32REC> rc;
    load_rec<D, F32REC>(srt, jc, rc);
    for (int t = 0; t < k; ++t) {
        const int j = jc;
        const RecRaw<F32REC> cur = rc;
        jc = jn;
        load_rec<D, F32REC>(srt, jc, rc);                 // record of entry t + 1
        jn = nb_at(nbr, ldn, s, t + 2 < k ? t + 2 : k - 1);  // index of entry t + 2
        double p[3], f[D + 2];
        unpack_rec<D, F32REC>(cur, p, f);
        double dx[3];
        disp_of<D, PER>(cfg, p, xi, dx);
        if (k > cap) {
            int o = octant<D>(dx);
            int rho;
            if (o < 4) { rho = (int)((s03 >> (16 * o)) & 0xffff); s03 += 1ull << (16 * o); }
            else { rho = (int)((s47 >> (16 * (o - 4))) & 0xffff); s47 += 1ull << (16 * (o - 4)); }
            bool take = rho < Rstar || (rho == Rstar && takenR < rem);
            if (rho == Rstar && take) ++takenR;
            if (!take) continue;
        }
        body(j, dx, f);
    }
}

// ---------------------------------------------------------------------------
// Small dense algebra in registers
// ---------------------------------------------------------------------------
// Cholesky of packed upper-triangular G (in place -> R, R^T R = G).
// Returns false on a non-positive pivot.  inv[j] = 1 / R_jj.
template <int N, typename T>
__device__ __forceinline__ bool cholesky(T G[N * (N + 1) / 2], T inv[N]) {
#pragma unroll
    for (int j = 0; j < N; ++j) {
        T s = G[tri(j, j, N)];
#pragma unroll
        for (int k = 0; k < j; ++k) s -= G[tri(k, j, N)] * G[tri(k, j, N)];
        if (!(s > T(0))) return false;
        T d = sqrt(s);
        G[tri(j, j, N)] = d;
        T iv = T(1) / d;
        inv[j] = iv;
#pragma unroll
        for (int i = j + 1; i < N; ++i) {
            T t = G[tri(j, i, N)];
#pragma unroll
            for (int k = 0; k < j; ++k) t -= G[tri(k, j, N)] * G[tri(k, i, N)];
            G[tri(j, i, N)] = t * iv;
        }
    }
    return true;
}

// ||R||_F^2 * ||R^-1||_F^2: an upper bound of cond_2(R)^2 (= cond_2 of the
// normal matrix) within a factor N^2; R^-1 is formed column by column.
template <int N, typename T>
__device__ __forceinline__ T cond_estimate(const T R[N * (N + 1) / 2], const T inv[N]) {
    T nr = 0, ni = 0;
#pragma unroll
    for (int q = 0; q < N * (N + 1) / 2; ++q) nr += R[q] * R[q];
#pragma unroll
    for (int j = 0; j < N; ++j) {
        T col[N];
        col[j] = inv[j];
        ni += col[j] * col[j];
#pragma unroll
        for (int i = j - 1; i >= 0; --i) {
            T acc = 0;
#pragma unroll
            for (int k = i + 1; k <= j; ++k) acc += R[tri(i, k, N)] * col[k];
            col[i] = -acc * inv[i];
            ni += col[i] * col[i];
        }
    }
    return nr * ni;
}

// Solve R^T R y = b for NR right-hand sides stored column-major b[c * N + p].
template <int N, int NR, typename T, typename TB>
__device__ __forceinline__ void chol_solve(const T R[N * (N + 1) / 2], const T inv[N], TB b[N * NR]) {
#pragma unroll
    for (int c = 0; c < NR; ++c) {
#pragma unroll
        for (int j = 0; j < N; ++j) {
            TB t = b[c * N + j];
#pragma unroll
            for (int k = 0; k < j; ++k) t -= TB(R[tri(k, j, N)]) * b[c * N + k];
            b[c * N + j] = t * TB(inv[j]);
        }
#pragma unroll
        for (int j = N - 1; j >= 0; --j) {
            TB t = b[c * N + j];
#pragma unroll
            for (int k = j + 1; k < N; ++k) t -= TB(R[tri(j, k, N)]) * b[c * N + k];
            b[c * N + j] = t * TB(inv[j]);
        }
    }
}

// Pivoted |R11|/|Rnn| of a D-column half-ball matrix from its normal matrix:
// with diagonal pivoting, Cholesky takes the same pivots as Householder QR
// with column pivoting and yields the same R (up to signs).
template <int D, typename T>
__device__ __forceinline__ T halfball_cond(const T G[D * (D + 1) / 2]) {
    if (D == 2) {
        T g00 = G[0], g01 = G[1], g11 = G[2];
        T gp = g00 >= g11 ? g00 : g11;
        T det = g00 * g11 - g01 * g01;
        if (!(det > T(0))) return T(INFINITY);
        return sqrt(gp * gp / det);
    } else {
        T g00 = G[0], g01 = G[1], g02 = G[2], g11 = G[3], g12 = G[4], g22 = G[5];
        T gpp, gpa, gpb, gaa, gbb, gab;
        if (g00 >= g11 && g00 >= g22) { gpp = g00; gpa = g01; gpb = g02; gaa = g11; gbb = g22; gab = g12; }
        else if (g11 >= g22) { gpp = g11; gpa = g01; gpb = g12; gaa = g00; gbb = g22; gab = g02; }
        else { gpp = g22; gpa = g02; gpb = g12; gaa = g00; gbb = g11; gab = g01; }
        if (!(gpp > T(0))) return T(INFINITY);
        T saa = gaa - gpa * gpa / gpp, sbb = gbb - gpb * gpb / gpp, sab = gab - gpa * gpb / gpp;
        T s2 = saa >= sbb ? saa : sbb;
        if (!(s2 > T(0))) return T(INFINITY);
        T s3 = (saa * sbb - sab * sab) / s2;
        if (!(s3 > T(0))) return T(INFINITY);
        return sqrt(gpp / s3);
    }
}


// ---------------------------------------------------------------------------
// Moments.  Every entry of the normal matrix A^T A of the second-order basis
// (xi_a, xi_a^2 / 2, xi_a xi_b) is c_p c_q sum_j xi_j^(alpha_p + alpha_q), a
// moment of degree 2..4 of the scaled offsets: 31 distinct moments in 3D
// (12 in 2D) instead of 45 (15) matrix entries, so the fit loop keeps fewer
// accumulators live.
// ---------------------------------------------------------------------------
template <int D> struct Mom;
template <> struct Mom<3> {
    static constexpr int N = 31;
    static constexpr int E[N][3] = {
        {2, 0, 0}, {0, 2, 0}, {0, 0, 2}, {1, 1, 0}, {1, 0, 1}, {0, 1, 1},
        {3, 0, 0}, {0, 3, 0}, {0, 0, 3}, {2, 1, 0}, {2, 0, 1}, {1, 2, 0}, {0, 2, 1}, {1, 0, 2}, {0, 1, 2}, {1, 1, 1},
        {4, 0, 0}, {0, 4, 0}, {0, 0, 4}, {3, 1, 0}, {3, 0, 1}, {1, 3, 0}, {0, 3, 1}, {1, 0, 3}, {0, 1, 3},
        {2, 2, 0}, {2, 0, 2}, {0, 2, 2}, {2, 1, 1}, {1, 2, 1}, {1, 1, 2}};
};
template <> struct Mom<2> {
    static constexpr int N = 12;
    static constexpr int E[N][3] = {{2, 0, 0}, {0, 2, 0}, {1, 1, 0}, {3, 0, 0}, {0, 3, 0}, {2, 1, 0},
                                    {1, 2, 0}, {4, 0, 0}, {0, 4, 0}, {3, 1, 0}, {1, 3, 0}, {2, 2, 0}};
};

// exponents of basis function p (0..NU-1) in the column order of second_order_row
template <int D>
__host__ __device__ constexpr int basis_exp(int p, int a) {
    return p < D ? (p == a ? 1 : 0)
         : p < 2 * D ? (p - D == a ? 2 : 0)
         : D == 2 ? 1
         : (p == 2 * D ? (a != 2 ? 1 : 0) : p == 2 * D + 1 ? (a != 1 ? 1 : 0) : (a != 0 ? 1 : 0));
}
template <int D>
__host__ __device__ constexpr double basis_coef(int p) { return (p >= D && p < 2 * D) ? 0.5 : 1.0; }
template <int D>
__host__ __device__ constexpr int mom_index(int e0, int e1, int e2) {
    for (int m = 0; m < Mom<D>::N; ++m)
        if (Mom<D>::E[m][0] == e0 && Mom<D>::E[m][1] == e1 && Mom<D>::E[m][2] == e2) return m;
    return -1;
}
template <int D>
__host__ __device__ constexpr int gram_mom(int p, int q) {
    return mom_index<D>(basis_exp<D>(p, 0) + basis_exp<D>(q, 0), basis_exp<D>(p, 1) + basis_exp<D>(q, 1),
                        D == 3 ? basis_exp<D>(p, 2) + basis_exp<D>(q, 2) : 0);
}

// add the moments of one scaled offset x
template <int D, typename T>
__device__ __forceinline__ void add_moments(const T x[3], T M[Mom<D>::N]) {
    T px[5], py[5], pz[5];
    px[0] = T(1); py[0] = T(1); pz[0] = T(1);
#pragma unroll
    for (int e = 1; e < 5; ++e) {
        px[e] = px[e - 1] * x[0];
        py[e] = py[e - 1] * x[1];
        pz[e] = D == 3 ? pz[e - 1] * x[2] : T(0);
    }
#pragma unroll
    for (int m = 0; m < Mom<D>::N; ++m) {
        constexpr int dummy = 0;
        (void)dummy;
        const int e0 = Mom<D>::E[m][0], e1 = Mom<D>::E[m][1], e2 = Mom<D>::E[m][2];
        T v = px[e0] * py[e1];
        if (D == 3 && e2) v *= pz[e2];
        M[m] += v;
    }
}

template <int D, typename T>
__device__ __forceinline__ void gram_from_moments(const T M[Mom<D>::N], T G[Dim<D>::NG]) {
    constexpr int NU = Dim<D>::NU;
#pragma unroll
    for (int p = 0; p < NU; ++p)
#pragma unroll
        for (int q = p; q < NU; ++q) G[tri(p, q, NU)] = T(basis_coef<D>(p) * basis_coef<D>(q)) * M[gram_mom<D>(p, q)];
}

// ---------------------------------------------------------------------------
// Rates (Sec. 2.1).  grad[f][a], hess[f][q] with q over (11, 22, [33,] 12 [, 13, 23]);
// fields f: 0 = V, 1..D = u, D+1 = P.
// ---------------------------------------------------------------------------
template <int D>
__device__ __forceinline__ int mixed_q(int a, int b) {
    if (a > b) { int t = a; a = b; b = t; }
    if (D == 2) return 2;
    return (a == 0 && b == 1) ? 3 : ((a == 0 && b == 2) ? 4 : 5);
}

template <int D, typename T>
__device__ __forceinline__ void lw_rates(T gamma, T dt, const T st[Dim<D>::NF], const T grad[Dim<D>::NF][3],
                                         const T hess[Dim<D>::NF][Dim<D>::NS], T rate[Dim<D>::NF]) {
    constexpr int FP = D + 1;
    T V = st[0], P = st[FP];
    T theta = 0, Tr = 0, gVgP = 0, lapP = 0;
#pragma unroll
    for (int a = 0; a < D; ++a) theta += grad[1 + a][a];
#pragma unroll
    for (int i = 0; i < D; ++i)
#pragma unroll
        for (int k = 0; k < D; ++k) Tr += grad[1 + k][i] * grad[1 + i][k];
#pragma unroll
    for (int a = 0; a < D; ++a) gVgP += grad[0][a] * grad[FP][a];
#pragma unroll
    for (int a = 0; a < D; ++a) lapP += hess[FP][a];
    T Vt = V * theta;
    T Pt = -gamma * P * theta;
    T Vtt = V * theta * theta - V * gVgP - V * V * lapP - V * Tr;
    T Ptt = gamma * gamma * P * theta * theta + gamma * P * gVgP + gamma * V * P * lapP + gamma * P * Tr;
    T half_dt = T(0.5) * dt;
    rate[0] = Vt + half_dt * Vtt;
    rate[FP] = Pt + half_dt * Ptt;
#pragma unroll
    for (int i = 0; i < D; ++i) {
        T dPi = grad[FP][i];
        T dth = 0, uxP = 0;
#pragma unroll
        for (int k = 0; k < D; ++k) {
            dth += (i == k) ? hess[1 + k][i] : hess[1 + k][mixed_q<D>(i, k)];
            uxP += grad[1 + k][i] * grad[FP][k];
        }
        T ut = -V * dPi;
        T utt = (gamma - T(1)) * V * theta * dPi + gamma * V * P * dth + V * uxP;
        rate[1 + i] = ut + half_dt * utt;
    }
}

template <int D, typename T>
__device__ __forceinline__ void uw_rates(T gamma, const T st[Dim<D>::NF], const T dl[3][3], const T dr[3][3],
                                         T rate[Dim<D>::NF]) {
    constexpr int FP = D + 1;
    T V = st[0], P = st[FP];
    T c = sqrt(gamma * P * V);
    T VV_c = V * V / c;
    T rv = 0, rp = 0;
#pragma unroll
    for (int a = 0; a < D; ++a) {
        T ul = dl[a][1], ur = dr[a][1], Pl = dl[a][2], Pr = dr[a][2];
        rv += T(0.5) * V * (ur + ul) - T(0.5) * VV_c * (Pr - Pl);
        rate[1 + a] = T(0.5) * c * (ur - ul) - T(0.5) * V * (Pr + Pl);
        rp += -T(0.5) * gamma * P * (ur + ul) + T(0.5) * c * (Pr - Pl);
    }
    rate[0] = rv;
    rate[FP] = rp;
}

template <typename T>
__device__ __forceinline__ T limiter(T r) {
    if (isinf(r)) return T(0);
    T q = sqrt(r);
    if (r <= T(1.5)) return T(1.25) * exp(T(1) - q);
    T t = q - T(1);
    return T(1.25) * exp(T(-4.5) * (t * t));
}

// ---------------------------------------------------------------------------
// Half-ball fits, estimator, blended update and mover for one particle, given
// its second-order derivatives.  Writes the caller's arrays at index i.
// ---------------------------------------------------------------------------
// Inputs of the network estimator (dimensionless; the definitions are the
// oracle's): h d_a(rho)/rho, h d_a P/P, h div u / c, for V and P on every axis
// the disagreement of the one-sided slopes (|log| of their quotient capped at
// 8, 8 for opposite signs, 0 where the estimator ignores the pair), the log
// range of V and P over the half-ball members, and h |grad u|_F / c.
template <int D, typename T>
__device__ __forceinline__ void estimator_features(const DevCfg &cfg, const double st[Dim<D>::NF],
                                                   const double grad[Dim<D>::NF][3], const T dl[3][3],
                                                   const T dr[3][3], const bool valid_l[3], const bool valid_r[3],
                                                   double h, T vmin, T vmax, T pmin, T pmax, float f[16]) {
    constexpr int FP = D + 1;
    const double V = st[0], P = st[FP];
    const double cs = sqrt(cfg.gamma * P * V);
    double div = 0.0, gu2 = 0.0;
#pragma unroll
    for (int q = 0; q < 16; ++q) f[q] = 0.f;
#pragma unroll
    for (int a = 0; a < D; ++a) {
        f[a] = (float)(-h * grad[0][a] / V);
        f[3 + a] = (float)(h * grad[FP][a] / P);
        div += grad[1 + a][a];
#pragma unroll
        for (int b = 0; b < D; ++b) gu2 += grad[1 + a][b] * grad[1 + a][b];
        const bool valid = valid_l[a] && valid_r[a];
#pragma unroll
        for (int q = 0; q < 2; ++q) {
            const double sl = (double)dl[a][2 * q], sr = (double)dr[a][2 * q];
            const double sv = q == 0 ? V : P;
            const double big = fabs(sl) > fabs(sr) ? fabs(sl) : fabs(sr);
            double g = 0.0;
            if (valid && big * h > cfg.est_eps * fabs(sv)) {
                if (!(sl * sr > 0.0)) g = 8.0;
                else {
                    g = fabs(log(fabs(sr) / fabs(sl)));
                    g = g < 8.0 ? g : 8.0;
                }
            }
            f[7 + 3 * q + a] = (float)g;
        }
    }
    f[6] = (float)(h * div / cs);
    f[13] = (float)log((double)vmax / (double)vmin);
    f[14] = (float)log((double)pmax / (double)pmin);
    f[15] = (float)(h * sqrt(gu2) / cs);
}

// ---------------------------------------------------------------------------
// Second-order derivatives kept between the fit and the update kernels
// (SoA, der[q * ld + t], t the particle's work slot): gradients of V, u_1..u_D, P (D each), the Hessians
// of u_1..u_D (NS each) and the diagonal second derivatives of P (D).
// ---------------------------------------------------------------------------
template <int D> struct Der { static constexpr int N = (D + 2) * D + D * Dim<D>::NS + D; };

template <int D>
__device__ __forceinline__ void store_der(double *der, int64_t ld, int s, const double grad[Dim<D>::NF][3],
                                          const double hess[Dim<D>::NF][Dim<D>::NS]) {
    constexpr int NF = Dim<D>::NF, NS = Dim<D>::NS;
    int q = 0;
#pragma unroll
    for (int f = 0; f < NF; ++f)
#pragma unroll
        for (int a = 0; a < D; ++a) der[(q++) * ld + s] = grad[f][a];
#pragma unroll
    for (int k = 0; k < D; ++k)
#pragma unroll
        for (int c = 0; c < NS; ++c) der[(q++) * ld + s] = hess[1 + k][c];
#pragma unroll
    for (int a = 0; a < D; ++a) der[(q++) * ld + s] = hess[D + 1][a];
}

template <int D>
__device__ __forceinline__ void load_der(const double *der, int64_t ld, int s, double grad[Dim<D>::NF][3],
                                         double hess[Dim<D>::NF][Dim<D>::NS]) {
    constexpr int NF = Dim<D>::NF, NS = Dim<D>::NS;
    int q = 0;
#pragma unroll
    for (int f = 0; f < NF; ++f) {
#pragma unroll
        for (int a = 0; a < 3; ++a) grad[f][a] = 0.0;
#pragma unroll
        for (int c = 0; c < NS; ++c) hess[f][c] = 0.0;
    }
#pragma unroll
    for (int f = 0; f < NF; ++f)
#pragma unroll
        for (int a = 0; a < D; ++a) grad[f][a] = der[(q++) * ld + s];
#pragma unroll
    for (int k = 0; k < D; ++k)
#pragma unroll
        for (int c = 0; c < NS; ++c) hess[1 + k][c] = der[(q++) * ld + s];
#pragma unroll
    for (int a = 0; a < D; ++a) hess[D + 1][a] = der[(q++) * ld + s];
}

// Where the update reads the particle's LW derivatives: registers (the
// fallback's own fit) or the derivative array of the fast fit, read where
// they are used, so that they hold no registers through the half-ball loops.
template <int D> struct DerRegs {
    const double (*grad)[3];
    const double (*hess)[Dim<D>::NS];
    __device__ __forceinline__ double g(int f, int a) const { return grad[f][a]; }
    __device__ __forceinline__ void all(double gr[Dim<D>::NF][3], double he[Dim<D>::NF][Dim<D>::NS]) const {
#pragma unroll
        for (int f = 0; f < Dim<D>::NF; ++f) {
#pragma unroll
            for (int a = 0; a < 3; ++a) gr[f][a] = grad[f][a];
#pragma unroll
            for (int c = 0; c < Dim<D>::NS; ++c) he[f][c] = hess[f][c];
        }
    }
};

template <int D> struct DerMem {
    const double *der;
    int64_t ld;
    int t;
    // gradient entry (f, a) is entry f * D + a of the array's layout
    __device__ __forceinline__ double g(int f, int a) const { return der[(int64_t)(f * D + a) * ld + t]; }
    __device__ __forceinline__ void all(double gr[Dim<D>::NF][3], double he[Dim<D>::NF][Dim<D>::NS]) const {
        load_der<D>(der, ld, t, gr, he);
    }
};

// The FP32 fit's scaled coefficients B[f * NU + column] and 1/r, held in
// registers by the fused kernel: derivatives formed as the derivative array
// would hold them.
template <int D> struct DerCoef {
    const float *B;
    double inv_r;
    __device__ __forceinline__ double g(int f, int a) const { return (double)B[f * Dim<D>::NU + a] * inv_r; }
    __device__ __forceinline__ void all(double gr[Dim<D>::NF][3], double he[Dim<D>::NF][Dim<D>::NS]) const {
#pragma unroll
        for (int f = 0; f < Dim<D>::NF; ++f) {
#pragma unroll
            for (int a = 0; a < 3; ++a) gr[f][a] = a < D ? (double)B[f * Dim<D>::NU + a] * inv_r : 0.0;
#pragma unroll
            for (int c = 0; c < Dim<D>::NS; ++c) he[f][c] = (double)B[f * Dim<D>::NU + D + c] * inv_r * inv_r;
        }
    }
};

// What the update of a particle hands to the network in the fused kernel:
// the inputs go to the lane's row of the block's feature array in LDS, the
// rates and the quotient estimator's phi stay in registers.
template <int D> struct NetLane {
    float *feat;
    float lw[D + 2], uw[D + 2];
    double phi_plain;
    uint8_t mf;
    bool in_range;  // every input within +-mlp_feat_max
    bool have;
};

template <int D, typename T, bool PER = true, int PF = 1, class DS>
__device__ __forceinline__ bool finish_particle(const Sorted &srt, const Soa &p, const DevCfg &cfg, DevScalars *sc,
                                                const int *nbr, int ldn, int s, int i, int k, double dt,
                                                const double xi[3], const double st[Dim<D>::NF], double h, double r,
                                                const DS &ds, int lw_status, uint8_t flags,
                                                const MlpStage *ms = nullptr, NetLane<D> *nl = nullptr,
                                                unsigned long long oct = ~0ull) {
    constexpr int NF = Dim<D>::NF, FP = D + 1, NGD = D * (D + 1) / 2;
    // V and P over the particle and its half-ball members (network inputs)
    T vmin = (T)st[0], vmax = (T)st[0], pmin = (T)st[FP], pmax = (T)st[FP];
    const int ucap = cfg.uw_cap;
    const double inv_r = 1.0 / r;
    T dl[3][3], dr[3][3];
    bool valid_l[3] = {false, false, false}, valid_r[3] = {false, false, false};
    bool vac = false, subst = false;
    const T Pi_T = (T)st[FP];
#pragma unroll
    for (int a = 0; a < D; ++a) {
        T Gl[NGD], Gr[NGD], Bl[D * 3], Br[D * 3], Sl[D], Sr[D];
#pragma unroll
        for (int q = 0; q < NGD; ++q) { Gl[q] = 0; Gr[q] = 0; }
#pragma unroll
        for (int q = 0; q < D * 3; ++q) { Bl[q] = 0; Br[q] = 0; }
#pragma unroll
        for (int q = 0; q < D; ++q) { Sl[q] = 0; Sr[q] = 0; }
        int nl = 0, nr = 0;
        // the walk ends once both sides are as full as they can get: oct (the
        // list's members per octant, 8 bits each, or ~0 when unknown) bounds
        // the members left of the particle along a exactly (octant bit a
        // clear) and those right of it from above (bit a set: dx_a >= 0)
        int capl = ucap, capr = ucap;
        if (oct != ~0ull) {
            int cl = 0, cr = 0;
#pragma unroll
            for (int o = 0; o < (1 << D); ++o) {
                const int c = (int)((oct >> (8 * o)) & 0xffull);
                if ((o >> a) & 1) cr += c; else cl += c;
            }
            capl = cl < ucap ? cl : ucap;
            capr = cr < ucap ? cr : ucap;
        }
        const T fi[3] = {(T)st[0], (T)st[1 + a], (T)st[FP]};
        // a member of an open half-ball of axis a: accumulate it
        auto visit = [&](const double dx[3], const double fr[NF]) {
            const bool right = dx[a] > 0.0;
            T x[3];
#pragma unroll
            for (int b = 0; b < D; ++b) x[b] = (T)(dx[b] * inv_r);
            const T fj[3] = {(T)fr[0], (T)fr[1 + a], (T)fr[FP]};
            T bq[3] = {fj[0] - fi[0], fj[1] - fi[1], fj[2] - fi[2]};
            vmin = fj[0] < vmin ? fj[0] : vmin;
            vmax = fj[0] > vmax ? fj[0] : vmax;
            pmin = fj[2] < pmin ? fj[2] : pmin;
            pmax = fj[2] > pmax ? fj[2] : pmax;
            // both sides accumulate with 0/1 weights (no pointer selects, so the
            // accumulators stay in registers)
            T wr = right ? T(1) : T(0), wl = right ? T(0) : T(1);
            int q = 0;
#pragma unroll
            for (int b = 0; b < D; ++b)
#pragma unroll
                for (int c = b; c < D; ++c, ++q) {
                    T v = x[b] * x[c];
                    Gr[q] += wr * v;
                    Gl[q] += wl * v;
                }
#pragma unroll
            for (int b = 0; b < D; ++b) {
#pragma unroll
                for (int f = 0; f < 3; ++f) {
                    T v = x[b] * bq[f];
                    Br[b * 3 + f] += wr * v;
                    Bl[b * 3 + f] += wl * v;
                }
                Sr[b] += wr * x[b];
                Sl[b] += wl * x[b];
            }
            if (right) ++nr; else ++nl;
        };
        // the walk two entries deep over the gather records: the next record
        // and the index after it are in flight while an entry is examined
        // (loads unconditional, index clamped to the list); the FP64 variant
        // spills a few registers for it and is still faster.  The FP32 update
        // rounds every field it reads to FP32 first, so it reads the
        // FP32-field record.
        auto walk = [&](auto f32rec) {
            constexpr bool F32REC = decltype(f32rec)::value;
            int jc = nb_at(nbr, ldn, s, 0), jn = nb_at(nbr, ldn, s, k > 1 ? 1 : 0);
            RecRaw<F32REC> rc;
            load_rec<D, F32REC>(srt, jc, rc);
            for (int t = 0; t < k && (nl < capl || nr < capr); ++t) {
                const RecRaw<F32REC> cur = rc;
                jc = jn;
                load_rec<D, F32REC>(srt, jc, rc);
                jn = nb_at(nbr, ldn, s, t + 2 < k ? t + 2 : k - 1);
                double pj[3], fr[NF];
                unpack_rec<D, F32REC>(cur, pj, fr);
                double dx[3];
                disp_of<D, PER>(cfg, pj, xi, dx);
                const bool right = dx[a] > 0.0, left = dx[a] < 0.0;
                if (!((right && nr < ucap) || (left && nl < ucap))) continue;
                visit(dx, fr);
            }
        };
        // the same walk with the records of the next PF entries in flight
        // (PF > 1: the refinement's few particles, registers to spare); the
        // loop is unrolled PF times, so that the records rotate without copies
        auto walk_deep = [&](auto f32rec) {
            constexpr bool F32REC = decltype(f32rec)::value;
            RecRaw<F32REC> ring[PF];
#pragma unroll
            for (int q = 0; q < PF; ++q) load_rec<D, F32REC>(srt, nb_at(nbr, ldn, s, q < k ? q : k - 1), ring[q]);
            int jn = nb_at(nbr, ldn, s, PF < k ? PF : k - 1);  // index of entry t + PF
            bool go = true;
            for (int t0 = 0; t0 < k && go; t0 += PF) {
#pragma unroll
                for (int u = 0; u < PF; ++u) {
                    const int t = t0 + u;
                    go = go && t < k && (nl < capl || nr < capr);
                    if (go) {
                        const RecRaw<F32REC> cur = ring[u];
                        load_rec<D, F32REC>(srt, jn, ring[u]);
                        jn = nb_at(nbr, ldn, s, t + PF + 1 < k ? t + PF + 1 : k - 1);
                        double pj[3], fr[NF];
                        unpack_rec<D, F32REC>(cur, pj, fr);
                        double dx[3];
                        disp_of<D, PER>(cfg, pj, xi, dx);
                        const bool right = dx[a] > 0.0, left = dx[a] < 0.0;
                        if ((right && nr < ucap) || (left && nl < ucap)) visit(dx, fr);
                    }
                }
            }
        };
        bool walked = false;
        if constexpr (std::is_same<T, float>::value) {
            if (srt.recf && k > 0) {
                if constexpr (PF > 1) walk_deep(std::true_type{});
                else walk(std::true_type{});
                walked = true;
            }
        }
        if (walked) {
        } else if (srt.rec && k > 0) {
            walk(std::false_type{});
        } else {
            int jn = k > 0 ? nb_at(nbr, ldn, s, 0) : 0;  // next index loaded one iteration ahead
            for (int t = 0; t < k && (nl < capl || nr < capr); ++t) {
                const int j = jn;
                if (t + 1 < k) jn = nb_at(nbr, ldn, s, t + 1);
                double dx[3];
                displacement<D>(srt, cfg, j, xi, dx);
                const bool right = dx[a] > 0.0, left = dx[a] < 0.0;
                if (!((right && nr < ucap) || (left && nl < ucap))) continue;
                double fr[NF];
                gather_fields<D>(srt, j, fr);
                visit(dx, fr);
            }
        }
        // per side: fit, vacuum ghosts, or LW substitute
#pragma unroll
        for (int side = 0; side < 2; ++side) {
            const bool isr = side == 1;
            int n_own = isr ? nr : nl, n_opp = isr ? nl : nr;
            T d[3] = {0, 0, 0};
            bool ok = false, real_fit = false;
            if (cfg.vacuum && n_own < ucap) {
                // free boundary: the half-ball's real members plus the mirror
                // images (through x_i along a) of the opposite half-ball's
                // members, which carry P = 0 and the particle's own V and u, so
                // their right-hand sides are (0, 0, -P_i)
                T Gm[NGD], Bm[D * 3];
                int q = 0;
#pragma unroll
                for (int b = 0; b < D; ++b)
#pragma unroll
                    for (int c = b; c < D; ++c, ++q) {
                        T g = isr ? Gl[q] : Gr[q];
                        bool flip = (b == a) != (c == a);
                        Gm[q] = (isr ? Gr[q] : Gl[q]) + (flip ? -g : g);
                    }
#pragma unroll
                for (int b = 0; b < D; ++b) {
                    T sv = isr ? Sl[b] : Sr[b];
#pragma unroll
                    for (int f = 0; f < 3; ++f) Bm[f * D + b] = isr ? Br[b * 3 + f] : Bl[b * 3 + f];
                    Bm[2 * D + b] += -Pi_T * (b == a ? -sv : sv);
                }
                if (n_own + n_opp >= D && halfball_cond<D, T>(Gm) <= (T)cfg.uw_cond_max) {
                    T inv[D];
                    if (cholesky<D, T>(Gm, inv)) {
                        chol_solve<D, 3, T, T>(Gm, inv, Bm);
#pragma unroll
                        for (int f = 0; f < 3; ++f) d[f] = Bm[f * D + a] * (T)inv_r;
                        ok = true;
                        vac = true;
                    }
                }
            } else {
                T Gs[NGD], Bs[D * 3];
#pragma unroll
                for (int q = 0; q < NGD; ++q) Gs[q] = isr ? Gr[q] : Gl[q];
                // right-hand sides column-major for chol_solve: Bs[f * D + b]
#pragma unroll
                for (int b = 0; b < D; ++b)
#pragma unroll
                    for (int f = 0; f < 3; ++f) Bs[f * D + b] = isr ? Br[b * 3 + f] : Bl[b * 3 + f];
                if (n_own >= D && halfball_cond<D, T>(Gs) <= (T)cfg.uw_cond_max) {
                    T inv[D];
                    if (cholesky<D, T>(Gs, inv)) {
                        chol_solve<D, 3, T, T>(Gs, inv, Bs);
#pragma unroll
                        for (int f = 0; f < 3; ++f) d[f] = Bs[f * D + a] * (T)inv_r;
                        ok = true;
                        real_fit = true;
                    }
                }
            }
            if (!ok) {
                d[0] = (T)ds.g(0, a);
                d[1] = (T)ds.g(1 + a, a);
                d[2] = (T)ds.g(FP, a);
                subst = true;
            }
#pragma unroll
            for (int f = 0; f < 3; ++f) { if (isr) dr[a][f] = d[f]; else dl[a][f] = d[f]; }
            if (isr) valid_r[a] = real_fit; else valid_l[a] = real_fit;
        }
    }
    // state estimator on P and V, one phi per particle
    double phi;
    if (cfg.est_mode == LP_EST_INJECTED && p.phi) {
        phi = (double)p.phi[i];
    } else {
        T rmax = T(1);
#pragma unroll
        for (int a = 0; a < D; ++a) {
            if (!(valid_l[a] && valid_r[a])) continue;
#pragma unroll
            for (int q = 0; q < 3; q += 2) {
                T sl = dl[a][q], sr = dr[a][q];
                T sv = q == 0 ? (T)st[0] : (T)st[FP];
                T big = fabs(sl) > fabs(sr) ? fabs(sl) : fabs(sr);
                if (big * (T)h > (T)cfg.est_eps * fabs(sv)) {
                    T rr = (sl * sr <= T(0)) ? T(INFINITY) : T(0.5) * (sr / sl + sl / sr);
                    if (rr > rmax) rmax = rr;
                }
            }
        }
        T ph = limiter<T>(rmax);
        const T cap = (T)cfg.limiter_cap;
        phi = (double)((cap > T(0) && ph > cap) ? cap : ph);
        if (lw_status != 0 || vac) phi = 0.0;
    }
    // rates
    T stT[NF], gT[NF][3], hT[NF][Dim<D>::NS], lw[NF], uw[NF];
    double grad[NF][3], hess[NF][Dim<D>::NS];
    ds.all(grad, hess);
#pragma unroll
    for (int f = 0; f < NF; ++f) {
        stT[f] = (T)st[f];
#pragma unroll
        for (int a = 0; a < 3; ++a) gT[f][a] = (T)grad[f][a];
#pragma unroll
        for (int q = 0; q < Dim<D>::NS; ++q) hT[f][q] = (T)hess[f][q];
    }
    lw_rates<D, T>((T)cfg.gamma, (T)dt, stT, gT, hT, lw);
    uw_rates<D, T>((T)cfg.gamma, stT, dl, dr, uw);
    if (ms) {
        // network estimator: stage inputs, rates and the quotient estimator's
        // phi; the network decides phi and applies the update afterwards
        float fv[16];
        estimator_features<D, T>(cfg, st, grad, dl, dr, valid_l, valid_r, h, vmin, vmax, pmin, pmax, fv);
        uint8_t mf = flags;
        if (lw_status != 0) mf |= LP_FLAG_DEGENERATE;
        if (vac) mf |= LP_FLAG_VACUUM;
        if (subst) mf |= LP_FLAG_SUBSTITUTED;
        if (lw_status != 0 || vac) mf |= LP_MLP_FORCE0;
        if (nl) {
            bool in_range = true;
#pragma unroll
            for (int q = 0; q < 16; ++q) {
                nl->feat[q] = fv[q];
                in_range = in_range && fabsf(fv[q]) <= cfg.mlp_feat_max;
            }
#pragma unroll
            for (int f = 0; f < NF; ++f) {
                nl->lw[f] = (float)lw[f];
                nl->uw[f] = (float)uw[f];
            }
            nl->phi_plain = phi;
            nl->mf = mf;
            nl->in_range = in_range;
            nl->have = true;
            return false;
        }
#pragma unroll
        for (int q = 0; q < 16; ++q) ms->feat[(int64_t)s * 16 + q] = fv[q];
#pragma unroll
        for (int f = 0; f < NF; ++f) {
            ms->rates[(int64_t)f * ms->ld + s] = (double)lw[f];
            ms->rates[(int64_t)(NF + f) * ms->ld + s] = (double)uw[f];
        }
        ms->phi_plain[s] = phi;
        ms->mflag[s] = mf;
        return false;
    }
    double ns[NF];
#pragma unroll
    for (int f = 0; f < NF; ++f) {
        double u_ = (double)uw[f], l_ = (double)lw[f];
        ns[f] = st[f] + dt * (u_ - phi * (u_ - l_));
    }
    // particle mover: x^{n+1} = x^n + dt/2 (u^n + u^{n+1})
#pragma unroll
    for (int a = 0; a < D; ++a) {
        double xn = xi[a] + 0.5 * dt * (st[1 + a] + ns[1 + a]);
        if (cfg.periodic[a]) {
            if (xn >= cfg.hi[a]) xn -= cfg.L[a];
            else if (xn < cfg.lo[a]) xn += cfg.L[a];
        }
        p.x[a][i] = xn;
        p.u[a][i] = ns[1 + a];
    }
    p.V[i] = ns[0];
    p.P[i] = ns[FP];
    if (phi < 1.0) flags |= LP_FLAG_LIMITED;
    if (lw_status != 0) flags |= LP_FLAG_DEGENERATE;
    if (vac) flags |= LP_FLAG_VACUUM;
    if (subst) flags |= LP_FLAG_SUBSTITUTED;
    if (!(ns[0] > 0.0) || !(ns[FP] > 0.0)) {
        flags |= LP_FLAG_NUMERIC;
        atomicOr(&sc->error_bits, 2u);
    }
    if (p.flags) p.flags[i] = flags;
    if (p.phi && cfg.est_mode != LP_EST_INJECTED) p.phi[i] = (float)phi;
    return phi < 1.0;  // limited: counted by the caller
}


// ---------------------------------------------------------------------------
// Fast path: one thread per particle.
// ---------------------------------------------------------------------------
// One step of iterative refinement of an FP32 fit: the residual b - A y of
// the FP64 system at the FP32 solution y (promoted exactly) is formed in
// FP64; its normal-equation image A^T r and the correction solve use the FP32
// factor (R, 1/diag R), as the correction only needs working precision.  The
// refined coefficients are stored as the particle's derivatives, or (FINISH)
// go straight on to the particle's update; the result: limited.
template <int D, bool FINISH, int PF = 1, bool PER = true>
__device__ __forceinline__ bool lw_refine_tail(const SolveArgs &a, int s, int t, int k, const double xi[3],
                                               const double st[Dim<D>::NF], double inv_r, const float G[Dim<D>::NG],
                                               const float inv[Dim<D>::NU], const float B[Dim<D>::NF * Dim<D>::NU]) {
    constexpr int NU = Dim<D>::NU, NF = Dim<D>::NF, NS = Dim<D>::NS, FP = D + 1;
    using T = float;
    const Sorted &srt = a.srt;
    T Ar[NF * NU];
#pragma unroll
    for (int q = 0; q < NF * NU; ++q) Ar[q] = 0;
    auto member = [&](const double dx[3], const double fj[NF]) {
        double x[3];
#pragma unroll
        for (int q = 0; q < D; ++q) x[q] = dx[q] * inv_r;
        double row[NU];
        second_order_row<D, double>(x, row);
        T rowf[NU];
#pragma unroll
        for (int pp = 0; pp < NU; ++pp) rowf[pp] = (T)row[pp];
#pragma unroll
        for (int f = 0; f < NF; ++f) {
            double res = fj[f] - st[f];
#pragma unroll
            for (int pp = 0; pp < NU; ++pp) res -= row[pp] * (double)B[f * NU + pp];
            T rf = (T)res;
#pragma unroll
            for (int pp = 0; pp < NU; ++pp) Ar[f * NU + pp] += rowf[pp] * rf;
        }
    };
    if (srt.rec) {
        for_lw_stencil_rec<D>(
            srt, a.cfg, a.nbr, a.ldn, s, k, xi, [&](int, const double dx[3], const double fj[NF]) { member(dx, fj); },
            a.octc);
    } else if constexpr (PF > 1) {
        for_lw_stencil_deep<D, PF, PER>(
            srt, a.cfg, a.nbr, a.ldn, s, k, xi, [&](int, const double dx[3], const double fj[NF]) { member(dx, fj); },
            a.octc);
    } else {
        for_lw_stencil<D>(
            srt, a.cfg, a.nbr, a.ldn, s, k, xi,
            [&](int j, const double dx[3]) {
                double fj[NF];
                gather_fields<D>(srt, j, fj);
                member(dx, fj);
            },
            a.octc);
    }
    chol_solve<NU, NF, T, T>(G, inv, Ar);
    double grad[NF][3], hess[NF][NS];
#pragma unroll
    for (int f = 0; f < NF; ++f) {
#pragma unroll
        for (int q = 0; q < 3; ++q)
            grad[f][q] = q < D ? ((double)B[f * NU + q] + (double)Ar[f * NU + q]) * inv_r : 0.0;
#pragma unroll
        for (int q = 0; q < NS; ++q)
            hess[f][q] = ((double)B[f * NU + D + q] + (double)Ar[f * NU + D + q]) * inv_r * inv_r;
    }
    if constexpr (FINISH) {
        const double h = srt.h[s];
        const DerRegs<D> ds{grad, hess};
        return finish_particle<D, float, PER, PF>(srt, a.p, a.cfg, a.sc, a.nbr, a.ldn, s, srt.id[s], k, a.sc->dt,
                                                   xi, st, h, a.cfg.kappa * h, ds, 0, 0,
                                                   a.ms.feat ? &a.ms : nullptr, nullptr,
                                                   a.octc ? a.octc[s] : ~0ull);
    } else {
        store_der<D>(a.der, a.ld, t, grad, hess);
        return false;
    }
}

// s: cell-order particle; t: its work slot, which indexes der (the queue
// order, so that a wave's derivative stores and loads stay coalesced).
// REGS: the fused kernel's form -- the FP32 coefficients and 1/r are
// returned in bout / inv_r_out instead of being stored as derivatives, and the
// result says whether the caller goes on to the update (false: not a real
// particle, queued for the FP64 fallback, or queued for refinement, whose
// kernel finishes the particle)
template <int D, typename T, bool REFINE, bool REGS = false, bool PER = true>
__device__ __forceinline__ bool lw_fit_one(const SolveArgs &a, int s, int t, float *bout = nullptr,
                                           double *inv_r_out = nullptr) {
    constexpr int NU = Dim<D>::NU, NF = Dim<D>::NF, NG = Dim<D>::NG, NS = Dim<D>::NS, FP = D + 1;
    const bool use_f = sizeof(T) == 4;
    const Sorted &srt = a.srt;
    const DevCfg &cfg = a.cfg;
    int i = srt.id[s];
    // ghosts, and particles deleted since the cell order was built (no radius)
    if (i >= a.n_real || !(srt.h[s] > 0.0)) return false;
    int k = a.count[s];
    if (k > cfg.max_nb) k = cfg.max_nb;
    double xi[3] = {srt.x[0][s], srt.x[1][s], D == 3 ? srt.x[2][s] : 0.0};
    double st[NF];
    st[0] = srt.V[s];
#pragma unroll
    for (int q = 0; q < D; ++q) st[1 + q] = srt.u[q][s];
    st[FP] = srt.P[s];
    const double h = srt.h[s];
    const double r = cfg.kappa * h;
    const double inv_r = 1.0 / r;
    T fi[NF];
#pragma unroll
    for (int f = 0; f < NF; ++f) fi[f] = (T)st[f];
    // normal equations of the scaled second-order system over the LW stencil:
    // moments of the offsets (the normal matrix) and A^T b
    T M[Mom<D>::N], B[NF * NU];
#pragma unroll
    for (int q = 0; q < Mom<D>::N; ++q) M[q] = 0;
#pragma unroll
    for (int q = 0; q < NF * NU; ++q) B[q] = 0;
    int m = 0;
    auto member = [&](const double dx[3], const double fr[NF]) {
        T x[3];
#pragma unroll
        for (int q = 0; q < D; ++q) x[q] = (T)(dx[q] * inv_r);
        add_moments<D, T>(x, M);
        T row[NU];
        second_order_row<D, T>(x, row);
        T fj[NF];
#pragma unroll
        for (int f = 0; f < NF; ++f) fj[f] = (T)fr[f];
#pragma unroll
        for (int f = 0; f < NF; ++f) {
            T b = fj[f] - fi[f];
#pragma unroll
            for (int pp = 0; pp < NU; ++pp) B[f * NU + pp] += row[pp] * b;
        }
        ++m;
    };
    // the FP32 fit rounds every field it reads to FP32 first, so it reads the
    // FP32-field record (three loads instead of four); its refinement walks
    // the FP64 record
    constexpr bool F32REC = std::is_same<T, float>::value;
    if (F32REC && srt.recf) {
        for_lw_stencil_rec<D, F32REC, PER>(
            srt, cfg, a.nbr, a.ldn, s, k, xi, [&](int, const double dx[3], const double fr[NF]) { member(dx, fr); },
            a.octc);
    } else if (srt.rec) {
        // one record in flight while a member is accumulated
        for_lw_stencil_rec<D>(
            srt, cfg, a.nbr, a.ldn, s, k, xi, [&](int, const double dx[3], const double fr[NF]) { member(dx, fr); },
            a.octc);
    } else {
        for_lw_stencil<D>(
            srt, cfg, a.nbr, a.ldn, s, k, xi,
            [&](int j, const double dx[3]) {
                double fr[NF];
                gather_fields<D>(srt, j, fr);
                member(dx, fr);
            },
            a.octc);
    }
    T G[NG];
    gram_from_moments<D, T>(M, G);
    T inv[NU];
    bool good = m >= NU && cholesky<NU, T>(G, inv);
    T cond = 0;
    if (good) {
        cond = cond_estimate<NU, T>(G, inv);
        good = cond <= (T)cfg.cond_fb;
    }
    if (!good) {
        int slot = atomicAdd(&a.sc->n_fallback, 1);
        a.queue[slot] = s;
        a.lwst[s] = 1;
        return false;
    }
    a.lwst[s] = 0;
    // B <- (R^T R)^-1 B in place: the scaled coefficients of every field
    chol_solve<NU, NF, T, T>(G, inv, B);
    if constexpr (REFINE) {
        lw_refine_tail<D, false>(a, s, t, k, xi, st, inv_r, G, inv, B);
        return false;
    }
    if (use_f && a.rq && cfg.refine && cfg.refine_cond > 0.0f && cond > (T)cfg.refine_cond) {
        // refined by k_lw_refine from the stored factor and FP32 solution
        const int slot = atomicAdd(&a.sc->n_refine, 1);
        a.rq[2 * slot] = s;
        a.rq[2 * slot + 1] = t;
        float *keep = a.rkeep + (int64_t)slot * RefineKeep<D>::N;
#pragma unroll
        for (int q = 0; q < NG; ++q) keep[q] = (float)G[q];
#pragma unroll
        for (int q = 0; q < NU; ++q) keep[NG + q] = (float)inv[q];
#pragma unroll
        for (int q = 0; q < NF * NU; ++q) keep[NG + NU + q] = (float)B[q];
        return false;
    }
    if constexpr (REGS) {
        static_assert(std::is_same<T, float>::value, "the fused kernel runs the FP32 fit");
#pragma unroll
        for (int q = 0; q < NF * NU; ++q) bout[q] = B[q];
        *inv_r_out = inv_r;
    } else {
        double grad[NF][3], hess[NF][NS];
#pragma unroll
        for (int f = 0; f < NF; ++f) {
#pragma unroll
            for (int q = 0; q < 3; ++q) grad[f][q] = q < D ? (double)B[f * NU + q] * inv_r : 0.0;
#pragma unroll
            for (int q = 0; q < NS; ++q) hess[f][q] = (double)B[f * NU + D + q] * inv_r * inv_r;
        }
        store_der<D>(a.der, a.ld, t, grad, hess);
    }
    return true;
}

// Half-ball fits, estimator, blended update and mover of one particle whose
// second-order fit the fast path solved.
template <int D, typename T>
__device__ __forceinline__ bool finish_one(const SolveArgs &a, int s, int t) {
    constexpr int NF = Dim<D>::NF, NS = Dim<D>::NS, FP = D + 1;
    const Sorted &srt = a.srt;
    const DevCfg &cfg = a.cfg;
    int i = srt.id[s];
    if (i >= a.n_real || a.lwst[s] != 0 || !(srt.h[s] > 0.0)) return false;
    int k = a.count[s];
    if (k > cfg.max_nb) k = cfg.max_nb;
    double xi[3] = {srt.x[0][s], srt.x[1][s], D == 3 ? srt.x[2][s] : 0.0};
    double st[NF];
    st[0] = srt.V[s];
#pragma unroll
    for (int q = 0; q < D; ++q) st[1 + q] = srt.u[q][s];
    st[FP] = srt.P[s];
    const double h = srt.h[s];
    const double r = cfg.kappa * h;
    const DerMem<D> ds{a.der, a.ld, t};
    return finish_particle<D, T>(srt, a.p, cfg, a.sc, a.nbr, a.ldn, s, i, k, a.sc->dt, xi, st, h, r, ds, 0, 0,
                                 a.ms.feat ? &a.ms : nullptr, nullptr, a.octc ? a.octc[s] : ~0ull);
}

// Work distribution.  WQ_DIRECT: thread t of the grid serves cell-order
// particle t.  WQ_QUEUE: it serves wq[t], the cell-order particles regrouped
// tile by tile by stencil size, so the lanes of a wave loop over similar
// neighbour counts.  WQ_PERSISTENT: a grid sized to the resident capacity of
// the chip takes chunks of wq (blockDim entries each) from per-XCD ranges
// until every range is drained.
enum { WQ_DIRECT = 0, WQ_QUEUE = 1, WQ_PERSISTENT = 2 };

template <int MODE, typename F>
__device__ __forceinline__ void for_work(const SolveArgs &a, unsigned *head, F &&body) {
    const int n = *a.n_total_dev;
    if (MODE == WQ_PERSISTENT) {
        persistent_chunks(head, n, [&](int t) {
            if (t < n) body(a.wq[t], t);
        });
    } else {
        int t = xcd_remap(blockIdx.x, gridDim.x) * blockDim.x + threadIdx.x;
        if (t < n) body(MODE == WQ_QUEUE ? a.wq[t] : t, t);  // no early exit: callers reduce over the wave
    }
}

// count of limited particles: wave sums (every lane of the wave is here),
// then one atomic per block (same-address atomics serialise in L2)
__device__ __forceinline__ void block_add_limited(DevScalars *sc, int limited) {
    for (int o = 32; o > 0; o >>= 1) limited += __shfl_xor(limited, o);
    __shared__ int wl[LP_BLOCK / 64];
    if ((threadIdx.x & 63) == 0) wl[threadIdx.x >> 6] = limited;
    __syncthreads();
    if (threadIdx.x == 0) {
        int tot = 0;
        for (int q = 0; q < (int)(blockDim.x >> 6); ++q) tot += wl[q];
        if (tot) atomicAdd(&sc->n_limited, (unsigned long long)tot);
    }
}

template <int D, typename T, bool REFINE, int MODE>
__global__ __launch_bounds__(LP_BLOCK, 2) void k_lw_fit(SolveArgs a) {
    for_work<MODE>(a, a.sc->head[0], [&](int s, int t) { lw_fit_one<D, T, REFINE>(a, s, t); });
}

// Three waves per SIMD: the FP64 update spills a few registers at that
// bound, but the extra resident wave hides more of its gather latency.
template <int D, typename T, int MODE>
__global__ __launch_bounds__(LP_BLOCK) __attribute__((amdgpu_waves_per_eu(3))) void k_finish(SolveArgs a) {
    int limited = 0;
    for_work<MODE>(a, a.sc->head[1], [&](int s, int t) { limited += finish_one<D, T>(a, s, t) ? 1 : 0; });
    block_add_limited(a.sc, limited);
}

// The FP32 fit and the update of a particle in one kernel: the fit's
// coefficients stay in registers (no derivative array); particles queued for
// refinement are updated by the refinement kernel, those queued for the FP64
// fallback by the fallback kernel.  At most three waves per SIMD keeps the
// fit's and the update's registers within 168 without spilling.  NET: the
// estimator network decides phi -- the block stages the network's BF16
// weights in LDS, every lane leaves its particle's inputs in the block's
// feature array, and each wave runs its 64 particles through the network in
// four tiles before the blended update.
template <bool NET> struct FusedShared {};
template <> struct FusedShared<true> {
    MlpShared w;
    float feat[LP_BLOCK][MLP_IN + 1];  // padded rows: the tile loads spread over the banks
};

// PER: some axis is periodic (else every displacement is a plain difference)
template <int D, int MODE, bool NET, bool PER>
__global__ __launch_bounds__(LP_BLOCK) __attribute__((amdgpu_waves_per_eu(3))) void k_fit_finish(SolveArgs a) {
    constexpr int NF = Dim<D>::NF, NU = Dim<D>::NU, FP = D + 1;
    __shared__ FusedShared<NET> sh;
    NetLane<D> nl;
    nl.have = false;
    int own_i = 0;
    double own_st[NF], own_x[D];
    if constexpr (NET) {
        mlp_shared_load(a.ms.theta, sh.w);
        nl.feat = sh.feat[threadIdx.x];
        __syncthreads();
    }
    int limited = 0;
    for_work<MODE>(a, a.sc->head[0], [&](int s, int t) {
        float B[NF * NU];
        double inv_r;
        if (!lw_fit_one<D, float, false, true, PER>(a, s, t, B, &inv_r)) return;
        const Sorted &srt = a.srt;
        int k = a.count[s];
        if (k > a.cfg.max_nb) k = a.cfg.max_nb;
        const double xi[3] = {srt.x[0][s], srt.x[1][s], D == 3 ? srt.x[2][s] : 0.0};
        double st[NF];
        st[0] = srt.V[s];
#pragma unroll
        for (int q = 0; q < D; ++q) st[1 + q] = srt.u[q][s];
        st[FP] = srt.P[s];
        const double h = srt.h[s];
        const DerCoef<D> ds{B, inv_r};
        limited += finish_particle<D, float, PER>(srt, a.p, a.cfg, a.sc, a.nbr, a.ldn, s, srt.id[s], k, a.sc->dt,
                                                  xi, st, h, a.cfg.kappa * h, ds, 0, 0, a.ms.feat ? &a.ms : nullptr,
                                                  NET ? &nl : nullptr, a.octc ? a.octc[s] : ~0ull)
                       ? 1
                       : 0;
        if (NET && nl.have) {
            own_i = srt.id[s];
#pragma unroll
            for (int f = 0; f < NF; ++f) own_st[f] = st[f];
#pragma unroll
            for (int q = 0; q < D; ++q) own_x[q] = xi[q];
        }
    });
    if constexpr (NET) {
        if (!nl.have)
#pragma unroll
            for (int q = 0; q < MLP_IN; ++q) nl.feat[q] = 0.f;
        __syncthreads();
        const int l = threadIdx.x & 63, wv = threadIdx.x >> 6;
        const float *wfeat = sh.feat[64 * wv];
        // tile t: the wave's lanes 16 t .. 16 t + 15; after it, lane l of
        // quarter t holds the output of lane l's particle
        float z = 0.f;
#pragma unroll
        for (int t = 0; t < 4; ++t) {
            const bf16x4 x = load_x(wfeat, 16 * t + (l & 15), true, MLP_IN + 1);
            f32x4 d1[4], d2[4];
            bf16x4 h1[4];
            const float zt = forward(SharedWeights{sh.w}, x, d1, h1, d2);
            if ((l >> 4) == t) z = zt;
        }
        unsigned long long used = 0, plain = 0, lim = 0;
        if (nl.have) {
            double lwd[NF], uwd[NF];
#pragma unroll
            for (int f = 0; f < NF; ++f) {
                lwd[f] = (double)nl.lw[f];
                uwd[f] = (double)nl.uw[f];
            }
            mlp_blend_update<D>(a.cfg, a.p, a.sc, own_i, a.sc->dt, z, nl.in_range, own_st, lwd, uwd, own_x,
                                nl.phi_plain, nl.mf, used, plain, lim);
        }
        mlp_block_counts(a.sc, used, plain, lim);
    } else {
        block_add_limited(a.sc, limited);
    }
}

// The fits queued for refinement (condition estimate above refine_cond):
// the refinement step from the factor and FP32 solution the fit stored, so
// that each result is the always-refining launch's; after the fused kernel
// (FINISH) each refined particle is updated here.  Grid-stride over the
// device-side queue length.  PER: some axis is periodic.
template <int D, bool FINISH, bool PER = true>
__global__ __launch_bounds__(LP_BLOCK) void k_lw_refine(SolveArgs a) {
    constexpr int NU = Dim<D>::NU, NF = Dim<D>::NF, NG = Dim<D>::NG, FP = D + 1;
    const int n = a.sc->n_refine;
    int limited = 0;
    for (int w = blockIdx.x * blockDim.x + threadIdx.x; w < n; w += gridDim.x * blockDim.x) {
        const int s = a.rq[2 * w], t = a.rq[2 * w + 1];
        const Sorted &srt = a.srt;
        int k = a.count[s];
        if (k > a.cfg.max_nb) k = a.cfg.max_nb;
        const double xi[3] = {srt.x[0][s], srt.x[1][s], D == 3 ? srt.x[2][s] : 0.0};
        double st[NF];
        st[0] = srt.V[s];
#pragma unroll
        for (int q = 0; q < D; ++q) st[1 + q] = srt.u[q][s];
        st[FP] = srt.P[s];
        const double inv_r = 1.0 / (a.cfg.kappa * srt.h[s]);
        const float *keep = a.rkeep + (int64_t)w * RefineKeep<D>::N;
        float G[NG], inv[NU], B[NF * NU];
#pragma unroll
        for (int q = 0; q < NG; ++q) G[q] = keep[q];
#pragma unroll
        for (int q = 0; q < NU; ++q) inv[q] = keep[NG + q];
#pragma unroll
        for (int q = 0; q < NF * NU; ++q) B[q] = keep[NG + NU + q];
        limited += lw_refine_tail<D, FINISH, 4, PER>(a, s, t, k, xi, st, inv_r, G, inv, B) ? 1 : 0;
    }
    if (FINISH) block_add_limited(a.sc, limited);
}

// Grid of a persistent launch: the blocks that can be resident at once.
// Resident blocks per CU are queried once per (kernel, block size), so that a
// launch under stream capture makes no runtime query.
static unsigned persistent_grid(const void *kernel, int block, int n_total_cap) {
    static int n_cu = 0;
    struct Occ { const void *k; int block, per_cu; };
    static Occ occ[32];
    static int n_occ = 0;
    if (n_cu == 0) {
        int dev = 0;
        hipDeviceProp_t prop;
        if (hipGetDevice(&dev) == hipSuccess && hipGetDeviceProperties(&prop, dev) == hipSuccess)
            n_cu = prop.multiProcessorCount;
        if (n_cu <= 0) n_cu = 256;
    }
    int per_cu = 0;
    for (int q = 0; q < n_occ; ++q)
        if (occ[q].k == kernel && occ[q].block == block) per_cu = occ[q].per_cu;
    if (per_cu <= 0) {
        if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, kernel, block, 0) != hipSuccess || per_cu <= 0)
            per_cu = 1;
        (void)hipGetLastError();
        if (n_occ < 32) occ[n_occ++] = {kernel, block, per_cu};
    }
    uint64_t g = (uint64_t)n_cu * per_cu;
    uint64_t need = ((uint64_t)n_total_cap + block - 1) / block;
    if (g > need) g = need;
    return g < 1 ? 1u : (unsigned)g;
}

template <int D, typename T, bool RF, int MODE>
static void launch_solve_t(const SolveArgs &a, int n_total_cap, int block, void (*between)(void *),
                           void *between_arg, hipStream_t st) {
    unsigned blocks = (unsigned)((n_total_cap + block - 1) / block);
    if (blocks < 1) blocks = 1;
    const bool refine_queue = sizeof(T) == 4 && !RF && a.rq && a.cfg.refine && a.cfg.refine_cond > 0.0f;
    // refinement: one wave per block, so that the few queued fits spread over the CUs
    unsigned gr = (unsigned)((n_total_cap + 63) / 64);
    gr = gr < 1 ? 1 : (gr > 4096 ? 4096 : gr);
    if constexpr (std::is_same<T, float>::value && !RF) {
        // FP32 fits refined where ill-conditioned (or not at all): fused
        bool per = false;
        for (int q = 0; q < D; ++q) per = per || a.cfg.periodic[q] != 0;
        if constexpr (MODE != WQ_PERSISTENT) {
            const bool net = a.ms.feat && a.ms.theta;
            if (net && per)
                hipLaunchKernelGGL((k_fit_finish<D, MODE, true, true>), dim3(blocks), dim3(block), 0, st, a);
            else if (net)
                hipLaunchKernelGGL((k_fit_finish<D, MODE, true, false>), dim3(blocks), dim3(block), 0, st, a);
            else if (per)
                hipLaunchKernelGGL((k_fit_finish<D, MODE, false, true>), dim3(blocks), dim3(block), 0, st, a);
            else
                hipLaunchKernelGGL((k_fit_finish<D, MODE, false, false>), dim3(blocks), dim3(block), 0, st, a);
        } else {
            const void *kf = per ? (const void *)k_fit_finish<D, MODE, false, true>
                                 : (const void *)k_fit_finish<D, MODE, false, false>;
            const unsigned gff = persistent_grid(kf, block, n_total_cap);
            if (per)
                hipLaunchKernelGGL((k_fit_finish<D, MODE, false, true>), dim3(gff), dim3(block), 0, st, a);
            else
                hipLaunchKernelGGL((k_fit_finish<D, MODE, false, false>), dim3(gff), dim3(block), 0, st, a);
        }
        if (refine_queue) {
            if (per)
                hipLaunchKernelGGL((k_lw_refine<D, true, true>), dim3(gr), dim3(64), 0, st, a);
            else
                hipLaunchKernelGGL((k_lw_refine<D, true, false>), dim3(gr), dim3(64), 0, st, a);
        }
        if (between) between(between_arg);
        return;
    }
    unsigned gf = blocks, gu = blocks;
    if (MODE == WQ_PERSISTENT) {
        gf = persistent_grid((const void *)k_lw_fit<D, T, RF, MODE>, block, n_total_cap);
        gu = persistent_grid((const void *)k_finish<D, T, MODE>, block, n_total_cap);
    }
    hipLaunchKernelGGL((k_lw_fit<D, T, RF, MODE>), dim3(gf), dim3(block), 0, st, a);
    if (refine_queue) hipLaunchKernelGGL((k_lw_refine<D, false>), dim3(gr), dim3(64), 0, st, a);
    if (between) between(between_arg);
    hipLaunchKernelGGL((k_finish<D, T, MODE>), dim3(gu), dim3(block), 0, st, a);
}

int der_count(int D) { return D == 3 ? Der<3>::N : Der<2>::N; }
int refine_keep_count(int D) { return D == 3 ? RefineKeep<3>::N : RefineKeep<2>::N; }

template <int D, typename T, bool RF>
static void launch_solve_m(const SolveArgs &a, int n_total_cap, int block, int mode, void (*between)(void *),
                           void *between_arg, hipStream_t st) {
    if (mode == WQ_PERSISTENT) launch_solve_t<D, T, RF, WQ_PERSISTENT>(a, n_total_cap, block, between, between_arg, st);
    else if (mode == WQ_QUEUE) launch_solve_t<D, T, RF, WQ_QUEUE>(a, n_total_cap, block, between, between_arg, st);
    else launch_solve_t<D, T, RF, WQ_DIRECT>(a, n_total_cap, block, between, between_arg, st);
}

bool solve_fuses_network(const SolveArgs &a, int mode) {
    if (a.wq == nullptr) mode = WQ_DIRECT;
    const bool refine_all = a.cfg.refine && !(a.cfg.refine_cond > 0.0f && a.rq);
    return a.ms.feat && a.ms.theta && a.cfg.precision == LP_MIXED && !refine_all && mode != WQ_PERSISTENT;
}

void launch_solve(const SolveArgs &a, int n_total_cap, int block, int mode, void (*between)(void *),
                  void *between_arg, hipStream_t st) {
    if (a.wq == nullptr) mode = WQ_DIRECT;
    const bool mixed = a.cfg.precision == LP_MIXED;
    // refine_cond > 0: the FP32 fit queues the fits to refine for k_lw_refine
    const bool refine_all = a.cfg.refine && !(a.cfg.refine_cond > 0.0f && a.rq);
    if (a.cfg.D == 3) {
        if (!mixed) launch_solve_m<3, double, false>(a, n_total_cap, block, mode, between, between_arg, st);
        else if (refine_all) launch_solve_m<3, float, true>(a, n_total_cap, block, mode, between, between_arg, st);
        else launch_solve_m<3, float, false>(a, n_total_cap, block, mode, between, between_arg, st);
    } else {
        if (!mixed) launch_solve_m<2, double, false>(a, n_total_cap, block, mode, between, between_arg, st);
        else if (refine_all) launch_solve_m<2, float, true>(a, n_total_cap, block, mode, between, between_arg, st);
        else launch_solve_m<2, float, false>(a, n_total_cap, block, mode, between, between_arg, st);
    }
    (void)hipGetLastError();
}

// ---------------------------------------------------------------------------
// Work queue: within every tile of 256, 512 or LP_QTILE consecutive cell-order particles,
// a counting sort by neighbour count (largest first; ghosts, which need no
// solve, last).  Tiles stay in cell order, so the data a wave gathers stays
// local; inside a tile the lanes of a wave get similar loop lengths.
// ---------------------------------------------------------------------------
#define LP_NBIN 258  // counts 0..256 plus the ghost bin
__global__ __launch_bounds__(LP_QTILE) void k_bin_tiles(const int *count, const int *sid, const int *n_total_dev,
                                                        int n_real, int max_nb, int *wq) {
    __shared__ unsigned hist[LP_NBIN];
    __shared__ unsigned offs[LP_NBIN];
    const int n_total = *n_total_dev;
    const int base = blockIdx.x * (int)blockDim.x;  // one tile per block
    if (base >= n_total) return;
    for (int b = threadIdx.x; b < LP_NBIN; b += blockDim.x) hist[b] = 0u;
    __syncthreads();
    const int s = base + threadIdx.x;
    int bin = 0;
    unsigned rank = 0u;
    if (s < n_total) {
        if (sid[s] >= n_real) {
            bin = LP_NBIN - 1;
        } else {
            int k = count[s];
            k = k < max_nb ? k : max_nb;
            bin = max_nb - k;
        }
        rank = atomicAdd(&hist[bin], 1u);
    }
    __syncthreads();
    if (threadIdx.x < 64) {
        constexpr int PER = (LP_NBIN + 63) / 64;
        const int lane = threadIdx.x;
        unsigned loc[PER], sum = 0u;
#pragma unroll
        for (int q = 0; q < PER; ++q) {
            int b = lane * PER + q;
            loc[q] = b < LP_NBIN ? hist[b] : 0u;
            sum += loc[q];
        }
        unsigned incl = sum;
#pragma unroll
        for (int o = 1; o < 64; o <<= 1) {
            unsigned v = __shfl_up(incl, o);
            if (lane >= o) incl += v;
        }
        unsigned run = incl - sum;
#pragma unroll
        for (int q = 0; q < PER; ++q) {
            int b = lane * PER + q;
            if (b < LP_NBIN) offs[b] = run;
            run += loc[q];
        }
    }
    __syncthreads();
    if (s < n_total) wq[base + (int)(offs[bin] + rank)] = s;
}

void launch_bin_tiles(const int *count, const int *sid, const int *n_total_dev, int n_total_cap, int n_real,
                      int max_nb, int tile, int *wq, hipStream_t st) {
    if (tile != 256 && tile != 512) tile = LP_QTILE;
    unsigned blocks = (unsigned)((n_total_cap + tile - 1) / tile);
    if (blocks < 1) blocks = 1;
    hipLaunchKernelGGL(k_bin_tiles, dim3(blocks), dim3(tile), 0, st, count, sid, n_total_dev, n_real, max_nb, wq);
    (void)hipGetLastError();
}

// ---------------------------------------------------------------------------
// Wave-cooperative Householder QR with column pivoting (one wave, one row per
// lane).  a[N]: this lane's row, b[NR]: its right-hand sides.  Rows at lanes
// >= m are zero.  Returns |R11|/|Rnn| and the solution X[q][c] (all lanes).
// ---------------------------------------------------------------------------
__device__ __forceinline__ double wave_sum(double v) {
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o);
    return v;
}

template <int N, int NR>
__device__ __forceinline__ double wave_qrp_solve(double a[N], double b[NR], double X[N][NR]) {
    const int l = threadIdx.x & 63;
    int perm[N];
#pragma unroll
    for (int j = 0; j < N; ++j) perm[j] = j;
#pragma unroll
    for (int p = 0; p < N; ++p) {
        // pivot: remaining column of largest norm over rows p..
        int best = p;
        double bn = -1.0;
#pragma unroll
        for (int j = p; j < N; ++j) {
            double c = wave_sum(l >= p ? a[j] * a[j] : 0.0);
            if (c > bn) { bn = c; best = j; }
        }
#pragma unroll
        for (int j = p + 1; j < N; ++j)
            if (j == best) {  // wave-uniform
                double t = a[p]; a[p] = a[j]; a[j] = t;
                int u = perm[p]; perm[p] = perm[j]; perm[j] = u;
            }
        double x0 = __shfl(a[p], p);
        double sigma = wave_sum(l > p ? a[p] * a[p] : 0.0);
        double normx = sqrt(x0 * x0 + sigma);
        if (normx == 0.0) continue;
        double alpha = x0 >= 0.0 ? -normx : normx;
        double v0 = x0 - alpha;
        double tau = -1.0 / (alpha * v0);
        double v = l == p ? v0 : (l > p ? a[p] : 0.0);
#pragma unroll
        for (int j = p + 1; j < N; ++j) {
            double w = wave_sum(v * a[j]) * tau;
            a[j] -= w * v;
        }
#pragma unroll
        for (int c = 0; c < NR; ++c) {
            double w = wave_sum(v * b[c]) * tau;
            b[c] -= w * v;
        }
        a[p] = l == p ? alpha : (l > p ? 0.0 : a[p]);
    }
    double r11 = fabs(__shfl(a[0], 0));
    double rnn = fabs(__shfl(a[N - 1], N - 1));
    double cond = rnn == 0.0 ? INFINITY : r11 / rnn;
    double y[N][NR];
#pragma unroll
    for (int p = N - 1; p >= 0; --p) {
        double d = a[p];
#pragma unroll
        for (int c = 0; c < NR; ++c) {
            double t = b[c];
#pragma unroll
            for (int j = p + 1; j < N; ++j) t -= a[j] * y[j][c];
            double v = d == 0.0 ? 0.0 : t / d;
            y[p][c] = __shfl(v, p);
        }
    }
#pragma unroll
    for (int q = 0; q < N; ++q)
#pragma unroll
        for (int c = 0; c < NR; ++c) {
            double v = 0.0;
#pragma unroll
            for (int pp = 0; pp < N; ++pp)
                if (perm[pp] == q) v = y[pp][c];
            X[q][c] = v;
        }
    return cond;
}

// Second-order fit of particle s by the wave QR, with the deficiency rule of
// the definition: k < NU or |R11|/|Rnn| > cond_max -> linear fit on the same
// rows (status 1); fewer than D usable rows -> status 2.
// fj_of(j, f) returns field f of neighbour j; fi[f] the particle's own values.
template <int D, int NF, typename FJ>
__device__ __forceinline__ int lw_fit_wave(const Sorted &srt, const DevCfg &cfg, const int *nbr, int ldn, int s, int k,
                                          const double xi[3], double r, const double fi[NF], FJ &&fj_of,
                                          double grad[NF][3], double hess[NF][Dim<D>::NS], int *sel_lds) {
    constexpr int NU = Dim<D>::NU, NS = Dim<D>::NS;
    const int l = threadIdx.x & 63;
    __shared__ int m_sh;
    if (l == 0) {
        int m = 0;
        for_lw_stencil<D>(srt, cfg, nbr, ldn, s, k, xi, [&](int j, const double dx[3]) { sel_lds[m++] = j; });
        m_sh = m;
    }
    __syncthreads();
    const int m = m_sh;
    const double inv_r = 1.0 / r;
    double row[NU], b[NF];
#pragma unroll
    for (int q = 0; q < NU; ++q) row[q] = 0.0;
#pragma unroll
    for (int f = 0; f < NF; ++f) b[f] = 0.0;
    if (l < m) {
        int j = sel_lds[l];
        double dx[3];
        displacement<D>(srt, cfg, j, xi, dx);
        double x[3];
#pragma unroll
        for (int a = 0; a < D; ++a) x[a] = dx[a] / r;
        second_order_row<D, double>(x, row);
#pragma unroll
        for (int f = 0; f < NF; ++f) b[f] = fj_of(j, f) - fi[f];
    }
#pragma unroll
    for (int f = 0; f < NF; ++f) {
#pragma unroll
        for (int a = 0; a < 3; ++a) grad[f][a] = 0.0;
#pragma unroll
        for (int q = 0; q < NS; ++q) hess[f][q] = 0.0;
    }
    int status = 0;
    double cond = INFINITY;
    double X[NU][NF];
    double a2[NU], b2[NF];
#pragma unroll
    for (int q = 0; q < NU; ++q) a2[q] = row[q];
#pragma unroll
    for (int f = 0; f < NF; ++f) b2[f] = b[f];
    if (m >= NU) cond = wave_qrp_solve<NU, NF>(a2, b2, X);
    if (m >= NU && cond <= cfg.cond_max) {
#pragma unroll
        for (int f = 0; f < NF; ++f) {
#pragma unroll
            for (int a = 0; a < D; ++a) grad[f][a] = X[a][f] * inv_r;
#pragma unroll
            for (int q = 0; q < NS; ++q) hess[f][q] = X[D + q][f] * (inv_r * inv_r);
        }
    } else {
        status = 1;
        double a1[D], b1[NF], X1[D][NF];
#pragma unroll
        for (int q = 0; q < D; ++q) a1[q] = row[q];
#pragma unroll
        for (int f = 0; f < NF; ++f) b1[f] = b[f];
        double c1 = INFINITY;
        if (m >= D) c1 = wave_qrp_solve<D, NF>(a1, b1, X1);
        if (m >= D && c1 <= cfg.cond_max) {
#pragma unroll
            for (int f = 0; f < NF; ++f)
#pragma unroll
                for (int a = 0; a < D; ++a) grad[f][a] = X1[a][f] * inv_r;
        } else {
            status = 2;
        }
    }
    return status;
}

template <int D>
__global__ __launch_bounds__(64) void k_solve_fallback(Sorted srt, Soa p, const int *nbr, int ldn, const int *count,
                                                       int n_real, DevCfg cfg, DevScalars *sc, const int *queue,
                                                       MlpStage ms) {
    constexpr int NF = Dim<D>::NF, NS = Dim<D>::NS, FP = D + 1;
    __shared__ int sel[64];
    const int nq = sc->n_fallback;
    for (int w = blockIdx.x; w < nq; w += gridDim.x) {
        int s = queue[w];
        int i = srt.id[s];
        int k = count[s];
        if (k > cfg.max_nb) k = cfg.max_nb;
        double xi[3] = {srt.x[0][s], srt.x[1][s], D == 3 ? srt.x[2][s] : 0.0};
        double st[NF];
        st[0] = srt.V[s];
        for (int a = 0; a < D; ++a) st[1 + a] = srt.u[a][s];
        st[FP] = srt.P[s];
        const double h = srt.h[s];
        const double r = cfg.kappa * h;
        double grad[NF][3], hess[NF][NS];
        int status = lw_fit_wave<D, NF>(srt, cfg, nbr, ldn, s, k, xi, r, st,
                                        [&](int j, int f) {
                                            return f == 0 ? srt.V[j] : (f == FP ? srt.P[j] : srt.u[f - 1][j]);
                                        },
                                        grad, hess, sel);
        if ((threadIdx.x & 63) == 0 &&
            finish_particle<D, double>(srt, p, cfg, sc, nbr, ldn, s, i, k, sc->dt, xi, st, h, r,
                                       DerRegs<D>{grad, hess}, status, LP_FLAG_FALLBACK, ms.feat ? &ms : nullptr))
            atomicAdd(&sc->n_limited, 1ull);
        __syncthreads();
    }
}

void launch_solve_fallback(const Sorted &s, const Soa &p, const int *nbr, int ldn, const int *count, int n_real,
                           const DevCfg &cfg, DevScalars *sc, const int *queue, int queue_cap, const MlpStage &ms,
                           hipStream_t st) {
    unsigned blocks = queue_cap < 2048 ? (unsigned)(queue_cap > 0 ? queue_cap : 1) : 2048u;
    if (cfg.D == 3)
        hipLaunchKernelGGL(k_solve_fallback<3>, dim3(blocks), dim3(64), 0, st, s, p, nbr, ldn, count, n_real, cfg, sc,
                           queue, ms);
    else
        hipLaunchKernelGGL(k_solve_fallback<2>, dim3(blocks), dim3(64), 0, st, s, p, nbr, ldn, count, n_real, cfg, sc,
                           queue, ms);
    (void)hipGetLastError();
}

// ---------------------------------------------------------------------------
// Derivative operator alone (lp_gfd): FP64 normal-equation fit with the same
// fallback rule, nf <= 5 fields given in cell order.
// ---------------------------------------------------------------------------
struct FieldPtrs { const double *f[5]; };

template <int D>
__global__ __launch_bounds__(LP_BLOCK) void k_gfd(Sorted srt, FieldPtrs fs, int nf, const int *nbr, int ldn,
                                                  const int *count, int n, DevCfg cfg, DevScalars *sc, int *queue,
                                                  double *deriv, uint8_t *status) {
    constexpr int NU = Dim<D>::NU, NG = Dim<D>::NG, NS = Dim<D>::NS;
    int s = blockIdx.x * blockDim.x + threadIdx.x;
    if (s >= n) return;
    int i = srt.id[s];
    int k = count[s];
    if (k > cfg.max_nb) k = cfg.max_nb;
    double xi[3] = {srt.x[0][s], srt.x[1][s], D == 3 ? srt.x[2][s] : 0.0};
    const double r = srt.r[s];
    const double inv_r = 1.0 / r;
    double fi[5];
#pragma unroll
    for (int f = 0; f < 5; ++f) fi[f] = f < nf ? fs.f[f][s] : 0.0;
    double G[NG], B[5 * NU];
#pragma unroll
    for (int q = 0; q < NG; ++q) G[q] = 0;
#pragma unroll
    for (int q = 0; q < 5 * NU; ++q) B[q] = 0;
    int m = 0;
    auto member = [&](const double dx[3], const double *fj) {
        double x[3];
#pragma unroll
        for (int a = 0; a < D; ++a) x[a] = dx[a] * inv_r;
        double row[NU];
        second_order_row<D, double>(x, row);
#pragma unroll
        for (int pp = 0; pp < NU; ++pp)
#pragma unroll
            for (int qq = pp; qq < NU; ++qq) G[tri(pp, qq, NU)] += row[pp] * row[qq];
#pragma unroll
        for (int f = 0; f < 5; ++f) {
            if (f >= nf) break;
            double b = fj[f] - fi[f];
#pragma unroll
            for (int pp = 0; pp < NU; ++pp) B[f * NU + pp] += row[pp] * b;
        }
        ++m;
    };
    if (srt.rec) {
        // the caller's fields in the gather records (nf <= D + 2), walked one
        // entry ahead as in the step's fit
        for_lw_stencil_rec<D>(srt, cfg, nbr, ldn, s, k, xi,
                              [&](int, const double dx[3], const double fr[D + 2]) { member(dx, fr); });
    } else {
        for_lw_stencil<D>(srt, cfg, nbr, ldn, s, k, xi, [&](int j, const double dx[3]) {
            double fj[5];
#pragma unroll
            for (int f = 0; f < 5; ++f) fj[f] = f < nf ? fs.f[f][j] : 0.0;
            member(dx, fj);
        });
    }
    double inv[NU];
    bool good = m >= NU && cholesky<NU, double>(G, inv);
    if (good) good = cond_estimate<NU, double>(G, inv) <= cfg.cond_fb;
    if (!good) {
        int slot = atomicAdd(&sc->n_fallback, 1);
        queue[slot] = s;
        return;
    }
    chol_solve<NU, 5, double, double>(G, inv, B);
    const int nu = NU;
#pragma unroll
    for (int f = 0; f < 5; ++f) {
        if (f >= nf) break;  // constant indices keep the arrays in registers
        for (int a = 0; a < D; ++a) deriv[((int64_t)f * nu + a) * n + i] = B[f * NU + a] * inv_r;
        for (int q = 0; q < NS; ++q) deriv[((int64_t)f * nu + D + q) * n + i] = B[f * NU + D + q] * inv_r * inv_r;
    }
    status[i] = 0;
}

template <int D>
__global__ __launch_bounds__(64) void k_gfd_fallback(Sorted srt, FieldPtrs fs, int nf, const int *nbr, int ldn,
                                                     const int *count, int n, DevCfg cfg, DevScalars *sc,
                                                     const int *queue, double *deriv, uint8_t *status) {
    constexpr int NU = Dim<D>::NU, NS = Dim<D>::NS;
    __shared__ int sel[64];
    const int nq = sc->n_fallback;
    for (int w = blockIdx.x; w < nq; w += gridDim.x) {
        int s = queue[w];
        int i = srt.id[s];
        int k = count[s];
        if (k > cfg.max_nb) k = cfg.max_nb;
        double xi[3] = {srt.x[0][s], srt.x[1][s], D == 3 ? srt.x[2][s] : 0.0};
        double fi[5];
        for (int f = 0; f < 5; ++f) fi[f] = f < nf ? fs.f[f][s] : 0.0;
        double grad[5][3], hess[5][NS];
        int st = lw_fit_wave<D, 5>(srt, cfg, nbr, ldn, s, k, xi, srt.r[s], fi,
                                   [&](int j, int f) { return f < nf ? fs.f[f][j] : 0.0; }, grad, hess, sel);
        if ((threadIdx.x & 63) == 0) {
#pragma unroll
            for (int f = 0; f < 5; ++f) {
                if (f >= nf) break;  // constant indices keep the arrays in registers
                for (int a = 0; a < D; ++a) deriv[((int64_t)f * NU + a) * n + i] = grad[f][a];
                for (int q = 0; q < NS; ++q) deriv[((int64_t)f * NU + D + q) * n + i] = hess[f][q];
            }
            status[i] = (uint8_t)st;
        }
        __syncthreads();
    }
}

// ---------------------------------------------------------------------------
// Third-order derivative operator (lp_gfd3): the Taylor system of Sec. 2.1
// carried to the cubic terms, one wave per particle (one stencil row per
// lane), solved by pivoted Householder QR; a deficient cubic system takes the
// second-order fit of the same stencil.
// ---------------------------------------------------------------------------
template <int D> struct Dim3 { static constexpr int NU = D == 3 ? 19 : 9; };

// Second-order row followed by xi^alpha / alpha! for |alpha| = 3, in the order
// 3D: xxx, yyy, zzz, xxy, xxz, xyy, yyz, xzz, yzz, xyz; 2D: xxx, yyy, xxy, xyy.
template <int D>
__device__ __forceinline__ void third_order_row(const double xi[3], double row[Dim3<D>::NU]) {
    second_order_row<D, double>(xi, row);
    constexpr int o = Dim<D>::NU;
    const double x = xi[0], y = xi[1];
    if constexpr (D == 2) {
        row[o + 0] = x * x * x / 6.0;
        row[o + 1] = y * y * y / 6.0;
        row[o + 2] = 0.5 * x * x * y;
        row[o + 3] = 0.5 * x * y * y;
    } else {
        const double z = xi[2];
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

// degree of unknown q of the third-order fit
template <int D>
__device__ __forceinline__ int third_order_degree(int q) { return q < D ? 1 : (q < Dim<D>::NU ? 2 : 3); }

// lane permutation of a double by DPP (both halves; every lane is written)
template <int CTRL>
__device__ __forceinline__ double dpp_f64(double v) {
    const long long b = __double_as_longlong(v);
    const int lo = __builtin_amdgcn_mov_dpp((int)b, CTRL, 0xF, 0xF, false);
    const int hi = __builtin_amdgcn_mov_dpp((int)(b >> 32), CTRL, 0xF, 0xF, false);
    return __longlong_as_double(((long long)hi << 32) | (long long)(unsigned)lo);
}

// Sum over the 16 lanes of a DPP row, in every lane of the row (lanes ^ 1,
// ^ 2, then the 8- and 16-lane mirrors; each step adds two equal operands in
// either order, so every lane ends with the same bits).  All lanes active.
__device__ __forceinline__ double row_sum16(double v) {
    v += dpp_f64<0xB1>(v);
    v += dpp_f64<0x4E>(v);
    v += dpp_f64<0x141>(v);
    v += dpp_f64<0x140>(v);
    return v;
}

// row_sum16 of K values at once, stage by stage, so that no DPP read waits
// on the add just before it
template <int K>
__device__ __forceinline__ void row_sum16_k(double v[K]) {
#pragma unroll
    for (int q = 0; q < K; ++q) v[q] += dpp_f64<0xB1>(v[q]);
#pragma unroll
    for (int q = 0; q < K; ++q) v[q] += dpp_f64<0x4E>(v[q]);
#pragma unroll
    for (int q = 0; q < K; ++q) v[q] += dpp_f64<0x141>(v[q]);
#pragma unroll
    for (int q = 0; q < K; ++q) v[q] += dpp_f64<0x140>(v[q]);
}

// value of lane src (0..15) of the caller's 16-lane row
__device__ __forceinline__ double row_bcast16(double v, int src) {
    return __shfl(v, src, 16);
}

// The Lax-Wendroff stencil of for_lw_stencil, chosen by a 16-lane group (one
// particle): list entries are taken 16 at a time, one per lane; per-octant
// ballots of the group give the octant counts and each entry's rank within
// its octant, and the members taken are compacted into sel[] in list order.
// Returns their number (at most lw_cap <= 64).  The same members in the same
// order as for_lw_stencil.
template <int D>
__device__ __forceinline__ int group_lw_select(const Sorted &srt, const DevCfg &cfg, const int *nbr, int ldn, int s,
                                               int k, const double xi[3], int *sel) {
    const int gl = threadIdx.x & 15, gshift = threadIdx.x & 48;
    const unsigned below = (1u << gl) - 1u;
    const int cap = cfg.lw_cap;
    auto gballot = [&](bool pr) -> unsigned { return (unsigned)((__ballot(pr) >> gshift) & 0xFFFFull); };
    auto entry = [&](int t, int &j, int &o) {
        j = 0;
        o = -1;
        if (t < k) {
            j = nb_at(nbr, ldn, s, t);
            double dx[3];
            displacement<D>(srt, cfg, j, xi, dx);
            o = octant<D>(dx);
        }
    };
    if (k <= cap) {
        for (int t0 = 0; t0 < k; t0 += 16)
            if (t0 + gl < k) sel[t0 + gl] = nb_at(nbr, ldn, s, t0 + gl);
        return k;
    }
    // octant counts, then the round R* taken whole and rem of round R*
    int cnt[8];
#pragma unroll
    for (int q = 0; q < 8; ++q) cnt[q] = 0;
    for (int t0 = 0; t0 < k; t0 += 16) {
        int j, o;
        entry(t0 + gl, j, o);
#pragma unroll
        for (int q = 0; q < 8; ++q) cnt[q] += __popc(gballot(o == q));
    }
    int R = 0, taken = 0;
    for (;;) {
        int next = 0;
#pragma unroll
        for (int q = 0; q < 8; ++q) next += cnt[q] < R + 1 ? cnt[q] : R + 1;
        if (next > cap) break;
        taken = next;
        ++R;
    }
    const int rem = cap - taken;
    int seen[8];  // entries of each octant in earlier chunks
#pragma unroll
    for (int q = 0; q < 8; ++q) seen[q] = 0;
    int seenR = 0, m = 0;  // entries of round R in earlier chunks; members taken
    for (int t0 = 0; t0 < k; t0 += 16) {
        int j, o;
        entry(t0 + gl, j, o);
        int rho = 0;
#pragma unroll
        for (int q = 0; q < 8; ++q) {
            const unsigned mq = gballot(o == q);
            if (o == q) rho = seen[q] + __popc(mq & below);
            seen[q] += __popc(mq);
        }
        const unsigned onR = gballot(o >= 0 && rho == R);
        const bool take = o >= 0 && (rho < R || (rho == R && seenR + __popc(onR & below) < rem));
        seenR += __popc(onR);
        const unsigned mt = gballot(take);
        if (take) sel[m + __popc(mt & below)] = j;
        m += __popc(mt);
    }
    return m;
}

// The rows of a 16-lane group's system, ROWS slots per lane: the first RR
// in registers, the others (at most one) in LDS, column j of that slot at
// l[64 j] (l: this lane's entry of a 64-lane array, so that the lanes of a
// wave read consecutive words).  Indices fold to constants where the
// callers' loops are unrolled.
template <int N, int RR>
struct GroupRows {
    static constexpr int kRR = RR;
    double r[RR][N];
    double *l;
    __device__ __forceinline__ double &operator()(int c, int j) { return c < RR ? r[c][j] : l[64 * j]; }
    __device__ __forceinline__ double operator()(int c, int j) const { return c < RR ? r[c][j] : l[64 * j]; }
};

// Pivoted Householder QR of a 16-lane group's rows.  Row q of the system
// (q < 16 ROWS; rows past the stencil are zero) is a(q / 16, .) of lane q % 16.
// The pivot is the remaining column of largest norm over the remaining rows.
// Each dot product adds the lane's rows, then the 16 lanes (DPP row sums,
// every lane of the wave takes part).  On return a holds R above the
// diagonal and the reflectors below it (the reflector's head v0 on the
// diagonal); the group's LDS arrays hold the column order perm, R's diagonal
// alpha and the reflector scales tau (written by lane 0).  Returns
// |R11| / |Rnn|.
template <int N, int ROWS, class M>
__device__ __forceinline__ double group_qrp(M &a, int *perm, double *alpha_out, double *tau_out) {
    const int gl = threadIdx.x & 15;
    if (gl == 0)
        for (int j = 0; j < N; ++j) perm[j] = j;
    double r11 = 0.0, rnn = 0.0;
#pragma clang loop unroll(full)
    for (int p = 0; p < N; ++p) {
        int best = p;
        double bn = -1.0;
        // norms of the remaining columns over rows >= p, three at a time
#pragma clang loop unroll(full)
        for (int j0 = p; j0 < N; j0 += 3) {
            double part[3];
#pragma clang loop unroll(full)
            for (int e = 0; e < 3; ++e) {
                const int j = j0 + e < N ? j0 + e : N - 1;
                part[e] = 0.0;
#pragma clang loop unroll(full)
                for (int c = 0; c < ROWS; ++c)
                    if (16 * c + 15 >= p)  // else every row of slot c is above p
                        part[e] += (16 * c >= p || gl + 16 * c >= p) ? a(c, j) * a(c, j) : 0.0;
            }
            row_sum16_k<3>(part);
#pragma clang loop unroll(full)
            for (int e = 0; e < 3; ++e)
                if (j0 + e < N && part[e] > bn) {
                    bn = part[e];
                    best = j0 + e;
                }
        }
        // best is the same in the 16 lanes of a group (groups differ); the
        // swap is written as selects, so that every column keeps a register
        // (a slot in LDS swaps its two words by address)
#pragma clang loop unroll(full)
        for (int j = p + 1; j < N; ++j) {
            const bool sw = j == best;
#pragma clang loop unroll(full)
            for (int c = 0; c < ROWS && c < M::kRR; ++c) {
                const double t = a(c, p), u = a(c, j);
                a(c, p) = sw ? u : t;
                a(c, j) = sw ? t : u;
            }
        }
        if constexpr (ROWS > M::kRR) {
            const double t = a.l[64 * p], u = a.l[64 * best];
            a.l[64 * p] = u;
            a.l[64 * best] = t;
        }
        const double x0 = row_bcast16(a(p / 16, p), p % 16);
        double sg = 0.0;
#pragma clang loop unroll(full)
        for (int c = 0; c < ROWS; ++c) sg += gl + 16 * c > p ? a(c, p) * a(c, p) : 0.0;
        const double sigma = row_sum16(sg);
        const double normx = sqrt(x0 * x0 + sigma);
        // a zero column (normx = 0) leaves the rows as they are: tau = 0
        const double alpha = x0 >= 0.0 ? -normx : normx;
        const double v0 = x0 - alpha;
        const double tau = normx != 0.0 ? -1.0 / (alpha * v0) : 0.0;
        double v[ROWS];
#pragma clang loop unroll(full)
        for (int c = 0; c < ROWS; ++c) {
            const int q = gl + 16 * c;
            v[c] = q == p ? v0 : (q > p ? a(c, p) : 0.0);
            a(c, p) = q == p ? v0 : a(c, p);
        }
        // the reflector applied to the remaining columns, three at a time
#pragma clang loop unroll(full)
        for (int j0 = p + 1; j0 < N; j0 += 3) {
            double d[3];
#pragma clang loop unroll(full)
            for (int e = 0; e < 3; ++e) {
                const int j = j0 + e < N ? j0 + e : N - 1;
                d[e] = 0.0;
#pragma clang loop unroll(full)
                for (int c = 0; c < ROWS; ++c) d[e] += v[c] * a(c, j);
            }
            row_sum16_k<3>(d);
#pragma clang loop unroll(full)
            for (int e = 0; e < 3; ++e)
                if (j0 + e < N) {
                    const double w = d[e] * tau;
#pragma clang loop unroll(full)
                    for (int c = 0; c < ROWS; ++c) a(c, j0 + e) -= w * v[c];
                }
        }
        if (gl == 0) {
            if (best != p) {
                const int u = perm[p];
                perm[p] = perm[best];
                perm[best] = u;
            }
            alpha_out[p] = alpha;
            tau_out[p] = tau;
        }
        if (p == 0) r11 = fabs(alpha);
        if (p == N - 1) rnn = fabs(alpha);
    }
    return rnn == 0.0 ? INFINITY : r11 / rnn;
}

// Least squares for one right-hand side from group_qrp's factors: the
// reflectors applied to b (row q in b[q / 16] of lane q % 16), then back
// substitution; on return row p of b holds the solution for unknown perm[p].
template <int N, int ROWS, class M>
__device__ __forceinline__ void group_qr_solve(const M &a, const double *alpha, const double *tau,
                                               double b[ROWS]) {
    const int gl = threadIdx.x & 15;
#pragma unroll
    for (int p = 0; p < N; ++p) {
        double d = 0.0;
#pragma unroll
        for (int c = 0; c < ROWS; ++c) d += gl + 16 * c >= p ? a(c, p) * b[c] : 0.0;
        const double w = row_sum16(d) * tau[p];
#pragma unroll
        for (int c = 0; c < ROWS; ++c) b[c] -= gl + 16 * c >= p ? w * a(c, p) : 0.0;
    }
    // row p of R: alpha[p] on the diagonal, a(p / 16, j > p) of lane p % 16
#pragma unroll
    for (int p = N - 1; p >= 0; --p) {
        const double dg = alpha[p];
        const double t = (gl == p % 16 && dg != 0.0) ? b[p / 16] / dg : 0.0;
        const double yp = row_bcast16(t, p % 16);
        if (gl == p % 16) b[p / 16] = yp;
#pragma unroll
        for (int c = 0; c < ROWS; ++c)
            if (gl + 16 * c < p) b[c] -= a(c, p) * yp;
    }
}

// Four particles per wave, one 16-lane group (a DPP row) each, up to four
// stencil rows per lane.  A deficient cubic system (fewer members than
// unknowns, or |R11| / |Rnn| above cond_max) is queued for k_gfd3_fallback.
// The right-hand sides are gathered after the factorisation, one field at a
// time, so that only the factors stay in registers (two waves per SIMD).
template <int D>
__global__ __launch_bounds__(64) __attribute__((amdgpu_waves_per_eu(2))) void k_gfd3(Sorted srt, FieldPtrs fs, int nf, const int *nbr, int ldn,
                                             const int *count, int n, DevCfg cfg, DevScalars *sc, int *queue,
                                             double *deriv, uint8_t *status) {
    constexpr int N3 = Dim3<D>::NU, ROWS = 4;
    // 3D: the fourth row slot of every lane in LDS (registers for the rest)
    constexpr int RR = D == 3 ? 3 : 4;
    __shared__ double row4[RR < ROWS ? N3 * 64 : 1];
    __shared__ int sel_all[4][64];
    __shared__ int perm_all[4][32];
    __shared__ double alpha_all[4][32], tau_all[4][32];
    const int gl = threadIdx.x & 15, grp = (threadIdx.x >> 4) & 3;
    int *sel = sel_all[grp];
    int *perm = perm_all[grp];
    const int s = xcd_remap(blockIdx.x, gridDim.x) * 4 + grp;
    const bool real = s < n;
    const int i = real ? srt.id[s] : 0;
    int k = real ? count[s] : 0;
    if (k > cfg.max_nb) k = cfg.max_nb;
    const double xi[3] = {real ? srt.x[0][s] : 0.0, real ? srt.x[1][s] : 0.0,
                          D == 3 && real ? srt.x[2][s] : 0.0};
    const double r = real ? srt.r[s] : 1.0;
    const int m = real ? group_lw_select<D>(srt, cfg, nbr, ldn, s, k, xi, sel) : 0;
    __syncthreads();  // sel written by the group's lanes
    GroupRows<N3, RR> a;
    a.l = row4 + (threadIdx.x & 63);
#pragma unroll
    for (int c = 0; c < ROWS; ++c) {
        const int q = gl + 16 * c;
        const bool in = q < m;
        const int jrc = in ? sel[q] : (real ? s : 0);
        double dx[3];
        displacement<D>(srt, cfg, jrc, xi, dx);
        double x[3] = {0.0, 0.0, 0.0};
#pragma unroll
        for (int e = 0; e < D; ++e) x[e] = in ? dx[e] / r : 0.0;
        double row[N3];
        third_order_row<D>(x, row);
#pragma unroll
        for (int u = 0; u < N3; ++u) a(c, u) = row[u];
    }
    const double cond = group_qrp<N3, ROWS>(a, perm, alpha_all[grp], tau_all[grp]);
    __syncthreads();  // perm, alpha and tau written by lane 0 of each group
    const bool cubic = real && m >= N3 && cond <= cfg.cond_max;
    for (int f = 0; f < nf; ++f) {
        // rows past the stencil read the particle's own value: difference 0
        const double fi = real ? fs.f[f][s] : 0.0;
        double b[ROWS];
#pragma unroll
        for (int c = 0; c < ROWS; ++c) {
            const int q = gl + 16 * c;
            const int jrc = q < m ? sel[q] : (real ? s : 0);
            b[c] = real ? fs.f[f][jrc] - fi : 0.0;
        }
        group_qr_solve<N3, ROWS>(a, alpha_all[grp], tau_all[grp], b);
        if (cubic) {
#pragma unroll
            for (int c = 0; c < ROWS; ++c) {
                const int q = gl + 16 * c;
                if (q < N3) {
                    const int col = perm[q];
                    const int deg = third_order_degree<D>(col);
                    const double sp = deg == 1 ? r : (deg == 2 ? r * r : r * r * r);
                    deriv[((int64_t)f * N3 + col) * n + i] = b[c] / sp;
                }
            }
        }
    }
    if (!real) return;
    if (cubic) {
        if (gl == 0) status[i] = 0;
    } else if (gl == 0) {
        queue[atomicAdd(&sc->n_fallback, 1)] = s;
    }
}

// The deficient cubic systems: the second-order fit of the same stencil (one
// wave per queued particle), cubic columns zero, status 1 + its status.
template <int D>
__global__ __launch_bounds__(64) void k_gfd3_fallback(Sorted srt, FieldPtrs fs, int nf, const int *nbr, int ldn,
                                                      const int *count, int n, DevCfg cfg, const DevScalars *sc,
                                                      const int *queue, double *deriv, uint8_t *status) {
    constexpr int N3 = Dim3<D>::NU, NU = Dim<D>::NU, NS = Dim<D>::NS;
    __shared__ int sel[64];
    const int l = threadIdx.x & 63;
    const int nq = sc->n_fallback;
    for (int w = blockIdx.x; w < nq; w += gridDim.x) {
        const int s = queue[w];
        const int i = srt.id[s];
        int k = count[s];
        if (k > cfg.max_nb) k = cfg.max_nb;
        const double xi[3] = {srt.x[0][s], srt.x[1][s], D == 3 ? srt.x[2][s] : 0.0};
        const double r = srt.r[s];
        double fi[5];
#pragma unroll
        for (int f = 0; f < 5; ++f) fi[f] = f < nf ? fs.f[f][s] : 0.0;
        double grad[5][3], hess[5][NS];
        const int st2 = lw_fit_wave<D, 5>(srt, cfg, nbr, ldn, s, k, xi, r, fi,
                                          [&](int j, int f) { return f < nf ? fs.f[f][j] : 0.0; }, grad, hess, sel);
        if (l == 0) {
#pragma unroll
            for (int f = 0; f < 5; ++f) {
                if (f >= nf) break;  // constant indices keep the arrays in registers
                for (int a = 0; a < D; ++a) deriv[((int64_t)f * N3 + a) * n + i] = grad[f][a];
                for (int q = 0; q < NS; ++q) deriv[((int64_t)f * N3 + D + q) * n + i] = hess[f][q];
                for (int q = NU; q < N3; ++q) deriv[((int64_t)f * N3 + q) * n + i] = 0.0;
            }
            status[i] = (uint8_t)(1 + st2);
        }
        __syncthreads();
    }
}

void launch_gfd3(const Sorted &s, const double *const *fs, int nf, const int *nbr, int ldn, const int *count, int n,
                 const DevCfg &cfg, DevScalars *sc, int *queue, double *deriv, uint8_t *status, hipStream_t st) {
    FieldPtrs f{};
    for (int q = 0; q < nf && q < 5; ++q) f.f[q] = fs[q];
    const unsigned blocks = (unsigned)((n + 3) / 4 > 0 ? (n + 3) / 4 : 1);
    const unsigned fb = (unsigned)(n < 4096 ? (n > 0 ? n : 1) : 4096);
    if (cfg.D == 3) {
        hipLaunchKernelGGL(k_gfd3<3>, dim3(blocks), dim3(64), 0, st, s, f, nf, nbr, ldn, count, n, cfg, sc, queue,
                           deriv, status);
        hipLaunchKernelGGL(k_gfd3_fallback<3>, dim3(fb), dim3(64), 0, st, s, f, nf, nbr, ldn, count, n, cfg, sc,
                           queue, deriv, status);
    } else {
        hipLaunchKernelGGL(k_gfd3<2>, dim3(blocks), dim3(64), 0, st, s, f, nf, nbr, ldn, count, n, cfg, sc, queue,
                           deriv, status);
        hipLaunchKernelGGL(k_gfd3_fallback<2>, dim3(fb), dim3(64), 0, st, s, f, nf, nbr, ldn, count, n, cfg, sc,
                           queue, deriv, status);
    }
    (void)hipGetLastError();
}

void launch_gfd(const Sorted &s, const double *const *fs, int nf, const int *nbr, int ldn, const int *count, int n,
                const DevCfg &cfg, DevScalars *sc, int *queue, double *deriv, uint8_t *status, hipStream_t st) {
    FieldPtrs f{};
    for (int q = 0; q < nf && q < 5; ++q) f.f[q] = fs[q];
    unsigned blocks = (unsigned)((n + LP_BLOCK - 1) / LP_BLOCK);
    if (blocks < 1) blocks = 1;
    if (cfg.D == 3)
        hipLaunchKernelGGL(k_gfd<3>, dim3(blocks), dim3(LP_BLOCK), 0, st, s, f, nf, nbr, ldn, count, n, cfg, sc, queue,
                           deriv, status);
    else
        hipLaunchKernelGGL(k_gfd<2>, dim3(blocks), dim3(LP_BLOCK), 0, st, s, f, nf, nbr, ldn, count, n, cfg, sc, queue,
                           deriv, status);
    (void)hipGetLastError();
}

void launch_gfd_fallback(const Sorted &s, const double *const *fs, int nf, const int *nbr, int ldn, const int *count,
                         int n, const DevCfg &cfg, DevScalars *sc, const int *queue, int queue_cap, double *deriv,
                         uint8_t *status, hipStream_t st) {
    FieldPtrs f{};
    for (int q = 0; q < nf && q < 5; ++q) f.f[q] = fs[q];
    unsigned blocks = queue_cap < 2048 ? (unsigned)(queue_cap > 0 ? queue_cap : 1) : 2048u;
    if (cfg.D == 3)
        hipLaunchKernelGGL(k_gfd_fallback<3>, dim3(blocks), dim3(64), 0, st, s, f, nf, nbr, ldn, count, n, cfg, sc,
                           queue, deriv, status);
    else
        hipLaunchKernelGGL(k_gfd_fallback<2>, dim3(blocks), dim3(64), 0, st, s, f, nf, nbr, ldn, count, n, cfg, sc,
                           queue, deriv, status);
    (void)hipGetLastError();
}
