"""FP64 CPU oracle of the Lagrangian particle time step (test infrastructure only).

Only ``tests/``, ``__graft_entry__.smoke()`` and the ``cpu_baseline`` leg of
``bench.py`` import this package.  The product library never does.  The C
source (``lp_oracle.c``) follows the paper's Sec. 2.1 (GFD fit, upwind and
Lax-Wendroff rates, estimator, limiter, mover) and Sec. 2.2 (steps 1-6 of the
time-step loop); this module only marshals numpy arrays.
"""
from __future__ import annotations

import ctypes as C
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "lp_oracle.c")
_LIB = os.path.join(_HERE, "liblp_oracle.so")

FLAG_LIMITED, FLAG_DEGENERATE, FLAG_VACUUM, FLAG_SUBSTITUTED, FLAG_NUMERIC = 1, 2, 4, 8, 32
OK, E_ARG, E_CAPACITY, E_NUMERIC, E_NOMEM = 0, 1, 2, 3, 5


def build(force: bool = False) -> str:
    """Compile the oracle with gcc (plain C99, FP64, no contraction, OpenMP)."""
    if force or not os.path.exists(_LIB) or os.path.getmtime(_LIB) < max(
            os.path.getmtime(_SRC), os.path.getmtime(os.path.join(_HERE, "lp_oracle.h"))):
        tmp = _LIB + ".tmp%d" % os.getpid()
        subprocess.check_call([
            "gcc", "-O2", "-std=c99", "-fopenmp", "-ffp-contract=off", "-fno-fast-math",
            "-shared", "-fPIC", "-o", tmp, _SRC, "-lm"])
        os.replace(tmp, _LIB)
    return _LIB


class Cfg(C.Structure):
    _fields_ = [
        ("dim", C.c_int32), ("lw_cap", C.c_int32), ("uw_cap", C.c_int32), ("max_nb", C.c_int32),
        ("gamma", C.c_double), ("cfl", C.c_double), ("kappa", C.c_double),
        ("est_eps", C.c_double), ("cond_max", C.c_double), ("uw_cond_max", C.c_double),
        ("lo", C.c_double * 3), ("hi", C.c_double * 3),
        ("periodic", C.c_int32 * 3), ("wall_lo", C.c_int32 * 3), ("wall_hi", C.c_int32 * 3),
        ("vacuum", C.c_int32), ("phi_fixed", C.c_double), ("limiter_cap", C.c_double),
    ]


_lib = None


def lib():
    global _lib
    if _lib is None:
        build()
        L = C.CDLL(_LIB)
        dp = C.POINTER(C.c_double)
        ip = C.POINTER(C.c_int32)
        i64p = C.POINTER(C.c_int64)
        u8p = C.POINTER(C.c_uint8)
        cp = C.POINTER(Cfg)
        L.lpo_num_threads.restype = C.c_int
        L.lpo_num_threads.argtypes = []
        L.lpo_set_num_threads.restype = None
        L.lpo_set_num_threads.argtypes = [C.c_int]
        L.lpo_limiter.restype = C.c_double
        L.lpo_limiter.argtypes = [C.c_double]
        L.lpo_estimator_ratio.restype = C.c_double
        L.lpo_estimator_ratio.argtypes = [C.c_double, C.c_double]
        L.lpo_lstsq_qrp.restype = C.c_double
        L.lpo_lstsq_qrp.argtypes = [C.c_int, C.c_int, C.c_int, dp, dp, dp]
        L.lpo_lw_select.restype = C.c_int
        L.lpo_lw_select.argtypes = [C.c_int, C.c_int, dp, C.c_int, C.POINTER(C.c_int)]
        L.lpo_lw_rates.restype = None
        L.lpo_lw_rates.argtypes = [C.c_int, C.c_double, C.c_double, dp, dp, dp, dp]
        L.lpo_uw_rates.restype = None
        L.lpo_uw_rates.argtypes = [C.c_int, C.c_double, dp, dp, dp, dp]
        L.lpo_neighbors.restype = C.c_int
        L.lpo_neighbors.argtypes = [cp, C.c_int64, dp, dp, dp, dp, C.c_int32, ip, ip]
        L.lpo_neighbors_subset.restype = C.c_int
        L.lpo_neighbors_subset.argtypes = [cp, C.c_int64, dp, dp, dp, dp, C.c_int32, C.c_int64, i64p, ip, ip]
        L.lpo_gfd.restype = C.c_int
        L.lpo_gfd.argtypes = [cp, C.c_int64, dp, dp, dp, dp, C.c_int32, C.POINTER(dp), dp, u8p]
        L.lpo_gfd3.restype = C.c_int
        L.lpo_gfd3.argtypes = [cp, C.c_int64, dp, dp, dp, dp, C.c_int32, C.POINTER(dp), dp, u8p]
        L.lpo_outflow.restype = C.c_int
        L.lpo_outflow.argtypes = [cp, C.c_int64, C.POINTER(dp), C.c_int, C.POINTER(dp), C.c_uint32, C.c_uint32,
                                  C.POINTER(C.c_int64)]
        L.lpo_inflow_layer.restype = C.c_int
        L.lpo_inflow_layer.argtypes = [cp, C.c_int64, C.c_int64, C.POINTER(dp), C.POINTER(dp), dp, dp, dp, C.c_int,
                                       C.c_int, C.c_double, C.c_double, C.c_double, C.c_double, C.c_double,
                                       C.POINTER(C.c_int64)]
        L.lpo_reservoir_inflow.restype = C.c_int
        L.lpo_reservoir_inflow.argtypes = [cp, C.c_int64, C.POINTER(dp), dp, C.c_int, C.c_int, C.c_double,
                                           C.c_double, C.c_double, dp]
        L.lpo_timestep.restype = C.c_double
        L.lpo_timestep.argtypes = [cp, C.c_int64, dp, dp, dp]
        L.lpo_step_subset.restype = C.c_int
        L.lpo_step_subset.argtypes = [cp, C.c_int64, dp, dp, dp, dp, dp, dp, dp, dp, dp, C.c_double,
                                      C.c_int64, i64p, dp, dp, dp, dp, dp, dp, dp, dp, dp, u8p, dp, i64p, dp]
        L.lpo_mlp_forward.restype = None
        L.lpo_mlp_forward.argtypes = [dp, C.c_int64, dp, dp, dp]
        L.lpo_mlp_loss_grad.restype = C.c_double
        L.lpo_mlp_loss_grad.argtypes = [dp, C.c_int64, dp, dp, dp]
        L.lpo_step.restype = C.c_int
        L.lpo_step.argtypes = [cp, C.c_int64, dp, dp, dp, dp, dp, dp, dp, dp, dp, C.c_double, dp, u8p,
                               dp, i64p]
        L.lpo_conservation.restype = None
        L.lpo_conservation.argtypes = [cp, C.c_int64, dp, dp, dp, dp, dp, dp, dp]
        L.lpo_particle_derivs.restype = C.c_int
        L.lpo_particle_derivs.argtypes = [cp, C.c_int64, dp, dp, dp, dp, dp, dp, dp, dp, C.c_int64, ip,
                                          C.c_int32, C.c_double, C.c_double, dp, dp, dp, dp, ip, dp, ip]
        _lib = L
    return _lib


def _dp(a):
    if a is None:
        return None
    assert a.dtype == np.float64 and a.flags.c_contiguous
    return a.ctypes.data_as(C.POINTER(C.c_double))


def _ip(a):
    assert a.dtype == np.int32 and a.flags.c_contiguous
    return a.ctypes.data_as(C.POINTER(C.c_int32))


def make_cfg(cfg: dict) -> Cfg:
    """Build the oracle's config struct from a workload config dict."""
    c = Cfg()
    d = int(cfg["dim"])
    c.dim = d
    c.lw_cap = int(cfg.get("lw_cap", 0))
    c.uw_cap = int(cfg.get("uw_cap", 0))
    c.max_nb = int(cfg.get("max_nb", 128))
    c.gamma = float(cfg.get("gamma", 1.4))
    c.cfl = float(cfg.get("cfl", 0.5))
    c.kappa = float(cfg["kappa"])
    c.est_eps = float(cfg.get("est_eps", 1e-5))
    c.cond_max = float(cfg.get("cond_max", 1e12))
    c.uw_cond_max = float(cfg.get("uw_cond_max", 1e2))
    lo = list(cfg["box_lo"]) + [0.0] * (3 - d)
    hi = list(cfg["box_hi"]) + [1.0] * (3 - d)
    for a in range(3):
        c.lo[a] = float(lo[a])
        c.hi[a] = float(hi[a])
    per = cfg.get("periodic", [False] * d)
    wl = cfg.get("wall_lo", [False] * d)
    wh = cfg.get("wall_hi", [False] * d)
    for a in range(3):
        c.periodic[a] = int(bool(per[a])) if a < d else 0
        c.wall_lo[a] = int(bool(wl[a])) if a < d else 0
        c.wall_hi[a] = int(bool(wh[a])) if a < d else 0
    c.vacuum = int(bool(cfg.get("vacuum", False)))
    # blend with a fixed phi (1: pure Lax-Wendroff, 0: pure upwind); None: the estimator
    c.phi_fixed = -1.0 if cfg.get("phi_fixed") is None else float(cfg["phi_fixed"])
    # cap on the limiter's value (1: phi never exceeds pure Lax-Wendroff); 0: as printed (up to 1.25)
    c.limiter_cap = float(cfg.get("limiter_cap", 1.0))
    return c


def _xyz(x, d):
    x = np.ascontiguousarray(x, dtype=np.float64)
    cols = [np.ascontiguousarray(x[:, a]) for a in range(d)]
    return cols + [None] * (3 - d)


def set_num_threads(n: int) -> None:
    """OpenMP threads of later oracle calls (its results do not depend on the count)."""
    lib().lpo_set_num_threads(int(n))


def num_threads() -> int:
    return lib().lpo_num_threads()


def limiter(r: float) -> float:
    return lib().lpo_limiter(float(r))


def estimator_ratio(sl: float, sr: float) -> float:
    return lib().lpo_estimator_ratio(float(sl), float(sr))


def lstsq_qrp(A: np.ndarray, B: np.ndarray):
    """min ||A X - B|| by Householder QR with column pivoting; returns (X, cond)."""
    A = np.array(A, dtype=np.float64, order="C", copy=True)
    B = np.array(B, dtype=np.float64, order="C", copy=True)
    if B.ndim == 1:
        B = B[:, None].copy()
    k, n = A.shape
    X = np.zeros((n, B.shape[1]), dtype=np.float64)
    cond = lib().lpo_lstsq_qrp(k, n, B.shape[1], _dp(A), _dp(B), _dp(X))
    return X, cond


def lw_select(dim: int, dxs: np.ndarray, cap: int) -> np.ndarray:
    dxs3 = np.zeros((dxs.shape[0], 3))
    dxs3[:, :dim] = dxs[:, :dim]
    dxs3 = np.ascontiguousarray(dxs3)
    sel = np.zeros(max(1, dxs.shape[0]), dtype=np.intc)
    m = lib().lpo_lw_select(dim, dxs.shape[0], _dp(dxs3), cap, sel.ctypes.data_as(C.POINTER(C.c_int)))
    return sel[:m].copy()


def lw_rates(dim, gamma, dt, state, grad, hess):
    """state = [V, u.., P]; grad[f, a] (f x 3); hess[f, c] (f x 6, order 11,22,[33],12,[13,23])."""
    st = np.ascontiguousarray(state, dtype=np.float64)
    g = np.zeros((5, 3)); g[:grad.shape[0], :grad.shape[1]] = grad
    h = np.zeros((5, 6)); h[:hess.shape[0], :hess.shape[1]] = hess
    out = np.zeros(dim + 2)
    lib().lpo_lw_rates(dim, gamma, dt, _dp(st), _dp(np.ascontiguousarray(g)), _dp(np.ascontiguousarray(h)),
                       _dp(out))
    return out


def uw_rates(dim, gamma, state, dl, dr):
    """dl/dr[a, q]: one-sided derivative along axis a of q = (V, u_a, P)."""
    st = np.ascontiguousarray(state, dtype=np.float64)
    L = np.zeros((3, 3)); L[:dl.shape[0]] = dl
    R = np.zeros((3, 3)); R[:dr.shape[0]] = dr
    out = np.zeros(dim + 2)
    lib().lpo_uw_rates(dim, gamma, _dp(st), _dp(np.ascontiguousarray(L)), _dp(np.ascontiguousarray(R)),
                       _dp(out))
    return out


def neighbors(cfg: dict, x: np.ndarray, r: np.ndarray, max_nb: int = 128):
    """Neighbour lists: count[n], idx[n, max_nb] ordered by (d2, id); status."""
    c = make_cfg(cfg)
    d = c.dim
    n = x.shape[0]
    X = _xyz(x, d)
    r = np.ascontiguousarray(r, dtype=np.float64)
    count = np.zeros(n, dtype=np.int32)
    idx = np.full((n, max_nb), -1, dtype=np.int32)
    st = lib().lpo_neighbors(C.byref(c), n, _dp(X[0]), _dp(X[1]), _dp(X[2]), _dp(r), max_nb, _ip(count), _ip(idx))
    return count, idx, st


def neighbors_subset(cfg: dict, x: np.ndarray, r: np.ndarray, q: np.ndarray, max_nb: int = 128):
    """Neighbour lists of the particles q only (over all particles): count[nq], idx[nq, max_nb]; status."""
    c = make_cfg(cfg)
    d = c.dim
    X = _xyz(x, d)
    r = np.ascontiguousarray(r, dtype=np.float64)
    q = np.ascontiguousarray(q, dtype=np.int64)
    count = np.zeros(q.size, dtype=np.int32)
    idx = np.full((q.size, max_nb), -1, dtype=np.int32)
    st = lib().lpo_neighbors_subset(C.byref(c), x.shape[0], _dp(X[0]), _dp(X[1]), _dp(X[2]), _dp(r), max_nb,
                                    q.size, q.ctypes.data_as(C.POINTER(C.c_int64)), _ip(count), _ip(idx))
    return count, idx, st


def gfd(cfg: dict, x: np.ndarray, r: np.ndarray, fields):
    """Second-order GFD derivatives: deriv[f, c, i], status[i]."""
    c = make_cfg(cfg)
    d = c.dim
    n = x.shape[0]
    nu = 9 if d == 3 else 5
    X = _xyz(x, d)
    r = np.ascontiguousarray(r, dtype=np.float64)
    fs = [np.ascontiguousarray(f, dtype=np.float64) for f in fields]
    arr = (C.POINTER(C.c_double) * len(fs))(*[_dp(f) for f in fs])
    deriv = np.zeros((len(fs), nu, n))
    status = np.zeros(n, dtype=np.uint8)
    st = lib().lpo_gfd(C.byref(c), n, _dp(X[0]), _dp(X[1]), _dp(X[2]), _dp(r), len(fs), arr, _dp(deriv),
                       status.ctypes.data_as(C.POINTER(C.c_uint8)))
    return deriv, status, st


def gfd3(cfg: dict, x: np.ndarray, r: np.ndarray, fields):
    """Third-order GFD derivatives: deriv[f, c, i] (c over the 19 / 9 columns:
    x, y, z, xx, yy, zz, xy, xz, yz, xxx, yyy, zzz, xxy, xxz, xyy, yyz, xzz,
    yzz, xyz in 3D; x, y, xx, yy, xy, xxx, yyy, xxy, xyy in 2D), status[i]
    (0 cubic, 1 quadratic, 2 linear, 3 none)."""
    c = make_cfg(cfg)
    d = c.dim
    n = x.shape[0]
    nu = 19 if d == 3 else 9
    X = _xyz(x, d)
    r = np.ascontiguousarray(r, dtype=np.float64)
    fs = [np.ascontiguousarray(f, dtype=np.float64) for f in fields]
    arr = (C.POINTER(C.c_double) * len(fs))(*[_dp(f) for f in fs])
    deriv = np.zeros((len(fs), nu, n))
    status = np.zeros(n, dtype=np.uint8)
    st = lib().lpo_gfd3(C.byref(c), n, _dp(X[0]), _dp(X[1]), _dp(X[2]), _dp(r), len(fs), arr, _dp(deriv),
                        status.ctypes.data_as(C.POINTER(C.c_uint8)))
    return deriv, status, st


def outflow(cfg: dict, state: dict, lo_mask: int, hi_mask: int) -> dict:
    """Delete the particles past the outflow faces; returns the kept state
    (every per-particle array, order kept)."""
    c = make_cfg(cfg)
    d = c.dim
    n = state["V"].shape[0]
    cols = [np.ascontiguousarray(state["x"][:, a], dtype=np.float64).copy() for a in range(d)]
    cols += [np.ascontiguousarray(state["u"][:, a], dtype=np.float64).copy() for a in range(d)]
    cols += [np.ascontiguousarray(state[k], dtype=np.float64).copy() for k in ("V", "P", "m")]
    arr = (C.POINTER(C.c_double) * len(cols))(*[_dp(a) for a in cols])
    xs = (C.POINTER(C.c_double) * d)(*[_dp(cols[a]) for a in range(d)])
    kept = C.c_int64(0)
    st = lib().lpo_outflow(C.byref(c), n, arr, len(cols), xs, lo_mask, hi_mask, C.byref(kept))
    assert st == 0
    k = kept.value
    return {"x": np.stack([cols[a][:k] for a in range(d)], axis=1),
            "u": np.stack([cols[d + a][:k] for a in range(d)], axis=1),
            "V": cols[2 * d][:k], "P": cols[2 * d + 1][:k], "m": cols[2 * d + 2][:k]}


def reservoir_inflow(cfg: dict, state: dict, axis: int, side: int, width: float, p_res: float, rho_res: float):
    """(P_in, rho_in, u_in, particles averaged) of the reservoir inflow condition."""
    c = make_cfg(cfg)
    d = c.dim
    n = state["V"].shape[0]
    cols = [np.ascontiguousarray(state["x"][:, a], dtype=np.float64) for a in range(d)]
    xs = (C.POINTER(C.c_double) * d)(*[_dp(a) for a in cols])
    P = np.ascontiguousarray(state["P"], dtype=np.float64)
    out = np.zeros(4)
    st = lib().lpo_reservoir_inflow(C.byref(c), n, xs, _dp(P), axis, side, width, p_res, rho_res, _dp(out))
    return out, st


def inflow_layer(cfg: dict, n: int, cap: int, axis: int, side: int, spacing: float, depth: float, rho: float,
                 p_in: float, u_n: float):
    """The particles of the inflow layer (x, u, V, P, m of entries n .. n_new - 1)
    and the status."""
    c = make_cfg(cfg)
    d = c.dim
    xs = [np.zeros(cap) for _ in range(d)]
    us = [np.zeros(cap) for _ in range(d)]
    V, P, m = np.zeros(cap), np.zeros(cap), np.zeros(cap)
    xp = (C.POINTER(C.c_double) * d)(*[_dp(a) for a in xs])
    up = (C.POINTER(C.c_double) * d)(*[_dp(a) for a in us])
    nn = C.c_int64(0)
    st = lib().lpo_inflow_layer(C.byref(c), n, cap, xp, up, _dp(V), _dp(P), _dp(m), axis, side, spacing, depth, rho,
                                p_in, u_n, C.byref(nn))
    k = nn.value
    return {"x": np.stack([a[n:k] for a in xs], axis=1), "u": np.stack([a[n:k] for a in us], axis=1),
            "V": V[n:k], "P": P[n:k], "m": m[n:k]}, k, st


def timestep(cfg: dict, state: dict) -> float:
    c = make_cfg(cfg)
    V = np.ascontiguousarray(state["V"]); P = np.ascontiguousarray(state["P"]); m = np.ascontiguousarray(state["m"])
    return lib().lpo_timestep(C.byref(c), V.shape[0], _dp(V), _dp(P), _dp(m))


def _state_cols(state, d):
    X = _xyz(state["x"], d)
    U = _xyz(state["u"], d)
    V = np.ascontiguousarray(state["V"], dtype=np.float64)
    P = np.ascontiguousarray(state["P"], dtype=np.float64)
    m = np.ascontiguousarray(state["m"], dtype=np.float64)
    return X, U, V, P, m


def step(cfg: dict, state: dict, dt: float = 0.0):
    """One full time step; returns (new_state, info)."""
    c = make_cfg(cfg)
    d = c.dim
    X, U, V, P, m = _state_cols(state, d)
    X = [None if a is None else a.copy() for a in X]
    U = [None if a is None else a.copy() for a in U]
    V = V.copy(); P = P.copy()
    n = V.shape[0]
    phi = np.zeros(n)
    flags = np.zeros(n, dtype=np.uint8)
    dt_used = C.c_double(0.0)
    ng = C.c_int64(0)
    st = lib().lpo_step(C.byref(c), n, _dp(X[0]), _dp(X[1]), _dp(X[2]), _dp(V), _dp(U[0]), _dp(U[1]),
                        _dp(U[2]), _dp(P), _dp(m), float(dt), _dp(phi),
                        flags.ctypes.data_as(C.POINTER(C.c_uint8)), C.byref(dt_used), C.byref(ng))
    new = dict(state)
    new["x"] = np.stack([a for a in X if a is not None], axis=1)
    new["u"] = np.stack([a for a in U if a is not None], axis=1)
    new["V"] = V
    new["P"] = P
    return new, {"dt": dt_used.value, "phi": phi, "flags": flags, "n_ghost": ng.value, "status": st}


def step_subset(cfg: dict, state: dict, sub: np.ndarray, dt: float = 0.0, features: bool = False):
    """One time step evaluated only for the particles in ``sub`` (global dt, ghosts, neighbours).
    With features=True the result also holds the 16 estimator-network inputs
    of every particle of ``sub`` (key "feat", shape (len(sub), 16))."""
    c = make_cfg(cfg)
    d = c.dim
    X, U, V, P, m = _state_cols(state, d)
    n = V.shape[0]
    sub = np.ascontiguousarray(sub, dtype=np.int64)
    ns = sub.shape[0]
    o = [np.zeros(ns) for _ in range(8)]
    phi = np.zeros(ns)
    flags = np.zeros(ns, dtype=np.uint8)
    dt_used = C.c_double(0.0)
    ng = C.c_int64(0)
    feat = np.zeros((ns, 16)) if features else None
    st = lib().lpo_step_subset(C.byref(c), n, _dp(X[0]), _dp(X[1]), _dp(X[2]), _dp(V), _dp(U[0]), _dp(U[1]),
                               _dp(U[2]), _dp(P), _dp(m), float(dt), ns,
                               sub.ctypes.data_as(C.POINTER(C.c_int64)), *[_dp(a) for a in o], _dp(phi),
                               flags.ctypes.data_as(C.POINTER(C.c_uint8)), C.byref(dt_used), C.byref(ng),
                               _dp(feat) if features else None)
    out = {"x": np.stack(o[0:d], axis=1), "V": o[3], "u": np.stack(o[4:4 + d], axis=1), "P": o[7],
           "phi": phi, "flags": flags}
    if features:
        out["feat"] = feat
    return out, {"dt": dt_used.value, "n_ghost": ng.value, "status": st}


def conservation(cfg: dict, state: dict) -> np.ndarray:
    c = make_cfg(cfg)
    d = c.dim
    X, U, V, P, m = _state_cols(state, d)
    out = np.zeros(5)
    lib().lpo_conservation(C.byref(c), V.shape[0], _dp(V), _dp(U[0]), _dp(U[1]), _dp(U[2]), _dp(P), _dp(m),
                           _dp(out))
    return out


def particle_derivs(cfg: dict, state: dict, i: int, nb: np.ndarray, h: float, s: float):
    """LW gradient/Hessian, one-sided derivatives, validity and phi for particle i."""
    c = make_cfg(cfg)
    d = c.dim
    X, U, V, P, m = _state_cols(state, d)
    nb = np.ascontiguousarray(nb, dtype=np.int32)
    grad = np.zeros(15); hess = np.zeros(30); dl = np.zeros(9); dr = np.zeros(9)
    valid = np.zeros(6, dtype=np.int32)
    phi = C.c_double(0.0)
    flags = C.c_int32(0)
    lib().lpo_particle_derivs(C.byref(c), V.shape[0], _dp(X[0]), _dp(X[1]), _dp(X[2]), _dp(V), _dp(U[0]),
                              _dp(U[1]), _dp(U[2]), _dp(P), int(i), _ip(nb), nb.shape[0], float(h), float(s),
                              _dp(grad), _dp(hess), _dp(dl), _dp(dr), _ip(valid), C.byref(phi), C.byref(flags))
    return {"grad": grad.reshape(5, 3), "hess": hess.reshape(5, 6), "dl": dl.reshape(3, 3),
            "dr": dr.reshape(3, 3), "valid": valid.reshape(3, 2), "phi": phi.value, "flags": flags.value}


MLP_NPARAM = 5313


def mlp_forward(theta: np.ndarray, feat: np.ndarray):
    """Estimator network on feat (n x 16): returns (z, y = sigmoid(z))."""
    theta = np.ascontiguousarray(theta, dtype=np.float64)
    feat = np.ascontiguousarray(feat, dtype=np.float64)
    n = feat.shape[0]
    z = np.zeros(n)
    y = np.zeros(n)
    lib().lpo_mlp_forward(_dp(theta), n, _dp(feat), _dp(z), _dp(y))
    return z, y


def mlp_loss_grad(theta: np.ndarray, feat: np.ndarray, target: np.ndarray):
    """Mean binary cross-entropy of the network output against target, and its gradient."""
    theta = np.ascontiguousarray(theta, dtype=np.float64)
    feat = np.ascontiguousarray(feat, dtype=np.float64)
    target = np.ascontiguousarray(target, dtype=np.float64)
    grad = np.zeros(MLP_NPARAM)
    loss = lib().lpo_mlp_loss_grad(_dp(theta), feat.shape[0], _dp(feat), _dp(target), _dp(grad))
    return loss, grad
