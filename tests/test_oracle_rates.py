"""Pins P5-P7 for the time-derivative formulas (Sec. 2.1).

* The printed characteristic matrices are checked against each other and the
  printed upwind equations are re-derived from them.
* The multi-dimensional Lax-Wendroff second derivatives are checked against
  exact solutions of the Euler equations (a rotating isentropic vortex placed
  at an arbitrary 3D orientation, and a homologous expansion), and reduce to
  the printed 1D second-derivative equations.
"""
import json
import math
import os

import numpy as np
import pytest
import sympy as sp

GOLD = os.path.join(os.path.dirname(__file__), "golden")
GAMMA = 1.4


def _golden(name):
    with open(os.path.join(GOLD, name)) as f:
        return json.load(f)


def _ideal_gas_K():
    V, P, g = sp.symbols("V P gamma", positive=True)
    e = P * V / (g - 1)
    return sp.simplify((P + sp.diff(e, V)) / sp.diff(e, P)), (V, P, g)


def test_ideal_gas_K():
    K, (V, P, g) = _ideal_gas_K()
    assert sp.simplify(K - g * P / V) == 0
    # V sqrt(K) is the sound speed sqrt(gamma P V)
    assert sp.simplify(V * sp.sqrt(K) - sp.sqrt(g * P * V)) == 0


def _mat(rows, K, V):
    return sp.Matrix([[sp.sympify(e, locals={"K": K, "V": V}) for e in row] for row in rows])


def test_characteristic_matrices():
    gold = _golden("characteristics.json")
    K, V = sp.symbols("K V", positive=True)
    A = V * _mat(gold["A_over_V"], K, V)
    R = _mat(gold["R"], K, V)
    Ri = _mat(gold["Rinv"], K, V)
    Lam = V * _mat(gold["Lambda_over_V"], K, V)
    assert sp.simplify(R * Ri - sp.eye(3)) == sp.zeros(3)
    assert sp.simplify(R * Lam * Ri - A) == sp.zeros(3)


def test_upwind_from_characteristics(oracle_lib):
    """Upwinding each characteristic field (+V sqrt(K) wave from the left, -V sqrt(K)
    wave from the right) reproduces the printed rates and the oracle's 1D rates."""
    gold = _golden("characteristics.json")
    Ks, Vs = sp.symbols("K V", positive=True)
    R = _mat(gold["R"], Ks, Vs)
    Ri = _mat(gold["Rinv"], Ks, Vs)
    Lam = Vs * _mat(gold["Lambda_over_V"], Ks, Vs)
    rng = np.random.default_rng(0)
    for _ in range(20):
        V, P = rng.uniform(0.5, 3.0), rng.uniform(0.2, 4.0)
        K = GAMMA * P / V
        Ul = rng.standard_normal(3)  # left derivatives of (V, u, P)
        Ur = rng.standard_normal(3)
        sub = {Ks: K, Vs: V}
        Rn = np.array(R.subs(sub), dtype=float)
        Rin = np.array(Ri.subs(sub), dtype=float)
        lam = np.diag(np.array(Lam.subs(sub), dtype=float))
        wl, wr = Rin @ Ul, Rin @ Ur
        wt = np.where(lam > 0, -lam * wl, np.where(lam < 0, -lam * wr, 0.0))
        Ut = Rn @ wt
        loc = {"V": V, "K": K, "uxl": Ul[1], "uxr": Ur[1], "Pxl": Ul[2], "Pxr": Ur[2], "sqrt": math.sqrt}
        printed = [eval(gold["upwind_rates"][q], {}, loc) for q in ("V", "u", "P")]
        assert np.allclose(Ut, printed, rtol=1e-12, atol=1e-12)
        # oracle, 3D embedding with variation along x only
        dl = np.zeros((3, 3)); dr = np.zeros((3, 3))
        dl[0] = [Ul[0], Ul[1], Ul[2]]
        dr[0] = [Ur[0], Ur[1], Ur[2]]
        out = oracle_lib.uw_rates(3, GAMMA, np.array([V, 0.1, 0.2, 0.3, P]), dl, dr)
        assert np.allclose(out[[0, 1, 4]], Ut, rtol=1e-12, atol=1e-12)
        assert out[2] == 0.0 and out[3] == 0.0


def test_upwind_sums_over_axes(oracle_lib):
    rng = np.random.default_rng(1)
    st = np.array([1.3, 0.1, -0.2, 0.3, 2.0])
    dl = rng.standard_normal((3, 3)); dr = rng.standard_normal((3, 3))
    tot = oracle_lib.uw_rates(3, GAMMA, st, dl, dr)
    part = np.zeros(5)
    for a in range(3):
        L = np.zeros((3, 3)); Rr = np.zeros((3, 3))
        L[a] = dl[a]; Rr[a] = dr[a]
        part += oracle_lib.uw_rates(3, GAMMA, st, L, Rr)
    assert np.allclose(tot, part, rtol=1e-13, atol=1e-13)


@pytest.mark.parametrize("dim", [2, 3])
def test_smooth_limit_consistency(oracle_lib, dim):
    """Pin P7: equal one-sided derivatives make the upwind rate the first-order LW rate."""
    rng = np.random.default_rng(2)
    for _ in range(10):
        st = np.concatenate([[rng.uniform(0.5, 2)], rng.standard_normal(dim), [rng.uniform(0.5, 2)]])
        grad = rng.standard_normal((dim + 2, 3))
        grad[:, dim:] = 0.0
        hess = rng.standard_normal((dim + 2, 6))
        lw0 = oracle_lib.lw_rates(dim, GAMMA, 0.0, st, grad, hess)
        d = np.zeros((3, 3))
        for a in range(dim):
            d[a] = [grad[0, a], grad[1 + a, a], grad[dim + 1, a]]
        uw = oracle_lib.uw_rates(dim, GAMMA, st, d, d)
        assert np.allclose(uw, lw0, rtol=1e-12, atol=1e-12)


def _derivs_from_fields(V, u, P, X, pt):
    """Gradients and Hessians (oracle layout) of sympy fields at a point."""
    dim = len(X)
    fields = [V] + list(u) + [P]
    sub = dict(zip(X, pt))
    grad = np.zeros((dim + 2, 3))
    hess = np.zeros((dim + 2, 6))
    pairs = [(0, 1)] if dim == 2 else [(0, 1), (0, 2), (1, 2)]
    for f, F in enumerate(fields):
        for a in range(dim):
            grad[f, a] = float(sp.diff(F, X[a]).evalf(subs=sub))
            hess[f, a] = float(sp.diff(F, X[a], 2).evalf(subs=sub))
        for q, (a, b) in enumerate(pairs):
            hess[f, dim + q] = float(sp.diff(F, X[a], X[b]).evalf(subs=sub))
    st = np.array([float(F.evalf(subs=sub)) for F in fields])
    return st, grad, hess


def _vortex(beta=5.0, g=GAMMA):
    xi, eta = sp.symbols("xi eta", real=True)
    r2 = xi ** 2 + eta ** 2
    f = sp.exp((1 - r2) / 2)
    uu = -beta / (2 * sp.pi) * f * eta
    vv = beta / (2 * sp.pi) * f * xi
    T = 1 - (g - 1) * beta ** 2 / (8 * g * sp.pi ** 2) * sp.exp(1 - r2)
    rho = T ** (1 / (g - 1))
    return xi, eta, uu, vv, 1 / rho, rho ** g


def test_vortex_is_exact_steady_solution():
    xi, eta, uu, vv, V, P = _vortex()
    rho = 1 / V
    mom_x = rho * (uu * sp.diff(uu, xi) + vv * sp.diff(uu, eta)) + sp.diff(P, xi)
    mom_y = rho * (uu * sp.diff(vv, xi) + vv * sp.diff(vv, eta)) + sp.diff(P, eta)
    for pt in [(0.3, -0.7), (1.1, 0.4), (-0.2, 1.5)]:
        s = {xi: pt[0], eta: pt[1]}
        assert abs(float(mom_x.evalf(subs=s))) < 1e-12
        assert abs(float(mom_y.evalf(subs=s))) < 1e-12
    assert sp.simplify(sp.diff(uu, xi) + sp.diff(vv, eta)) == 0


@pytest.mark.parametrize("dim", [2, 3])
def test_lw_rates_on_rotating_vortex(oracle_lib, dim):
    """Steady flow: material derivatives are s_t = u.grad s and s_tt = u.grad(u.grad s)."""
    xi, eta, uu, vv, V2, P2 = _vortex()
    rng = np.random.default_rng(3)
    if dim == 2:
        X = sp.symbols("x y", real=True)
        Q = np.array([[0.6, -0.8], [0.8, 0.6]])
        loc = sp.Matrix(Q.T) * sp.Matrix(X)
        sub = {xi: loc[0], eta: loc[1]}
        vel = sp.Matrix(Q) * sp.Matrix([uu.subs(sub, simultaneous=True), vv.subs(sub, simultaneous=True)])
    else:
        X = sp.symbols("x y z", real=True)
        Q, _ = np.linalg.qr(rng.standard_normal((3, 3)))
        loc = sp.Matrix(Q.T) * sp.Matrix(X)
        sub = {xi: loc[0], eta: loc[1]}
        vel = sp.Matrix(Q) * sp.Matrix([uu.subs(sub, simultaneous=True), vv.subs(sub, simultaneous=True), 0])
    V = V2.subs(sub, simultaneous=True)
    P = P2.subs(sub, simultaneous=True)
    u = list(vel)
    mat = lambda F: sum(u[a] * sp.diff(F, X[a]) for a in range(dim))
    fields = [V] + u + [P]
    for _ in range(3):
        pt = rng.uniform(-1.2, 1.2, size=dim)
        s = dict(zip(X, pt))
        st, grad, hess = _derivs_from_fields(V, u, P, X, pt)
        st_t = np.array([float(mat(F).evalf(subs=s)) for F in fields])
        st_tt = np.array([float(mat(mat(F)).evalf(subs=s)) for F in fields])
        r0 = oracle_lib.lw_rates(dim, GAMMA, 0.0, st, grad, hess)
        r2 = oracle_lib.lw_rates(dim, GAMMA, 2.0, st, grad, hess)
        scale = np.abs(st_tt).max() + np.abs(st_t).max()
        assert np.allclose(r0, st_t, rtol=0, atol=1e-11 * scale)
        assert np.allclose(r2 - r0, st_tt, rtol=0, atol=1e-10 * scale)


def test_lw_rates_on_homologous_expansion(oracle_lib):
    """u = x/(1+t), uniform V = V0 (1+t)^3, P = P0 (1+t)^(-3 gamma): an exact solution."""
    V0, P0 = 1.7, 0.9
    st = np.array([V0, 0.2, -0.4, 0.1, P0])
    grad = np.zeros((5, 3))
    for a in range(3):
        grad[1 + a, a] = 1.0
    hess = np.zeros((5, 6))
    r0 = oracle_lib.lw_rates(3, GAMMA, 0.0, st, grad, hess)
    r2 = oracle_lib.lw_rates(3, GAMMA, 2.0, st, grad, hess)
    g = GAMMA
    assert np.allclose(r0, [3 * V0, 0, 0, 0, -3 * g * P0], rtol=1e-14, atol=1e-14)
    assert np.allclose(r2 - r0, [6 * V0, 0, 0, 0, 3 * g * (3 * g + 1) * P0], rtol=1e-14, atol=1e-14)


@pytest.mark.parametrize("dim", [2, 3])
def test_lw_reduces_to_printed_1d(oracle_lib, dim):
    """Pin P6: fields varying along x only give the printed 1D second derivatives."""
    gold = _golden("lw_1d.json")
    rng = np.random.default_rng(4)
    for _ in range(20):
        V, P, u = rng.uniform(0.5, 2), rng.uniform(0.5, 2), rng.standard_normal()
        Vx, ux, Px, Pxx, uxx = rng.standard_normal(5)
        st = np.zeros(dim + 2); st[0] = V; st[1] = u; st[-1] = P
        grad = np.zeros((dim + 2, 3)); hess = np.zeros((dim + 2, 6))
        grad[0, 0] = Vx; grad[1, 0] = ux; grad[dim + 1, 0] = Px
        hess[1, 0] = uxx; hess[dim + 1, 0] = Pxx
        hess[0, 0] = rng.standard_normal()  # V_xx does not enter
        loc = dict(V=V, P=P, Vx=Vx, ux=ux, Px=Px, Pxx=Pxx, uxx=uxx, gamma=GAMMA)
        want = np.array([eval(gold[q], {}, loc) for q in ("Vtt", "utt", "Ptt")])
        r0 = oracle_lib.lw_rates(dim, GAMMA, 0.0, st, grad, hess)
        r2 = oracle_lib.lw_rates(dim, GAMMA, 2.0, st, grad, hess)
        tt = r2 - r0
        assert np.allclose(tt[[0, 1, dim + 1]], want, rtol=1e-12, atol=1e-12)
        assert np.allclose(r0[[0, 1, dim + 1]], [V * ux, -V * Px, -GAMMA * P * ux], rtol=1e-13, atol=1e-13)
