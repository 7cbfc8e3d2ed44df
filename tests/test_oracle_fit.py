"""Pins P2-P4 for the GFD least-squares fits (Sec. 2.1, Taylor expansion,
system A x = b, 'QR decomposition with column pivoting')."""
import numpy as np
import pytest

from paper_2206_11998_amd import workloads as W


def test_qrp_matches_lapack(oracle_lib):
    rng = np.random.default_rng(0)
    for trial in range(400):
        n = int(rng.choice([2, 3, 5, 9]))
        k = int(rng.integers(n, 60))
        A = rng.standard_normal((k, n))
        B = rng.standard_normal((k, 5))
        X, cond = oracle_lib.lstsq_qrp(A, B)
        Xr = np.linalg.lstsq(A, B, rcond=None)[0]
        assert np.max(np.abs(X - Xr)) <= 1e-12 * max(1.0, np.max(np.abs(Xr))), trial
        s = np.linalg.svd(A, compute_uv=False)
        # pivoted |R11|/|Rnn| never exceeds the 2-norm condition number
        assert cond <= s[0] / s[-1] * (1 + 1e-10)


def test_qrp_rank_deficient(oracle_lib):
    rng = np.random.default_rng(1)
    A = rng.standard_normal((20, 5))
    A[:, 3] = 2.0 * A[:, 1] - A[:, 0]
    X, cond = oracle_lib.lstsq_qrp(A, rng.standard_normal(20))
    assert cond > 1e12


def test_qrp_pivot_order(oracle_lib):
    # a dominant column is taken first: |R11| equals its norm
    rng = np.random.default_rng(2)
    A = rng.standard_normal((12, 4))
    A[:, 2] *= 100.0
    A[:, 1] *= 1e-3
    X, cond = oracle_lib.lstsq_qrp(A, rng.standard_normal(12))
    s = np.linalg.norm(A, axis=0)
    assert cond > s[2] / s[1] / 50


def _quadratic(dim, rng):
    c0 = rng.standard_normal()
    g = rng.standard_normal(dim)
    H = rng.standard_normal((dim, dim))
    H = 0.5 * (H + H.T)
    return c0, g, H


@pytest.mark.parametrize("dim", [2, 3])
def test_quadratic_reproduction(oracle_lib, dim):
    """Second-order GFD is exact for quadratic fields on scattered points."""
    rng = np.random.default_rng(3 + dim)
    n = 12 if dim == 3 else 30
    cfg, st = W.uniform_box(dim, n, seed=9, periodic=False)
    x = st["x"]
    h = (st["m"] * st["V"]) ** (1.0 / dim)
    r = cfg["kappa"] * h
    fields, want = [], []
    for f in range(3):
        c0, g, H = _quadratic(dim, rng)
        fields.append(c0 + x @ g + 0.5 * np.einsum("ia,ab,ib->i", x, H, x))
        grad = g[None, :] + x @ H
        cols = [grad[:, a] for a in range(dim)] + [np.full(len(x), H[a, a]) for a in range(dim)]
        pairs = [(0, 1)] if dim == 2 else [(0, 1), (0, 2), (1, 2)]
        cols += [np.full(len(x), H[a, b]) for a, b in pairs]
        want.append(np.stack(cols))
    deriv, status, stt = oracle_lib.gfd(cfg, x, r, fields)
    assert stt == 0 and np.all(status == 0)
    for f in range(3):
        err = np.abs(deriv[f] - want[f]).max()
        assert err <= 1e-9 * np.abs(want[f]).max(), err


@pytest.mark.parametrize("dim", [2, 3])
def test_one_sided_linear_reproduction(oracle_lib, dim):
    """Pin P4: the half-ball (upwind) fits reproduce linear fields exactly."""
    rng = np.random.default_rng(7)
    cfg, st = W.uniform_box(dim, 10 if dim == 3 else 24, seed=4)
    x = st["x"]
    g = rng.standard_normal((dim + 2, dim))
    st = dict(st)
    st["V"] = 2.0 + x @ g[0] * 0.1
    st["u"] = np.stack([0.3 + x @ g[1 + a] * 0.1 for a in range(dim)], axis=1)
    st["P"] = 3.0 + x @ g[dim + 1] * 0.1
    cfg = dict(cfg, periodic=[False] * dim, box_lo=[-5.0] * dim, box_hi=[5.0] * dim)
    h = (st["m"] * 1.0) ** (1.0 / dim)
    r = cfg["kappa"] * h
    count, idx, _ = oracle_lib.neighbors(cfg, x, r)
    centre = np.all(np.abs(x - 0.5) < 0.2, axis=1)
    for i in np.nonzero(centre)[0][:20]:
        res = oracle_lib.particle_derivs(cfg, st, i, idx[i, :count[i]], h[i], r[i])
        assert np.all(res["valid"][:dim] == 1)
        for a in range(dim):
            exp = np.array([g[0, a], g[1 + a, a], g[dim + 1, a]]) * 0.1
            assert np.allclose(res["dl"][a], exp, rtol=0, atol=1e-12)
            assert np.allclose(res["dr"][a], exp, rtol=0, atol=1e-12)


def test_lw_octant_selection(oracle_lib):
    """Sec. 2.2 step 4: when the stencil is capped, its top members come from all directions."""
    rng = np.random.default_rng(5)
    dxs = rng.standard_normal((70, 3))
    d2 = (dxs ** 2).sum(1)
    dxs = dxs[np.argsort(d2)]
    sel = oracle_lib.lw_select(3, dxs, 24)
    assert len(sel) == 24
    oct_ = ((dxs[:, 0] >= 0) * 1 + (dxs[:, 1] >= 0) * 2 + (dxs[:, 2] >= 0) * 4)
    counts = np.bincount(oct_[sel], minlength=8)
    avail = np.bincount(oct_, minlength=8)
    # every octant contributes min(available, 3) members: 24 = 8 x 3
    assert np.array_equal(counts, np.minimum(avail, 3))
    # within an octant the nearest ones are taken
    for o in range(8):
        members = np.nonzero(oct_ == o)[0]
        assert set(sel[oct_[sel] == o]) == set(members[:counts[o]])
    # uncapped: identity
    assert np.array_equal(oracle_lib.lw_select(3, dxs[:20], 54), np.arange(20))
