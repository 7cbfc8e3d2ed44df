"""Pins of the oracle's estimator network and of its input features.

The network (16 -> 64 -> 64 -> 1, ReLU, sigmoid output, mean binary
cross-entropy) is not part of the paper; its oracle is pinned by closed forms
of hand-built networks and by central finite differences of the loss.  The
features are pinned on fields whose derivatives are known exactly and against
a brute-force reading of the half-ball membership."""
import numpy as np
import pytest

from paper_2206_11998_amd import workloads as W

N = 5313
OFF_W1, OFF_B1, OFF_W2, OFF_B2, OFF_W3, OFF_B3 = 0, 1024, 1088, 5184, 5248, 5312


def _sigmoid(z):
    return 1.0 / (1.0 + np.exp(-z))


def test_zero_network_outputs_sigmoid_of_bias(oracle_lib):
    th = np.zeros(N)
    th[OFF_B3] = 0.3
    feat = np.random.default_rng(0).standard_normal((7, 16))
    z, y = oracle_lib.mlp_forward(th, feat)
    assert np.all(z == 0.3) and np.allclose(y, _sigmoid(0.3), rtol=0, atol=1e-15)


def test_hand_built_network_closed_form(oracle_lib):
    # hidden unit 0 of layer 1 reads feature 3, unit 0 of layer 2 reads it
    th = np.zeros(N)
    th[OFF_W1 + 0 * 16 + 3] = 2.0
    th[OFF_B1 + 0] = -0.5
    th[OFF_W2 + 0 * 64 + 0] = 1.5
    th[OFF_B2 + 0] = 0.1
    th[OFF_W3 + 0] = 0.7
    th[OFF_B3] = -0.2
    # a unit that never activates (negative bias, no inputs) must not matter
    th[OFF_B1 + 5] = -1.0
    th[OFF_W2 + 0 * 64 + 5] = 9.0
    feat = np.zeros((5, 16))
    feat[:, 3] = [-1.0, 0.0, 0.2, 0.3, 1.7]
    feat[:, 7] = 5.0  # ignored input
    z, y = oracle_lib.mlp_forward(th, feat)
    h1 = np.maximum(2.0 * feat[:, 3] - 0.5, 0.0)
    h2 = np.maximum(1.5 * h1 + 0.1, 0.0)
    ref = -0.2 + 0.7 * h2
    assert np.allclose(z, ref, rtol=0, atol=1e-15)
    assert np.allclose(y, _sigmoid(ref), rtol=0, atol=1e-15)


def test_loss_gradient_matches_finite_differences(oracle_lib):
    rng = np.random.default_rng(3)
    th = rng.standard_normal(N) * 0.3
    feat = rng.standard_normal((40, 16))
    target = rng.uniform(0.0, 1.0, 40)
    loss, grad = oracle_lib.mlp_loss_grad(th, feat, target)
    # the loss is the mean cross-entropy of the forward pass
    z, y = oracle_lib.mlp_forward(th, feat)
    ref = np.mean(-(target * np.log(y) + (1 - target) * np.log(1 - y)))
    assert abs(loss - ref) <= 1e-12 * abs(ref)
    # every block of parameters, a sample from each
    idx = np.concatenate([rng.choice(np.arange(a, b), size=min(40, b - a), replace=False)
                          for a, b in ((OFF_W1, OFF_B1), (OFF_B1, OFF_W2), (OFF_W2, OFF_B2), (OFF_B2, OFF_W3),
                                       (OFF_W3, OFF_B3), (OFF_B3, N))])
    eps = 1e-6
    for q in idx:
        tp = th.copy(); tp[q] += eps
        tm = th.copy(); tm[q] -= eps
        fd = (oracle_lib.mlp_loss_grad(tp, feat, target)[0] - oracle_lib.mlp_loss_grad(tm, feat, target)[0]) / (2 * eps)
        assert abs(fd - grad[q]) <= 1e-6 * max(abs(grad[q]), 1e-4), (q, fd, grad[q])


def _linear_state(n=9, seed=4):
    cfg, st = W.uniform_box(3, n, seed=seed, periodic=False)
    x = st["x"]
    st = dict(st)
    st["V"] = 1.0 + 0.1 * x[:, 0] + 0.05 * x[:, 1]
    st["P"] = 2.0 + 0.2 * x[:, 2]
    st["u"] = np.stack([0.1 * x[:, 0] + 0.3, 0.2 * x[:, 1] - 0.02 * x[:, 0], -0.05 * x[:, 2]], axis=1)
    st["m"] = st["m"] * 0 + (1.0 / n) ** 3 / st["V"]  # h = (m V)^(1/3) = 1/n for every particle
    return cfg, st


def test_features_of_linear_fields(oracle_lib):
    cfg, st = _linear_state()
    n = st["V"].shape[0]
    out, info = oracle_lib.step_subset(cfg, st, np.arange(n), dt=1e-6, features=True)
    assert info["status"] == 0
    f = out["feat"]
    h = (st["m"] * st["V"]) ** (1 / 3)
    V, P = st["V"], st["P"]
    c = np.sqrt(cfg["gamma"] * P * V)
    deg = (out["flags"] & 2) != 0
    ok = ~deg
    assert ok.sum() > 0.8 * n
    gV = np.array([0.1, 0.05, 0.0])
    gP = np.array([0.0, 0.0, 0.2])
    for a in range(3):
        assert np.allclose(f[ok, a], -h[ok] * gV[a] / V[ok], rtol=1e-9, atol=1e-12)
        assert np.allclose(f[ok, 3 + a], h[ok] * gP[a] / P[ok], rtol=1e-9, atol=1e-12)
    J = np.array([[0.1, 0.0, 0.0], [-0.02, 0.2, 0.0], [0.0, 0.0, -0.05]])
    assert np.allclose(f[ok, 6], h[ok] * np.trace(J) / c[ok], rtol=1e-9, atol=1e-12)
    assert np.allclose(f[ok, 15], h[ok] * np.sqrt((J * J).sum()) / c[ok], rtol=1e-9, atol=1e-12)
    # equal one-sided slopes of a linear field: no disagreement
    assert np.abs(f[ok, 7:13]).max() <= 1e-8


def test_stencil_extrema_features_brute_force(oracle_lib):
    cfg, st = _linear_state(n=7, seed=5)
    n = st["V"].shape[0]
    out, _ = oracle_lib.step_subset(cfg, st, np.arange(n), dt=1e-6, features=True)
    x = st["x"]
    r = cfg["kappa"] * (st["m"] * st["V"]) ** (1 / 3)
    count, idx, rs = oracle_lib.neighbors(cfg, x, r, max_nb=256)
    assert rs == 0
    for i in range(0, n, 17):
        nb = idx[i, :count[i]]  # (d2, id) order
        members = set()
        for a in range(3):
            d = x[nb, a] - x[i, a]
            members.update(nb[d > 0][:8].tolist())
            members.update(nb[d < 0][:8].tolist())
        sel = np.array(sorted(members | {i}))
        assert np.isclose(out["feat"][i, 13], np.log(st["V"][sel].max() / st["V"][sel].min()), rtol=1e-13, atol=1e-15)
        assert np.isclose(out["feat"][i, 14], np.log(st["P"][sel].max() / st["P"][sel].min()), rtol=1e-13, atol=1e-15)


def test_features_of_constant_state_vanish(oracle_lib):
    cfg, st = W.uniform_box(3, 8, u0=[0.2, 0.0, -0.1], p=1.3, rho=0.9)
    n = st["V"].shape[0]
    out, _ = oracle_lib.step_subset(cfg, st, np.arange(n), features=True)
    assert np.all(out["feat"] == 0.0)


def test_accuracy_phi_is_the_least_squares_blend():
    """The accuracy label of the network's training (tests/gpu_util.py): on
    random upwind / Lax-Wendroff / exact states it must equal a brute-force
    minimisation over a fine phi grid of the scaled squared error, clip at 0
    and 1, and be NaN where both results coincide."""
    from tests.gpu_util import accuracy_phi
    rng = np.random.default_rng(11)
    n, D = 200, 3
    s0 = {"V": rng.random(n) + 0.5, "u": rng.normal(size=(n, D)), "P": rng.random(n) + 0.5}
    s1 = {"V": s0["V"] + 0.1 * rng.normal(size=n), "u": s0["u"] + 0.1 * rng.normal(size=(n, D)),
          "P": s0["P"] + 0.1 * rng.normal(size=n)}
    s1["V"][:3], s1["u"][:3], s1["P"][:3] = s0["V"][:3], s0["u"][:3], s0["P"][:3]   # phi irrelevant
    ex = {"V": s0["V"] + 0.08 * rng.normal(size=n), "u": s0["u"] + 0.08 * rng.normal(size=(n, D)),
          "P": s0["P"] + 0.08 * rng.normal(size=n)}
    sc = (0.9, 1.7, 1.3)
    phi, den = accuracy_phi(s0, s1, ex["V"], ex["u"], ex["P"], *sc)
    assert np.all(np.isnan(phi[:3])) and np.all(den[:3] == 0.0)
    grid = np.linspace(0.0, 1.0, 20001)
    for i in range(3, n):
        err = ((s0["V"][i] - grid * (s0["V"][i] - s1["V"][i]) - ex["V"][i]) / sc[0]) ** 2
        for q in range(D):
            err += ((s0["u"][i, q] - grid * (s0["u"][i, q] - s1["u"][i, q]) - ex["u"][i, q]) / sc[1]) ** 2
        err += ((s0["P"][i] - grid * (s0["P"][i] - s1["P"][i]) - ex["P"][i]) / sc[2]) ** 2
        assert abs(phi[i] - grid[np.argmin(err)]) <= 1e-4
    assert np.any(phi[3:] == 0.0) and np.any(phi[3:] == 1.0) and np.any((phi > 0) & (phi < 1))
