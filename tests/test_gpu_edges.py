"""Edge cases on the GPU against the oracle.

- Sets of one to a hundred particles: the method's degenerate cases. With
  fewer than D neighbours the second-order fit is empty, half-balls stay
  incomplete, and vacuum ghosts have no mirror members.
- Isolated particles next to a dense cluster.
- A particle count that fills no launch evenly.
- An empty set, which the library rejects."""
import numpy as np
import pytest

from paper_2206_11998_amd import workloads as W
from tests.gpu_util import compare_states, say

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def lp():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2206_11998_amd import lp as _lp
    _lp.lib()
    return _lp


def _scattered(n, dim, seed, spread, h):
    """n particles uniform in a cube of side `spread` at the box centre, with
    smoothing length about h (m = rho h^dim)."""
    rng = np.random.default_rng(seed)
    x = 0.5 + spread * (rng.random((n, dim)) - 0.5)
    rho = 1.0 + 0.02 * rng.random(n)
    p = 1.0 + 0.02 * rng.random(n)
    u = 0.01 * rng.standard_normal((n, dim))
    m = rho * h ** dim
    return W._state(x, rho, u, p, m)


def _run_pair(lp, oracle_lib, cfg, st, nsteps, precision, tol, tag):
    say("edge case", tag, precision, st["V"].shape[0], "particles", nsteps, "steps")
    ctx = lp.Context(cfg, precision=precision)
    dev = lp.state_to_device(st)
    ref = st
    for _ in range(nsteps):
        d = oracle_lib.timestep(cfg, ref)
        ctx.step(dev, d)
        assert ctx.check() == lp.OK, lp.lib().lp_last_error(ctx._h)
        ref, info = oracle_lib.step(cfg, ref, d)
        assert info["status"] == 0
    got = lp.state_to_host(dev)
    compare_states(got, ref, cfg, tol, tag)
    if precision == "fp64":
        assert np.array_equal(got["flags"] & 15, info["flags"] & 15), tag
    ctx.close()
    return got, info


# (particles, smoothing length, free boundary): from every fit degenerate,
# through a mix, to complete stencils with vacuum ghosts.  Small vacuum clouds
# of scattered particles can drive V or P negative within two steps, in the
# oracle as on the GPU; these settings stay clear of that.
TINY = [(1, 0.05, True), (2, 0.05, True), (3, 0.05, True), (5, 0.05, True), (17, 0.058, False),
        (100, 0.032, False), (100, 0.065, True)]


@pytest.mark.parametrize("n,h,vacuum", TINY)
@pytest.mark.parametrize("precision,tol", [("fp64", 1e-10), ("mixed", 1e-4)])
def test_tiny_free_cloud(lp, oracle_lib, n, h, vacuum, precision, tol):
    """A few particles in an open box: many have fewer neighbours than the
    fit has unknowns."""
    cfg = W.base_config("tiny", 3, 2.2, [0.0] * 3, [1.0] * 3, [False] * 3, vacuum=vacuum, cfl=0.2)
    cfg["max_nb"] = 128
    st = _scattered(n, 3, seed=n, spread=0.2, h=h)
    got, info = _run_pair(lp, oracle_lib, cfg, st, 2, precision, tol, "free cloud n=%d h=%g" % (n, h))
    if n <= 5:
        assert np.all(info["flags"] & 2), "every fit is degenerate"


@pytest.mark.parametrize("n", [1, 4, 12])
def test_tiny_periodic_2d(lp, oracle_lib, n):
    cfg = W.base_config("tiny2d", 2, 2.5, [0.0, 0.0], [1.0, 1.0], [True, True])
    cfg["max_nb"] = 64
    st = _scattered(n, 2, seed=10 + n, spread=1.0, h=0.04)
    _run_pair(lp, oracle_lib, cfg, st, 2, "fp64", 1e-10, "periodic 2D n=%d" % n)


@pytest.mark.parametrize("n", [1, 6, 40])
def test_tiny_between_walls(lp, oracle_lib, n):
    """Mirror walls on x: particles near a wall get ghosts, isolated or not."""
    cfg = W.base_config("walls", 3, 2.1, [0.0] * 3, [1.0] * 3, [False, True, True],
                        wall_lo=[True, False, False], wall_hi=[True, False, False], cfl=0.2)
    cfg["max_nb"] = 128
    st = _scattered(n, 3, seed=20 + n, spread=1.0, h=0.06)
    got, info = _run_pair(lp, oracle_lib, cfg, st, 2, "fp64", 1e-10, "walls n=%d" % n)


def test_isolated_particles_beside_a_cluster(lp, oracle_lib):
    cfg, st = W.uniform_box(3, 10, seed=3, periodic=False)
    cfg = dict(cfg, box_lo=[-1.0] * 3, box_hi=[2.0] * 3, cfl=0.2)
    h = 0.1
    far = np.array([[-0.8, -0.8, -0.8], [1.8, 0.5, 0.5], [0.5, 1.9, -0.9], [1.7, 1.7, 1.7]])
    x = np.concatenate([st["x"], far])
    k = far.shape[0]
    st2 = {"x": x, "u": np.concatenate([st["u"], np.zeros((k, 3))]),
           "V": np.concatenate([st["V"], np.ones(k)]), "P": np.concatenate([st["P"], np.ones(k)]),
           "m": np.concatenate([st["m"], np.full(k, h ** 3)])}
    got, info = _run_pair(lp, oracle_lib, cfg, st2, 2, "fp64", 1e-10, "cluster + isolated")
    assert np.all(info["flags"][-k:] & 2)  # the isolated ones


@pytest.mark.parametrize("precision,tol", [("fp64", 1e-10), ("mixed", 1e-4)])
def test_ragged_count(lp, oracle_lib, precision, tol):
    """13^3 = 2197 particles: no launch of 64 or 256 lanes is filled evenly."""
    cfg, st = W.uniform_box(3, 13, seed=6)
    rng = np.random.default_rng(1)
    st = dict(st)
    st["P"] = st["P"] * (1.0 + 0.05 * rng.standard_normal(st["P"].shape))
    _run_pair(lp, oracle_lib, cfg, st, 3, precision, tol, "13^3 lattice")


def test_empty_set_rejected(lp):
    cfg, st = W.uniform_box(3, 4)
    empty = {k: v[:0] for k, v in st.items()}
    ctx = lp.Context(cfg)
    dev = lp.state_to_device(empty)
    with pytest.raises(lp.LpError) as e:
        ctx.step(dev)
    assert e.value.status == lp.E_ARG
    ctx.close()
