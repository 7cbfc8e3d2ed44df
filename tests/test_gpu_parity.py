"""GPU (liblp, through the C ABI) vs the FP64 oracle.

Neighbour lists bit-exact; GFD derivatives and full steps within the stated
relative L1 tolerances: 1e-10 (FP64 path), 1e-4 (mixed path)."""
import numpy as np
import pytest

from paper_2206_11998_amd import workloads as W
from tests.gpu_util import compare_phi, compare_states, radii, say

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def lp():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2206_11998_amd import lp as _lp
    _lp.lib()
    return _lp


def _dev(a):
    return torch.from_numpy(np.ascontiguousarray(a)).cuda()


SEARCH_MODES = [0, 1, 2]


def _nb_case(lp, oracle_lib, cfg, x, r, tag, mode=1, cap=0):
    say("neighbors", tag, x.shape, "search mode", mode, "cap", cap)
    ctx = lp.Context(cfg)
    ctx.set_tuning(lp.TUNE_SEARCH_MODE, mode)
    ctx.set_tuning(lp.TUNE_SEARCH_CAP, cap)
    count, idx, st = ctx.neighbors([_dev(x[:, a]) for a in range(cfg["dim"])], _dev(r))
    assert st == lp.OK
    count = count.cpu().numpy()
    idx = idx.cpu().numpy()
    rc, ri, rst = oracle_lib.neighbors(cfg, x, r, max_nb=ctx.max_nb)
    assert rst == 0
    assert np.array_equal(count, rc), np.nonzero(count != rc)[0][:5]
    for i in range(len(count)):
        k = count[i]
        assert np.array_equal(idx[i, :k], ri[i, :k]), i
    ctx.close()


@pytest.mark.parametrize("mode", SEARCH_MODES)
def test_neighbors_pulse2d(lp, oracle_lib, mode):
    cfg, st = W.pulse2d()
    _nb_case(lp, oracle_lib, cfg, st["x"], radii(cfg, st), "pulse2d", mode)


@pytest.mark.parametrize("mode", SEARCH_MODES)
def test_neighbors_lattice_ties(lp, oracle_lib, mode):
    cfg, st = W.uniform_box(3, 12, jitter=0.0)
    _nb_case(lp, oracle_lib, cfg, st["x"], radii(cfg, st), "exact lattice", mode)


@pytest.mark.parametrize("mode", SEARCH_MODES)
def test_neighbors_periodic_3d(lp, oracle_lib, mode):
    cfg, st = W.uniform_box(3, 24, seed=3)
    _nb_case(lp, oracle_lib, cfg, st["x"], radii(cfg, st), "jittered 24^3", mode)


@pytest.mark.parametrize("mode", SEARCH_MODES)
def test_neighbors_variable_radius(lp, oracle_lib, mode):
    cfg, st = W.vacuum3d(n_particles=150_000, seed=5)
    _nb_case(lp, oracle_lib, cfg, st["x"], radii(cfg, st), "vacuum 150k", mode)


@pytest.mark.parametrize("mode", SEARCH_MODES)
def test_neighbors_outside_box_and_anisotropic(lp, oracle_lib, mode):
    rng = np.random.default_rng(0)
    cfg = W.base_config("t", 3, 1.0, [0.0, 0.0, 0.0], [2.0, 1.0, 1.0], [True, False, True])
    x = rng.uniform([0, -0.2, 0], [2, 1.2, 1], size=(20000, 3))
    r = rng.uniform(0.02, 0.09, size=20000)
    cfg["max_nb"] = 256
    _nb_case(lp, oracle_lib, cfg, x, r, "mixed box", mode)


@pytest.mark.parametrize("mode", SEARCH_MODES)
def test_neighbors_long_lists(lp, oracle_lib, mode):
    """Lists longer than the search kernel's LDS buffer (128) take the overflow path."""
    cfg, st = W.uniform_box(3, 16, seed=8)
    cfg["max_nb"] = 256
    r = radii(cfg, st) * 1.75  # about 190 neighbours
    _nb_case(lp, oracle_lib, cfg, st["x"], r, "long lists", mode)


@pytest.mark.parametrize("cap", [8, 24])
def test_neighbors_small_lds_cap(lp, oracle_lib, cap):
    """With few LDS slots most lists are redone by the overflow kernel; on the
    exact lattice every shell of equal distances is a tie of staged keys."""
    cfg, st = W.uniform_box(3, 12, jitter=0.0)
    _nb_case(lp, oracle_lib, cfg, st["x"], radii(cfg, st), "exact lattice", 2, cap)


def test_neighbors_capacity(lp):
    cfg, st = W.uniform_box(2, 32)
    cfg["max_nb"] = 8
    ctx = lp.Context(cfg)
    count, idx, s = ctx.neighbors([_dev(st["x"][:, a]) for a in range(2)], _dev(radii(cfg, st)))
    assert s == lp.E_CAPACITY and int(count.max()) > 8


@pytest.mark.parametrize("dim", [2, 3])
def test_gfd_quadratic_and_oracle(lp, oracle_lib, dim):
    say("gfd", dim)
    rng = np.random.default_rng(10 + dim)
    cfg, st = W.uniform_box(dim, 40 if dim == 2 else 14, seed=2, periodic=False)
    cfg = dict(cfg, box_lo=[-0.5] * dim, box_hi=[1.5] * dim)
    x = st["x"]
    r = radii(cfg, st)
    fields = []
    for f in range(dim + 2):
        g = rng.standard_normal(dim)
        H = rng.standard_normal((dim, dim))
        H = 0.5 * (H + H.T)
        fields.append(1.0 + x @ g + 0.5 * np.einsum("ia,ab,ib->i", x, H, x) + 0.01 * np.sin(7 * x[:, 0]))
    ctx = lp.Context(cfg)
    deriv, status = ctx.gfd([_dev(x[:, a]) for a in range(dim)], _dev(r), [_dev(f) for f in fields])
    deriv = deriv.cpu().numpy()
    status = status.cpu().numpy()
    ref, rstat, rs = oracle_lib.gfd(cfg, x, r, fields)
    assert rs == 0
    assert np.array_equal(status, rstat)
    for f in range(len(fields)):
        for c in range(deriv.shape[1]):
            err = np.abs(deriv[f, c] - ref[f, c]).sum() / np.abs(ref[f, c]).sum()
            assert err <= 1e-10, (f, c, err)


def _run_both(lp, oracle_lib, cfg, st, nsteps, precision, tol, tag, dt=None, mode=None, refine_cond=0.0):
    say("step", tag, precision, st["V"].shape[0], "particles", nsteps, "steps", "search mode", mode,
        "refine_cond", refine_cond)
    ctx = lp.Context(cfg, precision=precision, refine_cond=refine_cond)
    if mode is not None:
        ctx.set_tuning(lp.TUNE_SEARCH_MODE, mode)
    dev = lp.state_to_device(st)
    ref = st
    for k in range(nsteps):
        d = oracle_lib.timestep(cfg, ref) if dt is None else dt
        ctx.step(dev, d)
        assert ctx.check() == lp.OK, lp.lib().lp_last_error(ctx._h)
        ref, info = oracle_lib.step(cfg, ref, d)
        assert info["status"] == 0
    got = lp.state_to_host(dev)
    compare_states(got, ref, cfg, tol, tag)
    compare_phi(got["phi"], info["phi"], precision == "fp64", tag)
    say(tag, "gpu info", ctx.info())
    return got, ref, info, ctx


@pytest.mark.parametrize("mode", SEARCH_MODES)
def test_step_pulse2d_fp64(lp, oracle_lib, mode):
    cfg, st = W.pulse2d()
    got, ref, info, ctx = _run_both(lp, oracle_lib, cfg, st, 10, "fp64", 1e-10, "pulse2d", mode=mode)
    assert np.array_equal(got["flags"] & 15, info["flags"] & 15)


def test_step_pulse2d_mixed(lp, oracle_lib):
    cfg, st = W.pulse2d()
    _run_both(lp, oracle_lib, cfg, st, 10, "mixed", 1e-4, "pulse2d")


def test_step_wave3d_fp64(lp, oracle_lib):
    cfg, st = W.smooth_wave(3, 20)
    _run_both(lp, oracle_lib, cfg, st, 5, "fp64", 1e-10, "wave3d")


def test_step_sod_slab_fp64(lp, oracle_lib):
    cfg, st = W.sod3d(n=64, ny=8, nz=8)
    got, ref, info, ctx = _run_both(lp, oracle_lib, cfg, st, 12, "fp64", 1e-10, "sod slab")
    assert ctx.info()["n_ghost"] == info["n_ghost"]


def test_step_sod_slab_mixed(lp, oracle_lib):
    cfg, st = W.sod3d(n=64, ny=8, nz=8)
    _run_both(lp, oracle_lib, cfg, st, 12, "mixed", 1e-4, "sod slab")


@pytest.mark.parametrize("refine_cond", [300.0, 1e3])
def test_step_vacuum_mixed_adaptive_refinement(lp, oracle_lib, refine_cond):
    """Mixed step refining only the fits whose condition estimate exceeds
    refine_cond (FP32 solution elsewhere)."""
    cfg, st = W.vacuum3d(n_particles=120_000, seed=9)
    got, ref, info, ctx = _run_both(lp, oracle_lib, cfg, st, 2, "mixed", 1e-4, "vacuum 120k", refine_cond=refine_cond)
    say("refined fits in the last step:", ctx.info()["n_refined"])


@pytest.mark.parametrize("mode", SEARCH_MODES)
def test_step_vacuum_fp64(lp, oracle_lib, mode):
    cfg, st = W.vacuum3d(n_particles=120_000, seed=9)
    got, ref, info, ctx = _run_both(lp, oracle_lib, cfg, st, 2, "fp64", 1e-10, "vacuum 120k", mode=mode)
    assert (info["flags"] & 4).sum() > 0  # vacuum ghosts were used


def test_constant_state_gpu(lp):
    cfg, st = W.uniform_box(3, 12, u0=[0.3, -0.2, 0.1], p=1.7, rho=0.8)
    ctx = lp.Context(cfg)
    dev = lp.state_to_device(st)
    ctx.step(dev)
    assert ctx.check() == lp.OK
    got = lp.state_to_host(dev)
    assert np.array_equal(got["V"], st["V"]) and np.array_equal(got["P"], st["P"])
    assert np.array_equal(got["u"], st["u"])


def test_conservation_and_determinism(lp, oracle_lib):
    cfg, st = W.pulse2d()
    outs = []
    for rep in range(2):
        ctx = lp.Context(cfg)
        dev = lp.state_to_device(st)
        m0 = ctx.conservation(dev)
        for _ in range(3):
            ctx.step(dev)
        m1 = ctx.conservation(dev)
        assert m1[0] == m0[0]
        outs.append(lp.state_to_host(dev))
    for k in ("V", "P", "u", "x"):
        assert np.array_equal(outs[0][k], outs[1][k]), k
    ref = oracle_lib.conservation(cfg, outs[0])
    assert np.allclose(m1, ref, rtol=1e-12, atol=1e-14)
