"""Open boundaries on the GPU against the oracle: outflow deletion must keep
the same particles in the same order, bit for bit, and the reservoir inflow
state must agree within rounding (the layer's mean pressure is summed in
another order)."""
import numpy as np
import pytest

from paper_2206_11998_amd import workloads as W
from tests.gpu_util import say
from tests.test_oracle_openbc import _cloud

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def lp():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2206_11998_amd import lp as _lp
    _lp.lib()
    return _lp


def _head(st, k):
    return {key: ([t[:k] for t in v] if isinstance(v, list) else v[:k]) for key, v in st.items()}


@pytest.mark.parametrize("dim", [2, 3])
@pytest.mark.parametrize("lo_mask,hi_mask", [(1, 0), (0, 1), (1, 2), (3, 3), (0, 0)])
def test_outflow_matches_oracle(lp, oracle_lib, dim, lo_mask, hi_mask):
    say("outflow", dim, lo_mask, hi_mask)
    cfg, st = _cloud(dim, 3001, seed=40 + dim + lo_mask + 4 * hi_mask)
    ref = oracle_lib.outflow(cfg, st, lo_mask, hi_mask)
    ctx = lp.Context(cfg)
    dev = lp.state_to_device(st)
    n = len(st["V"])
    dev["phi"].copy_(torch.arange(n, dtype=torch.float32))
    dev["flags"].copy_(torch.arange(n, dtype=torch.int64).remainder(251).to(torch.uint8))
    kept = ctx.outflow(dev, lo_mask, hi_mask)
    torch.cuda.synchronize()
    assert kept == len(ref["V"])
    got = lp.state_to_host(_head(dev, kept))
    for key in ("x", "u", "V", "P", "m"):
        assert np.array_equal(got[key], ref[key]), key
    # phi and flags follow the same particles
    idx = got["phi"].astype(np.int64)
    assert np.array_equal(st["V"][idx], ref["V"])
    assert np.array_equal(got["flags"], (idx % 251).astype(np.uint8))
    ctx.close()


@pytest.mark.parametrize("axis,side", [(0, 0), (1, 1), (2, 0)])
def test_reservoir_inflow_matches_oracle(lp, oracle_lib, axis, side):
    say("reservoir inflow", axis, side)
    cfg, st = _cloud(3, 20000, seed=7)
    st["P"] = 0.3 + 0.2 * np.random.default_rng(2).random(20000)
    ref, rs = oracle_lib.reservoir_inflow(cfg, st, axis, side, 0.1, 2.0, 1.5)
    assert rs == 0
    ctx = lp.Context(cfg)
    got = ctx.reservoir_inflow(lp.state_to_device(st), axis, side, 0.1, 2.0, 1.5)
    assert got[3] == ref[3]
    assert np.allclose(got[:3], ref[:3], rtol=1e-12, atol=0.0), (got, ref)
    with pytest.raises(lp.LpError):
        ctx.reservoir_inflow(lp.state_to_device(st), 3, 0, 0.1, 2.0, 1.5)
    ctx.close()


def test_outflow_2m_vacuum_cloud(lp):
    """The 2M-particle vacuum cloud with an outflow face through its middle:
    the kept count and the order of the kept particles at full size."""
    say("outflow 2M")
    cfg, st = W.vacuum3d()
    cfg = dict(cfg, box_hi=[0.0] + list(cfg["box_hi"][1:]))
    ctx = lp.Context(cfg)
    dev = lp.state_to_device(st)
    n = len(st["V"])
    dev["phi"].copy_(torch.arange(n, dtype=torch.float32))
    kept = ctx.outflow(dev, 0, 1)
    keep = st["x"][:, 0] < 0.0
    assert kept == keep.sum() and 0 < kept < n
    idx = dev["phi"][:kept].cpu().numpy().astype(np.int64)
    assert np.array_equal(idx, np.flatnonzero(keep))
    assert np.array_equal(dev["V"][:kept].cpu().numpy(), st["V"][keep])
    ctx.close()


def _capacity_state(st, cap, dim):
    """Device arrays of `cap` entries holding the particles of st first, the
    rest filled with a marker value."""
    n = len(st["V"])
    full = {"x": np.full((cap, dim), 7.0), "u": np.full((cap, dim), 7.0), "V": np.full(cap, 7.0),
            "P": np.full(cap, 7.0), "m": np.full(cap, 7.0)}
    for k in full:
        full[k][:n] = st[k]
    return full


@pytest.mark.parametrize("dim,axis,side", [(2, 0, 0), (2, 1, 1), (3, 0, 1), (3, 2, 0), (3, 1, 0)])
def test_inflow_layer_matches_oracle(lp, oracle_lib, dim, axis, side):
    say("inflow layer", dim, axis, side)
    cfg, st = _cloud(dim, 1000, seed=60 + dim + axis)
    cfg = dict(cfg, box_lo=[-0.5, 0.0, 0.25][:dim], box_hi=[0.5, 0.7, 1.0][:dim])
    h, depth, rho, p_in, u_n = 0.013, 0.002, 1.3, 0.8, 0.4
    n, cap = 1000, 1000 + 6000
    ref, n_ref, rs = oracle_lib.inflow_layer(cfg, n, cap, axis, side, h, depth, rho, p_in, u_n)
    assert rs == 0 and n_ref > n
    ctx = lp.Context(cfg)
    dev = lp.state_to_device(_capacity_state(st, cap, dim))
    dev["phi"].fill_(5.0)
    dev["flags"].fill_(9)
    n_new = ctx.inflow_layer(dev, n, axis, side, h, depth, rho, p_in, u_n)
    torch.cuda.synchronize()
    assert n_new == n_ref
    got = lp.state_to_host(dev)
    for key in ("x", "u", "V", "P", "m"):
        assert np.array_equal(got[key][n:n_new], ref[key]), key
        assert np.array_equal(got[key][:n], st[key]), key          # existing particles untouched
        assert np.all(got[key][n_new:] == 7.0), key                 # nothing past the layer
    assert np.all(got["phi"][n:n_new] == 1.0) and np.all(got["phi"][:n] == 5.0)
    assert np.all(got["flags"][n:n_new] == 0) and np.all(got["flags"][n_new:] == 9)
    ctx.close()


def test_inflow_layer_errors_leave_arrays(lp, oracle_lib):
    say("inflow layer errors")
    cfg, st = _cloud(2, 100, seed=3)
    ctx = lp.Context(cfg)
    dev = lp.state_to_device(_capacity_state(st, 105, 2))
    with pytest.raises(lp.LpError) as e:
        ctx.inflow_layer(dev, 100, 0, 0, 0.1, 0.0, 1.0, 1.0, 0.5)     # 10 new particles, room for 5
    assert e.value.status == 2
    with pytest.raises(lp.LpError) as e:
        ctx.inflow_layer(dev, 100, 2, 0, 0.1, 0.0, 1.0, 1.0, 0.5)     # no z axis in 2D
    assert e.value.status == 1
    assert ctx.inflow_layer(dev, 100, 1, 1, 1.5, 0.0, 1.0, 1.0, 0.5) == 100   # spacing wider than the face
    torch.cuda.synchronize()
    assert np.all(dev["V"][100:].cpu().numpy() == 7.0)
    ctx.close()


def test_inflow_layer_after_outflow_2m(lp, oracle_lib):
    """At the 2M vacuum cloud's size: delete past an outflow face, then append
    a 256 x 256 inflow layer carrying the reservoir state computed at the
    outflow face, checked against the oracle bit for bit."""
    say("outflow + inflow layer 2M")
    cfg, st = W.vacuum3d()
    n = len(st["V"])
    cfg = dict(cfg, box_hi=[0.0] + list(cfg["box_hi"][1:]))
    ctx = lp.Context(cfg)
    cap = n + 300000
    dev = lp.state_to_device(_capacity_state(st, cap, 3))
    head = {k: ([t[:n] for t in v] if isinstance(v, list) else v[:n]) for k, v in dev.items()}
    kept = ctx.outflow(head, 0, 1)
    p_in, rho_in, u_in, cnt = ctx.reservoir_inflow(_head(dev, kept), 0, 1, 0.02, 2.0, 1.5)
    assert cnt > 0 and u_in > 0.0
    ext = cfg["box_hi"][1] - cfg["box_lo"][1]
    h = ext / 256
    n_new = ctx.inflow_layer(dev, kept, 0, 0, h, 0.5 * h, rho_in, p_in, u_in)
    ref, n_ref, rs = oracle_lib.inflow_layer(cfg, kept, cap, 0, 0, h, 0.5 * h, rho_in, p_in, u_in)
    assert rs == 0 and n_new == n_ref
    torch.cuda.synchronize()
    for key in ("V", "P", "m"):
        assert np.array_equal(dev[key][kept:n_new].cpu().numpy(), ref[key]), key
    for a in range(3):
        assert np.array_equal(dev["x"][a][kept:n_new].cpu().numpy(), ref["x"][:, a])
        assert np.array_equal(dev["u"][a][kept:n_new].cpu().numpy(), ref["u"][:, a])
    ctx.close()


def test_run_across_outflow_and_inflow_layer(lp, oracle_lib):
    """Open-boundary calls between graph-replayed runs.  A jittered 2D pulse
    between mirror walls at x = -h and x = 0.9 (y periodic) is cut at the
    outflow face, run two steps with lp_run, given one inflow layer at the low
    face carrying a reservoir state, then run two more steps on the new count.
    That second run needs a new capture. FP64 against the oracle stepping the
    same particles, within 1e-10 relative L1."""
    from tests.gpu_util import compare_states
    say("lp_run across outflow and an inflow layer")
    cfg, st = W.pulse2d(n=48)
    h = 1.0 / 48
    cfg = dict(cfg, box_lo=[-h, 0.0], box_hi=[0.9, 1.0], periodic=[False, True], wall_lo=[True, False],
               wall_hi=[True, False])
    ctx = lp.Context(cfg, precision="fp64")
    dev = lp.state_to_device(st)
    kept = ctx.outflow(dev, 0, 1)
    ref = oracle_lib.outflow(cfg, st, 0, 1)
    assert kept == len(ref["V"]) < len(st["V"])
    ctx.run(_head(dev, kept), 2)
    assert ctx.check() == lp.OK
    for _ in range(2):
        ref, info = oracle_lib.step(cfg, ref)
        assert info["status"] == 0
    compare_states(lp.state_to_host(_head(dev, kept)), ref, cfg, 1e-10, "before the layer")
    res, rs = oracle_lib.reservoir_inflow(cfg, ref, 0, 0, 2 * h, 1.1, 1.05)
    got = ctx.reservoir_inflow(_head(dev, kept), 0, 0, 2 * h, 1.1, 1.05)
    assert rs == 0 and got[3] == res[3] and np.allclose(got[:3], res[:3], rtol=1e-10, atol=0.0)
    p_in, rho_in, u_in = (float(v) for v in res[:3])
    n_new = ctx.inflow_layer(dev, kept, 0, 0, h, 0.5 * h, rho_in, p_in, u_in)
    lay, n_ref, rs = oracle_lib.inflow_layer(cfg, kept, len(st["V"]), 0, 0, h, 0.5 * h, rho_in, p_in, u_in)
    assert rs == 0 and n_new == n_ref == kept + 48
    ref = {k: np.concatenate([ref[k], lay[k]]) for k in ("x", "u", "V", "P", "m")}
    ctx.run(_head(dev, n_new), 2)
    assert ctx.check() == lp.OK
    for _ in range(2):
        ref, info = oracle_lib.step(cfg, ref)
        assert info["status"] == 0
    compare_states(lp.state_to_host(_head(dev, n_new)), ref, cfg, 1e-10, "after the layer")
    ctx.close()


@pytest.mark.parametrize("dim", [2, 3])
def test_outflow_and_inflow_layer_without_phi_and_flags(lp, oracle_lib, dim):
    """phi and flags are optional: both calls leave them out and still match
    the oracle bit for bit."""
    say("open boundaries without phi/flags", dim)
    cfg, st = _cloud(dim, 2000, seed=90 + dim)
    ref = oracle_lib.outflow(cfg, st, 1, 2)
    ctx = lp.Context(cfg)
    dev = lp.state_to_device(st)
    del dev["phi"], dev["flags"]
    kept = ctx.outflow(dev, 1, 2)
    assert kept == len(ref["V"])
    got = lp.state_to_host(dict(_head(dev, kept), phi=torch.zeros(1), flags=torch.zeros(1)))
    for key in ("x", "u", "V", "P", "m"):
        assert np.array_equal(got[key], ref[key]), key
    lay, n_ref, rs = oracle_lib.inflow_layer(cfg, kept, len(st["V"]), 0, 1, 0.05, 0.01, 1.2, 0.9, 0.3)
    assert rs == 0
    n_new = ctx.inflow_layer(dev, kept, 0, 1, 0.05, 0.01, 1.2, 0.9, 0.3)
    assert n_new == n_ref
    torch.cuda.synchronize()
    for key in ("V", "P", "m"):
        assert np.array_equal(dev[key][kept:n_new].cpu().numpy(), lay[key]), key
    for a in range(dim):
        assert np.array_equal(dev["x"][a][kept:n_new].cpu().numpy(), lay["x"][:, a])
        assert np.array_equal(dev["u"][a][kept:n_new].cpu().numpy(), lay["u"][:, a])
    ctx.close()
