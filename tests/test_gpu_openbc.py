"""Open boundaries on the GPU against the oracle: outflow deletion must keep
the same particles in the same order, bit for bit, and the reservoir inflow
state must agree within rounding (the layer's mean pressure is summed in
another order)."""
import numpy as np
import pytest

from paper_2206_11998_amd import workloads as W
from tests.gpu_util import compare_states, say
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


def _channel(n=32, u0=1.0, seed=5):
    """2D channel, x open on both sides (no walls, free-surface treatment), y
    periodic: a jittered n x n lattice of h = 1/n in uniform flow u0 along x
    with a pressure pulse.  At u0 = 1 a column moves about h every two
    steps, so a layer every second step at half a spacing inside the face
    finds room."""
    h = 1.0 / n
    x, _ = W.jittered_lattice((n, n), h, 0.15, seed)
    rho = np.ones(x.shape[0])
    p = 1.0 + 0.1 * np.exp(-((x - 0.5) ** 2).sum(axis=1) / 0.02)
    u = np.zeros_like(x)
    u[:, 0] = u0
    cfg = W.base_config("channel2d", 2, 2.5, [0.0, 0.0], [1.0, 1.0], [False, True], vacuum=True)
    st = {"x": x, "u": u, "V": 1.0 / rho, "P": p, "m": rho * h * h}
    return cfg, st, h


def _oracle_open(oracle_lib, cfg, st, nsteps, lo_mask, hi_mask, every=0, axis=0, side=0, spacing=0.0, depth=0.0,
                 rho=0.0, p_in=0.0, u_n=0.0, res=None):
    """The oracle's sequence: each step, then the outflow, then on every
    every-th step the inflow layer (fixed state, or res = (width, p_res,
    rho_res): the reservoir state of that moment)."""
    ref = {k: st[k].copy() for k in ("x", "u", "V", "P", "m")}
    layers = 0
    for k in range(1, nsteps + 1):
        ref, info = oracle_lib.step(cfg, ref)
        assert info["status"] == 0
        ref = oracle_lib.outflow(cfg, ref, lo_mask, hi_mask)
        if every and k % every == 0:
            if res is not None:
                out, rs = oracle_lib.reservoir_inflow(cfg, ref, axis, side, res[0], res[1], res[2])
                assert rs == 0
                p_in, rho, u_n = (float(v) for v in out[:3])
            n = len(ref["V"])
            lay, n_new, rs = oracle_lib.inflow_layer(cfg, n, n + 100000, axis, side, spacing, depth, rho, p_in, u_n)
            assert rs == 0
            ref = {q: np.concatenate([ref[q], lay[q]]) for q in ("x", "u", "V", "P", "m")}
            layers += 1
    return ref, layers


@pytest.mark.parametrize("precision", ["fp64", "mixed"])
def test_run_open_without_faces_equals_run(lp, precision):
    """No outflow face and no inflow: lp_run_open on arrays with spare slots
    gives lp_run's result bit for bit (the absent slots change no ranking)."""
    say("run_open without faces", precision)
    cfg, st, h = _channel()
    n = len(st["V"])
    a = lp.state_to_device(st)
    ctx_a = lp.Context(cfg, precision=precision)
    ctx_a.run(a, 6)
    assert ctx_a.check() == lp.OK
    b = lp.state_to_device(_capacity_state(st, n + 777, 2))
    ctx_b = lp.Context(cfg, precision=precision)
    assert ctx_b.run_open(b, n, 6) == n
    assert ctx_b.check() == lp.OK
    ga, gb = lp.state_to_host(a), lp.state_to_host(_head(b, n))
    for key in ("x", "u", "V", "P", "m", "phi", "flags"):
        assert np.array_equal(ga[key], gb[key]), key
    assert ctx_b.info()["t"] == ctx_a.info()["t"]
    ctx_a.close()
    ctx_b.close()


@pytest.mark.parametrize("precision,tol", [("fp64", 1e-10), ("mixed", 1e-4)])
def test_run_open_outflow_and_inflow_matches_oracle(lp, oracle_lib, precision, tol):
    """Channel flow through an outflow face at x = 1 with a lattice layer of
    the inflow state entering at x = 0 every second step, all inside one
    lp_run_open call of 14 steps replaying one captured step, against the
    oracle's step, outflow and layer sequence."""
    say("run_open outflow + inflow", precision)
    cfg, st, h = _channel()
    n = len(st["V"])
    kw = dict(every=2, axis=0, side=0, spacing=h, depth=0.5 * h, rho=1.0, p_in=1.0, u_n=1.0)
    ref, layers = _oracle_open(oracle_lib, cfg, st, 14, 0, 1, **kw)
    assert layers == 7 and len(ref["V"]) != n
    dev = lp.state_to_device(_capacity_state(st, n + 7 * 32 + 5, 2))
    ctx = lp.Context(cfg, precision=precision)
    n_out = ctx.run_open(dev, n, 14, out_hi_mask=1, in_every=2, in_axis=0, in_side=0, spacing=h, depth=0.5 * h,
                         rho=1.0, p_in=1.0, u_n=1.0)
    assert ctx.check() == lp.OK
    assert n_out == len(ref["V"])
    info = ctx.info()
    assert info["n_captures"] == 1, info
    got = lp.state_to_host(_head(dev, n_out))
    assert np.array_equal(got["m"], ref["m"])    # the same particles, in the same order
    compare_states(got, ref, cfg, tol, "run_open " + precision)
    ctx.close()


def test_run_open_reservoir_matches_oracle(lp, oracle_lib):
    """The layers take the reservoir state of the particles inside the inflow
    face at the moment each is written (FP64, 1e-10: the layer's mean
    pressure is summed in another order)."""
    say("run_open reservoir inflow")
    cfg, st, h = _channel(seed=6)
    n = len(st["V"])
    res = (2 * h, 1.3, 1.0)
    ref, layers = _oracle_open(oracle_lib, cfg, st, 12, 0, 1, every=3, axis=0, side=0, spacing=h, depth=0.5 * h,
                               res=res)
    assert layers == 4
    dev = lp.state_to_device(_capacity_state(st, n + 4 * 32, 2))
    ctx = lp.Context(cfg, precision="fp64")
    n_out = ctx.run_open(dev, n, 12, out_hi_mask=1, in_every=3, in_axis=0, in_side=0, spacing=h, depth=0.5 * h,
                         res_width=res[0], res_p=res[1], res_rho=res[2])
    assert ctx.check() == lp.OK
    assert n_out == len(ref["V"])
    compare_states(lp.state_to_host(_head(dev, n_out)), ref, cfg, 1e-10, "run_open reservoir")
    ctx.close()


def test_run_open_layer_past_capacity_stops(lp, oracle_lib):
    """A layer that does not fit is not written: the run stops after that
    step, lp_check reports the capacity error, and the arrays are compacted
    to the particles of that step."""
    say("run_open capacity")
    cfg, st, h = _channel()
    n = len(st["V"])
    dev = lp.state_to_device(_capacity_state(st, n + 40, 2))     # one layer of 32 fits, two do not
    ctx = lp.Context(cfg, precision="fp64")
    kw = dict(in_every=2, in_axis=0, in_side=0, spacing=h, depth=0.5 * h, rho=1.0, p_in=1.0, u_n=1.0)
    n_out = ctx.run_open(dev, n, 8, out_hi_mask=1, **kw)
    assert ctx.check() == lp.E_CAPACITY
    ref, layers = _oracle_open(oracle_lib, cfg, st, 4, 0, 1, every=2, axis=0, side=0, spacing=h, depth=0.5 * h,
                               rho=1.0, p_in=1.0, u_n=1.0)
    # steps 1-4 ran; the second layer (after step 4) was refused
    ref2, _ = _oracle_open(oracle_lib, cfg, st, 3, 0, 1, every=2, axis=0, side=0, spacing=h, depth=0.5 * h,
                           rho=1.0, p_in=1.0, u_n=1.0)
    ref4 = oracle_lib.outflow(cfg, oracle_lib.step(cfg, ref2)[0], 0, 1)
    assert n_out == len(ref4["V"]) == len(ref["V"]) - 32
    compare_states(lp.state_to_host(_head(dev, n_out)), ref4, cfg, 1e-10, "run_open capacity")
    with pytest.raises(lp.LpError) as e:
        ctx.run_open(dev, n_out, 2, out_hi_mask=4)                  # no z axis in 2D
    assert e.value.status == lp.E_ARG
    ctx.close()


def test_run_open_when_every_particle_leaves(lp):
    """An outflow face behind every particle: the first step deletes them all,
    the run stops there (time advanced by that step alone), nothing is
    reported as an error, and the call returns a count of 0."""
    say("run_open: every particle leaves")
    cfg, st, h = _channel()
    cfg = dict(cfg, box_hi=[1e-9, 1.0])
    n = len(st["V"])
    dev = lp.state_to_device(_capacity_state(st, n + 64, 2))
    ctx = lp.Context(cfg, precision="fp64")
    assert ctx.run_open(dev, n, 6, out_hi_mask=1) == 0
    assert ctx.check() == lp.OK
    info = ctx.info()
    one = lp.Context(cfg, precision="fp64")
    ref = lp.state_to_device(st)
    one.step(ref)
    assert info["t"] == one.info()["t"] > 0.0
    ctx.close()
    one.close()


def test_run_open_zero_steps_keeps_the_particles(lp):
    """nsteps = 0: nothing advances, the spare slots are marked absent and the
    particles given come back as they were, in order."""
    say("run_open: zero steps")
    cfg, st, h = _channel()
    n = len(st["V"])
    dev = lp.state_to_device(_capacity_state(st, n + 10, 2))
    ctx = lp.Context(cfg, precision="fp64")
    assert ctx.run_open(dev, n, 0, out_hi_mask=1) == n
    got = lp.state_to_host(_head(dev, n))
    for key in ("x", "u", "V", "P", "m"):
        assert np.array_equal(got[key], st[key]), key
    assert np.all(dev["m"][n:].cpu().numpy() == 0.0)
    ctx.close()
