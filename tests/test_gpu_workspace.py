"""Caller-owned workspace (lp_workspace_bytes / lp_set_workspace): a time
step run entirely on a block the caller allocated (a torch uint8 tensor)
gives the library-allocated step's results bit for bit; a block too small
for the step returns LP_E_CAPACITY before anything changes; the network's
parameters move into the block; NULL returns to library buffers."""
import numpy as np
import pytest

from paper_2206_11998_amd import workloads as W
from tests.gpu_util import say

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def lp():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2206_11998_amd import lp as _lp
    _lp.lib()
    return _lp


CASES = {
    "pulse2d fp64": (lambda: W.pulse2d(), "fp64", 0.0),
    "sod slab fp64 (mirror ghosts)": (lambda: W.sod3d(n=64, ny=8, nz=8), "fp64", 0.0),
    "vacuum 60k mixed (refinement queue)": (lambda: W.vacuum3d(n_particles=60_000, seed=5), "mixed", 1e3),
}


def _same(a, b, tag):
    for k in ("x", "V", "u", "P", "phi", "flags"):
        assert np.array_equal(a[k], b[k]), (tag, k)


@pytest.mark.parametrize("case", list(CASES))
def test_run_on_caller_workspace_is_bit_identical(lp, case):
    gen, precision, rc = CASES[case]
    cfg, st = gen()
    own = lp.Context(cfg, precision=precision, refine_cond=rc)
    d_own = lp.state_to_device(st)
    own.run(d_own, 6)
    assert own.check() == lp.OK
    ws = lp.Context(cfg, precision=precision, refine_cond=rc)
    d_ws = lp.state_to_device(st)
    nbytes = ws.workspace_bytes(d_ws)
    block = torch.empty(nbytes, dtype=torch.uint8, device="cuda")
    ws.set_workspace(block)
    say("workspace", case, "%d bytes (%.1f MB) for %d particles" % (nbytes, nbytes / 1e6, st["V"].size))
    ws.run(d_ws, 6)
    assert ws.check() == lp.OK, lp.lib().lp_last_error(ws._h)
    _same(lp.state_to_host(d_ws), lp.state_to_host(d_own), case)
    # back to library-allocated buffers: the context still steps
    ws.set_workspace(None)
    ws.step(d_ws)
    own.step(d_own)
    _same(lp.state_to_host(d_ws), lp.state_to_host(d_own), case + " after NULL")
    own.close()
    ws.close()


def test_workspace_too_small(lp):
    cfg, st = W.pulse2d()
    ctx = lp.Context(cfg)
    dev = lp.state_to_device(st)
    nbytes = ctx.workspace_bytes(dev)
    block = torch.empty(nbytes // 2, dtype=torch.uint8, device="cuda")
    ctx.set_workspace(block)
    before = lp.state_to_host(dev)
    with pytest.raises(lp.LpError) as e:
        ctx.run(dev, 2)
    assert e.value.status == lp.E_CAPACITY
    say("too small:", lp.lib().lp_last_error(ctx._h))
    torch.cuda.synchronize()
    after = lp.state_to_host(dev)
    for k in ("x", "V", "u", "P"):
        assert np.array_equal(after[k], before[k]), k
    # a large enough block afterwards: the step runs
    big = torch.empty(nbytes, dtype=torch.uint8, device="cuda")
    ctx.set_workspace(big)
    ctx.run(dev, 2)
    assert ctx.check() == lp.OK
    with pytest.raises(lp.LpError):
        ctx.set_workspace(big[1:])  # not 256-byte aligned
    ctx.close()


def test_network_parameters_move_into_the_workspace(lp):
    cfg, st = W.pulse2d()
    ctx = lp.Context(cfg, estimator="mlp")
    ctx.mlp_init(5)
    p0 = ctx.mlp_get()
    dev = lp.state_to_device(st)
    block = torch.empty(ctx.workspace_bytes(dev), dtype=torch.uint8, device="cuda")
    ctx.set_workspace(block)
    assert np.array_equal(ctx.mlp_get(), p0)
    ctx.run(dev, 2)
    assert ctx.check() == lp.OK
    ctx.close()


def test_open_run_on_caller_workspace_is_bit_identical(lp):
    """lp_run_open (outflow and an inflow layer every second step, 14 steps)
    on a block sized by lp_workspace_bytes for the capacity -- the slots past
    the particles given absent, as the call makes them -- gives the
    library-allocated run's result bit for bit, compaction included."""
    from tests.test_gpu_openbc import _capacity_state, _channel, _head
    cfg, st, h = _channel()
    n = len(st["V"])
    cap = n + 7 * 32 + 5
    kw = dict(out_hi_mask=1, in_every=2, in_axis=0, in_side=0, spacing=h, depth=0.5 * h, rho=1.0, p_in=1.0, u_n=1.0)
    res = []
    for caller in (False, True):
        ctx = lp.Context(cfg, precision="mixed", refine_cond=1e3)
        dev = lp.state_to_device(_capacity_state(st, cap, 2))
        if caller:
            probe = {k: ([t.clone() for t in v] if isinstance(v, list) else v.clone()) for k, v in dev.items()}
            probe["m"][n:] = 0.0
            nbytes = ctx.workspace_bytes(probe)
            block = torch.empty(nbytes, dtype=torch.uint8, device="cuda")
            ctx.set_workspace(block)
            say("open run workspace: %d bytes for capacity %d" % (nbytes, cap))
        n_out = ctx.run_open(dev, n, 14, **kw)
        assert ctx.check() == lp.OK, lp.lib().lp_last_error(ctx._h)
        res.append((n_out, lp.state_to_host(_head(dev, n_out))))
        ctx.close()
    assert res[0][0] == res[1][0]
    _same(res[1][1], res[0][1], "open run")
