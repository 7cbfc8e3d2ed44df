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
