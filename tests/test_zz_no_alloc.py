"""lp_neighbors_noalloc (the neighbour search without device allocation,
for callers that cannot allocate) against lp_neighbors: bit-identical
counts and lists on two calls in a row, the second with fewer particles,
a call too large for the scratch block rejected with LP_E_NOMEM and nothing
written, and the context's own workspace still working afterwards."""
import numpy as np
import pytest

from paper_2206_11998_amd import workloads as W
from tests.gpu_util import radii, say

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


def _noalloc(lp, ctx, x, r, max_nb):
    n = r.shape[0]
    count = torch.full((n,), -7, dtype=torch.int32, device="cuda")
    idx = torch.full((n, max_nb), -7, dtype=torch.int32, device="cuda")
    st = ctx.neighbors_noalloc(x, r, count, idx)
    torch.cuda.synchronize()
    return st, count.cpu().numpy(), idx.cpu().numpy()


def _same(lp, a_count, a_idx, b_count, b_idx, tag):
    assert np.array_equal(a_count, b_count), tag
    k = a_idx.shape[1]
    mask = np.arange(k)[None, :] < np.minimum(a_count, k)[:, None]
    assert np.array_equal(np.where(mask, a_idx, -1), np.where(mask, b_idx, -1)), tag


@pytest.mark.parametrize("name", ["vacuum 40k", "jittered 32^3"])
def test_noalloc_matches_neighbors_two_calls(lp, name):
    if name == "vacuum 40k":
        cfg, st = W.vacuum3d(n_particles=40_000, seed=4)
    else:
        cfg, st = W.uniform_box(3, 32, seed=6)
    x, r = st["x"], radii(cfg, st)
    ctx = lp.Context(cfg)
    for n in (x.shape[0], x.shape[0] // 3 + 17):
        say("noalloc", name, "n =", n)
        xs = [_dev(x[:n, a]) for a in range(3)]
        rd = _dev(r[:n])
        st_a, ca, ia = _noalloc(lp, ctx, xs, rd, ctx.max_nb)
        assert st_a == lp.OK, lp.lib().lp_last_error(ctx._h)
        cb, ib, st_b = ctx.neighbors(xs, rd)
        assert st_b == lp.OK
        _same(lp, ca, ia, cb.cpu().numpy(), ib.cpu().numpy(), "%s n=%d" % (name, n))
    ctx.close()


def test_noalloc_rejects_too_large_and_leaves_context_working(lp):
    cfg, st = W.uniform_box(3, 64, seed=7)   # 262,144 particles: more than the scratch block holds
    x, r = st["x"], radii(cfg, st)
    ctx = lp.Context(cfg)
    xs = [_dev(x[:, a]) for a in range(3)]
    rd = _dev(r)
    s, count, idx = _noalloc(lp, ctx, xs, rd, ctx.max_nb)
    say("too large:", s, lp.lib().lp_last_error(ctx._h))
    assert s == lp.E_NOMEM
    assert np.all(count == -7) and np.all(idx == -7)
    cb, ib, sb = ctx.neighbors(xs, rd)
    assert sb == lp.OK
    # a step on the context's own workspace after the rejected call
    small_cfg, small = W.pulse2d()
    ctx2 = lp.Context(small_cfg)
    dev = lp.state_to_device(small)
    xs2 = dev["x"]
    r2 = _dev(radii(small_cfg, small))
    s2, c2, i2 = _noalloc(lp, ctx2, xs2, r2, ctx2.max_nb)
    assert s2 == lp.OK
    ctx2.step(dev)
    assert ctx2.check() == lp.OK
    c3, i3, s3 = ctx2.neighbors(xs2, r2)
    ctx.close()
    ctx2.close()
