"""Neighbour lists (Sec. 2.2, step 3) bit-exact against the oracle at the
full sizes of the workloads, in the search configuration the benchmark
times (the autotuner's default, search mode 2): every list of the
262,144-particle Sod tube and of the 2,097,152-particle vacuum cloud, and a
sample of 200,000 lists (plus the hardest particles) of the 4,194,304-particle
blast and the 16,777,216-particle shear layer."""
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


def _gpu_lists(lp, cfg, x, r):
    ctx = lp.Context(cfg)
    xs = [torch.from_numpy(np.ascontiguousarray(x[:, a])).cuda() for a in range(cfg["dim"])]
    count, idx, st = ctx.neighbors(xs, torch.from_numpy(r).cuda())
    assert st == lp.OK
    count = count.cpu().numpy()
    idx = idx.cpu().numpy()
    ctx.close()
    del xs
    torch.cuda.empty_cache()
    return count, idx


def _check(count, idx, rc, ri, rows, tag):
    assert np.array_equal(count[rows], rc), tag
    k = idx.shape[1]
    mask = np.arange(k)[None, :] < rc[:, None]
    g = idx[rows]
    assert np.array_equal(np.where(mask, g, -1), np.where(mask, ri[:, :k], -1)), tag
    say(tag, "%d lists equal, %d entries, longest %d" % (rows.size, int(rc.sum()), int(rc.max())))


@pytest.mark.parametrize("name", ["sod 64^3", "vacuum 2M"])
def test_full_lists(lp, oracle_lib, name):
    if name == "sod 64^3":
        cfg, st = W.sod3d(n=64)
    else:
        cfg, st = W.vacuum3d()
    x, r = st["x"], radii(cfg, st)
    say("full lists:", name, x.shape[0], "particles")
    count, idx = _gpu_lists(lp, cfg, x, r)
    rc, ri, rs = oracle_lib.neighbors(cfg, x, r, max_nb=int(cfg.get("max_nb", 128)))
    assert rs == 0
    _check(count, idx, rc, ri, np.arange(x.shape[0]), name)


@pytest.mark.parametrize("name", ["sedov 4M", "shear 16M"])
def test_sampled_lists(lp, oracle_lib, name):
    if name == "sedov 4M":
        cfg, st = W.sedov3d()
        special = np.argsort(-st["P"])[:2000]
    else:
        cfg, st = W.shear3d()
        y = st["x"][:, 1]
        special = np.concatenate([np.argsort(y)[:1000], np.argsort(-y)[:1000], np.argsort(np.abs(y - 0.5))[:1000]])
    x, r = st["x"], radii(cfg, st)
    n = x.shape[0]
    rng = np.random.default_rng(91)
    rows = np.unique(np.concatenate([rng.choice(n, 200_000, replace=False), special]))
    say("sampled lists:", name, n, "particles,", rows.size, "compared")
    count, idx = _gpu_lists(lp, cfg, x, r)
    rc, ri, rs = oracle_lib.neighbors_subset(cfg, x, r, rows, max_nb=int(cfg.get("max_nb", 128)))
    assert rs == 0
    _check(count, idx, rc, ri, rows, name)
