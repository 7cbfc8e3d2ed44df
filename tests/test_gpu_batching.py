"""Batching on the GPU: the stencil-size work queue (plain and persistent
launches), graph-replayed steps (lp_run) and the autotuner.

None of these may change a result: every comparison here is bit for bit
against the plain one-thread-per-particle, one-launch-per-step path, which the
parity tests tie to the oracle."""
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
    "pulse2d": lambda: W.pulse2d(),
    "sod slab": lambda: W.sod3d(n=64, ny=8, nz=8),
    "vacuum 60k": lambda: W.vacuum3d(n_particles=60_000, seed=5),
}


def _same(a, b, tag):
    for k in ("x", "V", "u", "P", "phi", "flags"):
        assert np.array_equal(a[k], b[k]), (tag, k, np.nonzero(np.asarray(a[k] != b[k]).reshape(len(a[k]), -1).any(1))[0][:5])


def _steps(lp, cfg, st, nsteps, precision="fp64", tuning=None):
    ctx = lp.Context(cfg, precision=precision)
    for p, v in (tuning or {}).items():
        ctx.set_tuning(p, v)
    dev = lp.state_to_device(st)
    for _ in range(nsteps):
        ctx.step(dev)
    assert ctx.check() == lp.OK, lp.lib().lp_last_error(ctx._h)
    out = lp.state_to_host(dev)
    ctx.close()
    return out


@pytest.mark.parametrize("case", list(CASES))
@pytest.mark.parametrize("precision", ["fp64", "mixed"])
def test_solve_modes_identical(lp, case, precision):
    cfg, st = CASES[case]()
    ref = None
    for mode, block, tile in ((0, 256, 1024), (1, 256, 1024), (1, 128, 256), (2, 256, 1024), (2, 64, 512)):
        tag = "%s %s solve mode %d block %d tile %d" % (case, precision, mode, block, tile)
        say("batching", tag)
        got = _steps(lp, cfg, st, 3, precision,
                     {lp.TUNE_SOLVE_MODE: mode, lp.TUNE_SOLVE_BLOCK: block, lp.TUNE_QUEUE_TILE: tile})
        if ref is None:
            ref = got
        else:
            _same(got, ref, tag)


@pytest.mark.parametrize("case", list(CASES))
def test_search_cap_identical(lp, case):
    """The search's LDS list slots: automatic (from the previous step's
    longest list), the full 128, and caps small enough that most lists are
    redone by the overflow kernel."""
    cfg, st = CASES[case]()
    ref = _steps(lp, cfg, st, 3, tuning={lp.TUNE_SEARCH_CAP: 128})
    for cap in (0, 8, 40):
        say("search cap", case, cap)
        _same(_steps(lp, cfg, st, 3, tuning={lp.TUNE_SEARCH_CAP: cap}), ref, "%s search cap %d" % (case, cap))


def test_adaptive_refinement_selects_per_particle(lp):
    """refine_cond > 0: a particle's update depends only on its own fit, so
    after one step every particle equals, bit for bit, either the step that
    refines every fit or the step that refines none, and the particles taking
    the refined result are the ones counted as refined."""
    cfg, st = CASES["vacuum 60k"]()
    runs = {}
    for tag, refine, cond in (("all", True, 0.0), ("none", False, 0.0), ("adaptive", True, 300.0)):
        ctx = lp.Context(cfg, precision="mixed", refine=refine, refine_cond=cond)
        dev = lp.state_to_device(st)
        ctx.step(dev)
        assert ctx.check() == lp.OK
        runs[tag] = (lp.state_to_host(dev), ctx.info())
        ctx.close()
    n = st["V"].shape[0]

    def same(a, b):
        eq = np.ones(n, bool)
        for k in ("x", "V", "u", "P", "phi", "flags"):
            d = np.asarray(a[k] == b[k]).reshape(n, -1).all(1)
            eq &= d
        return eq
    ad, inf = runs["adaptive"]
    eq_all, eq_none = same(ad, runs["all"][0]), same(ad, runs["none"][0])
    assert np.all(eq_all | eq_none), np.nonzero(~(eq_all | eq_none))[0][:5]
    took_refined = int((eq_all & ~eq_none).sum())
    say("adaptive refinement: %d fits refined, %d particles differ from the unrefined step"
        % (inf["n_refined"], took_refined))
    assert runs["all"][1]["n_refined"] == 0 and runs["none"][1]["n_refined"] == 0
    assert 0.05 * n < inf["n_refined"] < 0.95 * n
    # a refined fit leaves the state unchanged where phi = 0 (no LW part) or
    # where its correction rounds away
    assert 0.25 * inf["n_refined"] <= took_refined <= inf["n_refined"]


@pytest.mark.parametrize("case", list(CASES))
def test_run_graph_matches_steps(lp, case):
    cfg, st = CASES[case]()
    # planning step + full replay chunks + a partial one (the edge of the
    # coarse 60k-particle vacuum cloud outgrows max_nb = 256 after 8 steps, so
    # that case stops at 5 + 2)
    nsteps = 5 if case.startswith("vacuum") else 19
    say("lp_run vs lp_step", case, nsteps)
    ref = _steps(lp, cfg, st, nsteps)
    for mode in (0, 2):
        ctx = lp.Context(cfg)
        ctx.set_tuning(lp.TUNE_SOLVE_MODE, mode)
        ctx.set_tuning(lp.TUNE_QUEUE_TILE, 256)
        dev = lp.state_to_device(st)
        ctx.run(dev, nsteps)
        assert ctx.check() == lp.OK
        _same(lp.state_to_host(dev), ref, "%s lp_run solve mode %d" % (case, mode))
        # a second call reuses the captured graph
        ctx.run(dev, 2)
        ref2 = _steps(lp, cfg, st, nsteps + 2)
        _same(lp.state_to_host(dev), ref2, "%s second lp_run" % case)
        ctx.close()


def test_run_stops_at_first_error(lp):
    """The coarse 60k-particle vacuum cloud outgrows max_nb = 256 after a few
    steps: lp_run stops at the step that overflows, with the time and state
    that lp_step reaches there, and lp_check reports the capacity error."""
    cfg, st = CASES["vacuum 60k"]()
    ctx = lp.Context(cfg)
    dev = lp.state_to_device(st)
    for k in range(1, 40):
        ctx.step(dev)
        if ctx.check() != lp.OK:
            break
    else:
        pytest.skip("no capacity error within 40 steps")
    t_fail = ctx.info()["t"]
    ref = lp.state_to_host(dev)
    ctx.close()
    say("first failing step", k, "t", t_fail)
    ctx = lp.Context(cfg)
    dev = lp.state_to_device(st)
    ctx.run(dev, k + 20)
    assert ctx.check() == lp.E_CAPACITY
    assert ctx.info()["t"] == t_fail
    _same(lp.state_to_host(dev), ref, "lp_run stopped at the failing step")
    ctx.close()


def test_run_stops_on_t_end(lp):
    cfg, st = CASES["sod slab"]()
    ctx = lp.Context(cfg)
    dev = lp.state_to_device(st)
    ctx.step(dev)
    dt0 = ctx.info()["dt"]
    ctx.close()
    t_end = 6.5 * dt0
    say("lp_run t_end", t_end)
    # reference: one planning step per call, each clipped on the device
    ctx = lp.Context(cfg)
    ref = lp.state_to_device(st)
    n_ref = 0
    while ctx.info()["t"] < t_end and n_ref < 100:
        ctx.run(ref, 1, t_end)
        n_ref += 1
    ctx.close()
    ctx = lp.Context(cfg)
    dev = lp.state_to_device(st)
    ctx.run(dev, 1000, t_end)
    info = ctx.info()
    assert info["t"] == t_end, (info["t"], t_end)
    _same(lp.state_to_host(dev), lp.state_to_host(ref), "t_end")
    assert 6 <= n_ref <= 9


def test_autotune_leaves_state_and_results(lp):
    cfg, st = CASES["sod slab"]()
    ctx = lp.Context(cfg)
    dev = lp.state_to_device(st)
    before = lp.state_to_host(dev)
    say("autotune")
    best, ms = ctx.autotune(dev, reps=1)
    say("autotune chose", best, "%.3f ms/step" % ms)
    assert ms > 0
    assert best["solve_mode"] in (0, 1, 2) and best["solve_block"] in (64, 128, 256)
    assert best["search_mode"] in (0, 1, 2) and best["search_group"] in (4, 8, 16, 32)
    assert best["queue_tile"] in (256, 512, 1024)
    assert ctx.info()["t"] == 0.0
    after = lp.state_to_host(dev)
    for k in ("x", "V", "u", "P"):
        assert np.array_equal(after[k], before[k]), k
    for q, name in enumerate(lp.TUNE_NAMES):
        assert ctx.get_tuning(q) == best[name]
    for _ in range(3):
        ctx.step(dev)
    _same(lp.state_to_host(dev), _steps(lp, cfg, st, 3), "after autotune")


def test_step_stage_timing(lp):
    cfg, st = CASES["pulse2d"]()
    ctx = lp.Context(cfg)
    dev = lp.state_to_device(st)
    ctx.profile(True)
    ctx.step(dev)
    ctx.run(dev, 10)
    prof = ctx.profile_read()
    ctx.profile(False)
    say("stages", prof)
    assert prof["step"][1] == 11  # one eager step, one planning step, nine replays
    assert prof["search"][1] == 2 and prof["fit"][1] == 2
    assert all(v[0] >= 0 for v in prof.values())


def test_autotune_failure_leaves_the_context_clean(lp):
    """A candidate step that runs out of list capacity makes lp_autotune
    fail, but the caller's context keeps its clock, step count and error
    bits: after widening nothing, a plain step of the same particles still
    reports the same capacity error, and a context whose autotune succeeded
    after steps of its own continues from its own time."""
    cfg, st = CASES["sod slab"]()
    small = dict(cfg, max_nb=16)
    ctx = lp.Context(small)
    dev = lp.state_to_device(st)
    with pytest.raises(lp.LpError) as e:
        ctx.autotune(dev, reps=1)
    assert e.value.status == lp.E_CAPACITY
    inf = ctx.info()
    assert inf["t"] == 0.0 and inf["error_bits"] == 0
    assert ctx.check() == lp.OK
    # a context that has already stepped keeps its own time and dt
    ctx2 = lp.Context(cfg)
    dev2 = lp.state_to_device(st)
    ctx2.step(dev2)
    ctx2.step(dev2)
    before = ctx2.info()
    ctx2.autotune(lp.state_to_device(st), reps=1)
    after = ctx2.info()
    assert after["t"] == before["t"] and after["dt"] == before["dt"] and after["error_bits"] == 0
    ctx2.run(dev2, 2)
    assert ctx2.check() == lp.OK
    assert ctx2.info()["t"] > before["t"]


def _run(lp, cfg, st, nsteps, precision="fp64", tuning=None, split=None):
    """lp_run over nsteps (in pieces of `split` steps if given); state and info."""
    ctx = lp.Context(cfg, precision=precision)
    for p, v in (tuning or {}).items():
        ctx.set_tuning(p, v)
    dev = lp.state_to_device(st)
    done = 0
    while done < nsteps:
        k = min(split or nsteps, nsteps - done)
        ctx.run(dev, k)
        done += k
    assert ctx.check() == lp.OK, lp.lib().lp_last_error(ctx._h)
    out, inf = lp.state_to_host(dev), ctx.info()
    ctx.close()
    return out, inf


@pytest.mark.parametrize("case", list(CASES))
@pytest.mark.parametrize("precision", ["fp64", "mixed"])
def test_list_reuse_identical(lp, case, precision):
    """Neighbour lists reused across steps (candidates within (1 + skin) r,
    filtered exactly every step) give the full search's results bit for bit,
    in graph-replayed runs and in eager steps; without mirror walls the
    candidate lists are rebuilt on fewer steps than there are steps."""
    cfg, st = CASES[case]()
    nsteps = 7  # the coarse vacuum cloud's lists outgrow 256 entries after 8 steps
    ref, rinf = _run(lp, cfg, st, nsteps, precision, {lp.TUNE_LIST_SKIN: 0})
    assert rinf["n_list_builds"] == 0
    for skin in (50, 150, 400):
        tag = "%s %s skin %d" % (case, precision, skin)
        got, inf = _run(lp, cfg, st, nsteps, precision, {lp.TUNE_LIST_SKIN: skin})
        say("list reuse", tag, "full searches:", inf["n_list_builds"], "of", nsteps, "steps")
        _same(got, ref, tag)
        if case == "sod slab":
            assert inf["n_list_builds"] == 0  # mirror walls: a full search every step
        elif skin <= 150:
            assert 1 <= inf["n_list_builds"] < nsteps
        else:
            # the coarse cloud's candidate lists within 1.4 r outgrow max_nb:
            # every step rebuilds, and the particles concerned are searched exactly
            assert 1 <= inf["n_list_builds"] <= nsteps
    got = _steps(lp, cfg, st, 4, precision, {lp.TUNE_LIST_SKIN: 150})
    _same(got, _steps(lp, cfg, st, 4, precision, {lp.TUNE_LIST_SKIN: 0}), "%s %s eager" % (case, precision))


def test_list_reuse_after_other_calls(lp):
    """A neighbour search, a derivative call and a run on other particles
    between steps of one context rebuild the candidate lists first."""
    cfg, st = CASES["vacuum 60k"]()
    ref, _ = _run(lp, cfg, st, 7, tuning={lp.TUNE_LIST_SKIN: 0})
    ctx = lp.Context(cfg)
    dev = lp.state_to_device(st)
    ctx.run(dev, 2)
    other = lp.state_to_device(W.vacuum3d(n_particles=30_000, seed=8)[1])
    ctx.run(other, 2)
    ctx.run(dev, 2)
    h = (dev["m"] * dev["V"]) ** (1.0 / 3.0) * cfg["kappa"]
    ctx.neighbors(dev["x"], h)
    ctx.gfd(dev["x"], h, [dev["V"], dev["P"]])
    ctx.run(dev, 3)
    assert ctx.check() == lp.OK
    _same(lp.state_to_host(dev), ref, "after other calls")
