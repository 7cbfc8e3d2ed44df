"""The estimator network on the GPU (BF16 matrix instructions, FP32
accumulation) against the FP64 oracle, the staged update path against the
plain one, and what a trained network gains on the Sod tube."""
import numpy as np
import pytest

from paper_2206_11998_amd import workloads as W
from tests import riemann
from tests.gpu_util import say

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

NP = 5313
OFF_W1, OFF_B1, OFF_W2, OFF_B2, OFF_W3, OFF_B3 = 0, 1024, 1088, 5184, 5248, 5312
BLOCKS = {"W1": (OFF_W1, OFF_B1), "b1": (OFF_B1, OFF_W2), "W2": (OFF_W2, OFF_B2), "b2": (OFF_B2, OFF_W3),
          "w3": (OFF_W3, OFF_B3), "b3": (OFF_B3, NP)}


@pytest.fixture(scope="module")
def lp():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2206_11998_amd import lp as _lp
    _lp.lib()
    return _lp


def bf16(a):
    """Round float values to bfloat16 (nearest even), returned as float64."""
    f = np.asarray(a, dtype=np.float32)
    u = f.view(np.uint32).astype(np.uint64)
    u = (u + 0x7FFF + ((u >> 16) & 1)) >> 16 << 16
    return u.astype(np.uint32).view(np.float32).astype(np.float64)


def _ctx(lp):
    cfg, _ = W.pulse2d()
    return lp.Context(cfg)


def test_forward_exact_on_integer_network(lp, oracle_lib):
    """Integer weights and inputs keep every product, sum and BF16 rounding
    exact, so the matrix-core forward pass must equal the oracle bit for bit:
    this pins the operand and accumulator layouts of all three layers."""
    rng = np.random.default_rng(11)
    th = rng.integers(-1, 2, NP).astype(np.float64)
    th[OFF_B1:OFF_W2] = rng.integers(-2, 3, 64)
    th[OFF_B3] = 1.0
    n = 16 * 37 + 5  # ragged last tile
    feat = rng.integers(-2, 3, (n, 16)).astype(np.float64)
    ctx = _ctx(lp)
    ctx.mlp_set(th.astype(np.float32))
    z, _ = ctx.mlp_forward(torch.from_numpy(feat.astype(np.float32)).cuda())
    zr, _ = oracle_lib.mlp_forward(th, feat)
    say("integer network: max |z| %.0f" % np.abs(zr).max())
    assert np.abs(zr).max() > 10  # the test exercises real sums
    assert np.array_equal(z.cpu().numpy().astype(np.float64), zr)


def test_forward_and_gradient_against_oracle(lp, oracle_lib):
    rng = np.random.default_rng(12)
    th = (rng.standard_normal(NP) * 0.2).astype(np.float32)
    n = 8000 + 9
    feat = rng.standard_normal((n, 16)).astype(np.float32)
    # one target for all samples: the per-sample gradients add up coherently,
    # so the rare ReLU masks that BF16 rounding of the hidden layer flips
    # (the oracle keeps it exact) stay small against the sum
    target = np.full(n, 0.05, dtype=np.float32)
    ctx = _ctx(lp)
    ctx.mlp_set(th)
    fd = torch.from_numpy(feat).cuda()
    td = torch.from_numpy(target).cuda()
    z, y = ctx.mlp_forward(fd)
    loss, g = ctx.mlp_grad(fd, td)
    # the oracle on the same BF16-rounded weights and inputs, in FP64
    thr = bf16(th)
    for name in ("b1", "b2", "w3", "b3"):  # kept in FP32 on the device
        a, b = BLOCKS[name]
        thr[a:b] = th[a:b]
    zr, yr = oracle_lib.mlp_forward(thr, bf16(feat))
    lr, gr = oracle_lib.mlp_loss_grad(thr, bf16(feat), target.astype(np.float64))
    ez = np.linalg.norm(z.cpu().numpy() - zr) / np.linalg.norm(zr)
    say("forward rel. L2 %.2e, loss %.6f vs %.6f" % (ez, loss, lr))
    assert ez <= 2e-2
    assert np.allclose(y.cpu().numpy(), yr, atol=5e-3)
    assert abs(loss - lr) <= 2e-3 * abs(lr)
    for name, (a, b) in BLOCKS.items():
        e = np.linalg.norm(g[a:b] - gr[a:b]) / max(np.linalg.norm(gr[a:b]), 1e-30)
        say("gradient %s rel. L2 %.2e" % (name, e))
        assert e <= 2e-2, name


def test_features_against_oracle(lp, oracle_lib):
    for tag, (cfg, st) in (("sod slab", W.sod3d(n=64, ny=8, nz=8)), ("pulse2d", W.pulse2d()),
                           ("vacuum 40k", W.vacuum3d(n_particles=40_000, seed=7))):
        say("features", tag)
        ctx = lp.Context(cfg)
        dev = lp.state_to_device(st)
        feat, phi, valid = ctx.features(dev)
        n = st["V"].shape[0]
        ref, info = oracle_lib.step_subset(cfg, st, np.arange(n), features=True)
        f = feat.cpu().numpy().astype(np.float64)
        rf = ref["feat"].astype(np.float32).astype(np.float64)
        close = np.all(np.abs(f - rf) <= 1e-5 * (1.0 + np.abs(rf)), axis=1)
        say(tag, "particles with all features within 1e-5: %.5f" % close.mean(),
            "mean |dphi| %.2e" % np.abs(phi.cpu().numpy() - ref["phi"]).mean())
        assert close.mean() >= 0.999
        assert np.abs(phi.cpu().numpy() - ref["phi"]).mean() <= 1e-4
        assert np.array_equal(valid.cpu().numpy() == 0, (ref["flags"] & 6) != 0)
        # nothing advanced: the state is untouched
        back = lp.state_to_host(dev)
        assert np.array_equal(back["V"], st["V"]) and np.array_equal(back["x"], st["x"])


def _run(lp, cfg, st, nsteps, estimator="plain", phi=None, params=None):
    ctx = lp.Context(cfg, estimator=estimator)
    if params is not None:
        ctx.mlp_set(params)
    dev = lp.state_to_device(st)
    if phi is not None:
        dev["phi"].fill_(phi)
    for _ in range(nsteps):
        ctx.step(dev)
        if phi is not None:
            dev["phi"].fill_(phi)
    assert ctx.check() == lp.OK
    info = ctx.info()
    out = lp.state_to_host(dev)
    ctx.close()
    return out, info


def test_staged_update_matches_plain_paths(lp):
    """A network saturated at phi = 1 gives the injected phi = 1 step; a network
    that is never trusted (output 1/2) gives the quotient estimator's step."""
    cfg, st = W.pulse2d()
    sat = np.zeros(NP, dtype=np.float32)
    sat[OFF_B3] = 30.0
    a, ia = _run(lp, cfg, st, 4, "mlp", params=sat)
    b, _ = _run(lp, cfg, st, 4, "injected", phi=1.0)
    for k in ("x", "V", "u", "P"):
        assert np.array_equal(a[k], b[k]), k
    assert ia["n_mlp"] == st["V"].shape[0]
    half = np.zeros(NP, dtype=np.float32)
    half[OFF_B3] = np.log(0.4 / 0.6)  # 1.25 sigmoid = 1/2: never trusted
    c, ic = _run(lp, cfg, st, 4, "mlp", params=half)
    d, _ = _run(lp, cfg, st, 4, "plain")
    for k in ("x", "V", "u", "P", "phi", "flags"):
        assert np.array_equal(c[k], d[k]), k
    assert ic["n_mlp"] == 0 and ic["n_mlp_plain"] == st["V"].shape[0]


def _sod_error(s, T=0.1):
    x = s["x"][:, 0]
    ex = riemann.sample(x, T, 0.5, 1.0, 0.0, 1.0, 0.125, 0.0, 0.1)
    return np.mean(np.abs(1.0 / s["V"] - ex[:, 0])), np.mean(np.abs(s["P"] - ex[:, 2]))


def _sod_run(lp, cfg, st, T, estimator="plain", phi=None, params=None, harvest=None):
    ctx = lp.Context(cfg, estimator=estimator)
    if params is not None:
        ctx.mlp_set(params)
    dev = lp.state_to_device(st)
    hctx = lp.Context(cfg) if harvest is not None else None
    while ctx.info()["t"] < T:
        if harvest is not None:
            f, p, v = hctx.features(dev)
            keep = v.bool()
            harvest.append((f[keep].clone(), p[keep].clone()))
        if phi is not None:
            dev["phi"].fill_(phi)
        try:
            ctx.run(dev, 1, T)  # one step, clipped to T
        except lp.LpError:
            break
        if ctx.check() != lp.OK:
            break
    status = ctx.check()
    ok = status == lp.OK and ctx.info()["t"] >= T
    out = lp.state_to_host(dev)
    info = ctx.info()
    ctx.close()
    return out, info, ok


def _steps_harvest(lp, cfg, st, nsteps, harvest):
    ctx = lp.Context(cfg)
    dev = lp.state_to_device(st)
    for _ in range(nsteps):
        f, p, v = ctx.features(dev)
        keep = v.bool()
        harvest.append((f[keep].clone(), p[keep].clone()))
        ctx.step(dev)
    assert ctx.check() == lp.OK
    ctx.close()


def test_trained_network_on_sod(lp):
    """Harvest (inputs, quotient-estimator phi) from Sod tubes, train the
    network on the GPU, and run a Sod tube it has not seen with the network
    as the estimator: it must decide most particles, track the quotient
    estimator's error against the exact solution, and beat the scheme without
    an estimator (phi = 1 everywhere)."""
    T = 0.1
    harvest = []
    for seed in (21, 22):
        cfg, st = W.sod3d(n=128, ny=8, nz=8, seed=seed)
        assert _sod_run(lp, cfg, st, T, harvest=harvest)[2]
    # smooth flow too, where the quotient estimator keeps phi = 1
    wcfg, wst = W.smooth_wave(3, 20, seed=31, amp=3e-2)
    _steps_harvest(lp, wcfg, wst, 12, harvest)
    feat = torch.cat([h[0] for h in harvest])
    phi = torch.cat([h[1] for h in harvest])
    lim = phi < 1.0
    gen = torch.Generator().manual_seed(5)
    ia = torch.nonzero(lim).flatten().cpu()
    ib = torch.nonzero(~lim).flatten().cpu()
    m = min(len(ia), len(ib))
    sel = torch.cat([ia[torch.randperm(len(ia), generator=gen)[:m]], ib[torch.randperm(len(ib), generator=gen)[:m]]])
    sel = sel[torch.randperm(len(sel), generator=gen)].cuda()
    fx = feat[sel].contiguous()
    tx = (phi[sel] / 1.25).contiguous()  # the estimator uses min(1, 1.25 sigmoid)
    say("training samples %d (limited %d of %d harvested)" % (len(sel), len(ia), len(phi)))
    cfg, st = W.sod3d(n=128, ny=8, nz=8, seed=23)
    ctx = lp.Context(cfg)
    ctx.mlp_init(7)
    loss0 = ctx.mlp_grad(fx, tx)[0]
    losses = ctx.mlp_train(fx, tx, epochs=40, batch=2048, lr=3e-3)
    # cross-entropy against soft targets cannot go below their entropy
    t = tx.double().cpu().numpy()
    tc = np.clip(t, 1e-12, 1 - 1e-12)
    floor = float(np.mean(-(t * np.log(tc) + (1 - t) * np.log(1 - tc))))
    say("loss: untrained %.4f, by epoch %s, floor %.4f" % (loss0, np.round(losses[[0, 4, 9, 19, 39]], 4), floor))
    assert losses[-1] - floor < 0.2 * (loss0 - floor)
    params = ctx.mlp_get()
    _, y = ctx.mlp_forward(fx)
    agree = (torch.abs(torch.clamp(1.25 * y, max=1.0) - 1.25 * tx) < 0.1).float().mean().item()
    say("training samples within 0.1 of the quotient estimator: %.3f" % agree)
    assert agree > 0.8
    # a tube the network has not seen
    res = {}
    for name, kw in (("plain", {}), ("mlp", {"estimator": "mlp", "params": params}),
                     ("no estimator (phi=1)", {"estimator": "injected", "phi": 1.0}),
                     ("upwind only (phi=0)", {"estimator": "injected", "phi": 0.0})):
        out, info, ok = _sod_run(lp, cfg, st, T, **kw)
        res[name] = (_sod_error(out) if ok else (np.inf, np.inf), info, ok)
        say("%-22s reached t=%.3f %s  L1 rho %.5f  L1 p %.5f  network decided %d, fell back %d" % (
            name, info["t"], "ok" if ok else "BROKE DOWN", res[name][0][0], res[name][0][1], info["n_mlp"],
            info["n_mlp_plain"]))
    e_plain, e_mlp = res["plain"][0], res["mlp"][0]
    e_lw, e_uw = res["no estimator (phi=1)"][0], res["upwind only (phi=0)"][0]
    info = res["mlp"][1]
    n = st["V"].shape[0]
    assert res["plain"][2] and res["mlp"][2]
    assert info["n_mlp"] > 0.5 * n
    # the gain over the scheme without an estimator: on the Sod tube that one
    # breaks down (or ends farther from the exact solution); the network ends
    # as close to it as the quotient estimator and pure upwind do
    assert e_mlp[0] < e_lw[0] and e_mlp[1] < e_lw[1]
    assert e_mlp[0] <= 1.01 * e_uw[0] and e_mlp[1] <= 1.01 * e_uw[1]
    assert e_mlp[0] <= 1.15 * e_plain[0] and e_mlp[1] <= 1.15 * e_plain[1]
    # on a smooth wave it has not seen, it keeps the second-order update where
    # the quotient estimator does (pure upwind damps the wave)
    wcfg, wst = W.smooth_wave(3, 20, seed=37, amp=3e-2)
    waves = {}
    for name, kw in (("plain", {}), ("mlp", {"estimator": "mlp", "params": params}),
                     ("upwind only (phi=0)", {"estimator": "injected", "phi": 0.0})):
        waves[name] = _run(lp, wcfg, wst, 12, **kw)
    d_mlp = np.abs(waves["mlp"][0]["P"] - waves["plain"][0]["P"]).sum()
    d_uw = np.abs(waves["upwind only (phi=0)"][0]["P"] - waves["plain"][0]["P"]).sum()
    say("smooth wave: L1 distance of P to the quotient estimator's run: network %.3e, pure upwind %.3e; "
        "network decided %d of %d" % (d_mlp, d_uw, waves["mlp"][1]["n_mlp"], wst["V"].shape[0]))
    assert d_mlp < 0.25 * d_uw


def _accuracy_harvest(lp, oracle_lib, cfg, st, exact, T, out):
    """Inputs and accuracy labels of every step of the quotient-estimator run
    to T: at each state, one step with phi = 0 and one with phi = 1 from it
    (same dt), scored against the exact state at the end of the step.  The
    label is 1 where the Lax-Wendroff result lands closer (in the scaled
    squared error over V, u, P) than the upwind one, i.e. where the
    least-squares blend weight of tests/gpu_util.accuracy_phi exceeds 1/2,
    else 0."""
    from tests.gpu_util import accuracy_phi

    def clone(dev):
        return {k: ([t.clone() for t in v] if isinstance(v, list) else v.clone()) for k, v in dev.items()}

    ctx = lp.Context(cfg)
    dev = lp.state_to_device(st)
    V_s, P_s = st["V"].mean(), st["P"].mean()
    u_s = np.sqrt(cfg["gamma"] * st["P"] * st["V"]).max()
    t = 0.0
    while t < T - 1e-12:
        f, _, v = ctx.features(dev)
        host = lp.state_to_host(dev)
        dt = min(oracle_lib.timestep(cfg, {q: host[q] for q in ("x", "u", "V", "P", "m")}), T - t)
        ends = []
        for phi in (0.0, 1.0):
            c = lp.Context(cfg, estimator="injected")
            d = clone(dev)
            d["phi"].fill_(phi)
            c.step(d, dt)
            assert c.check() == lp.OK
            ends.append(lp.state_to_host(d))
            c.close()
        rho, u, p = exact(0.5 * (ends[0]["x"] + ends[1]["x"]), t + dt)
        phi_star, _ = accuracy_phi(ends[0], ends[1], 1.0 / rho, u, p, V_s, u_s, P_s)
        keep = (v.cpu().numpy() != 0) & np.isfinite(phi_star)
        idx = torch.from_numpy(np.flatnonzero(keep)).cuda()
        label = (phi_star[keep] > 0.5).astype(np.float32)
        out.append((f[idx].clone(), torch.from_numpy(label).cuda()))
        ctx.step(dev, dt)
        assert ctx.check() == lp.OK
        t += dt
    ctx.close()


def _sod_exact(x, t):
    ex = riemann.sample(x[:, 0], t, 0.5, 1.0, 0.0, 1.0, 0.125, 0.0, 0.1)
    u = np.zeros((len(x), 3))
    u[:, 0] = ex[:, 1]
    return ex[:, 0], u, ex[:, 2]


def _yee_l2(lp, oracle_lib, dx, T, **kw):
    """L2 (RMS) errors of P and |u| of the Yee vortex at T against the exact
    solution, steps as the oracle's timestep gives them."""
    cfg, st = W.yee_vortex(dx)
    ctx = lp.Context(cfg, estimator=kw.get("estimator", "plain"))
    if kw.get("params") is not None:
        ctx.mlp_set(kw["params"])
    dev = lp.state_to_device(st)
    t, n_mlp = 0.0, 0
    while t < T - 1e-12:
        host = lp.state_to_host(dev)
        d = min(oracle_lib.timestep(cfg, {q: host[q] for q in ("x", "u", "V", "P", "m")}), T - t)
        if kw.get("phi") is not None:
            dev["phi"].fill_(kw["phi"])
        ctx.step(dev, d)
        assert ctx.check() == lp.OK
        n_mlp += ctx.info()["n_mlp"]
        t += d
    s = lp.state_to_host(dev)
    ctx.close()
    rho, u, p = W.yee_exact(s["x"], T)
    eu = np.sqrt(((s["u"] - u) ** 2).sum(axis=1))
    return np.sqrt(((s["P"] - p) ** 2).mean()), np.sqrt((eu ** 2).mean()), n_mlp


_ACC = {}


def _accuracy_network(lp, oracle_lib):
    """Parameters of the network trained on accuracy labels (harvest and
    training as the test below describes; once per module)."""
    if "params" in _ACC:
        return _ACC["params"]
    harvest = []
    for seed in (21, 22):
        cfg, st = W.sod3d(n=128, ny=8, nz=8, seed=seed)
        _accuracy_harvest(lp, oracle_lib, cfg, st, _sod_exact, 0.1, harvest)
    n_sod = sum(len(h[1]) for h in harvest)
    for dx, seed in ((0.25, 3), (0.3, 4)):
        cfg, st = W.yee_vortex(dx, jitter=0.1, seed=seed)
        _accuracy_harvest(lp, oracle_lib, cfg, st, W.yee_exact, 2.0, harvest)
    feat = torch.cat([h[0] for h in harvest])
    target = torch.cat([h[1] for h in harvest])
    say("accuracy labels: %d Sod, %d Yee; Lax-Wendroff closer for %.3f" % (n_sod, len(target) - n_sod,
                                                                      target.mean().item()))
    # the Yee samples whole, the Sod samples thinned to four times as many
    gen = torch.Generator().manual_seed(5)
    n_yee = len(target) - n_sod
    pick = torch.randperm(n_sod, generator=gen)[:min(4 * n_yee, n_sod)]
    sel = torch.cat([pick, torch.arange(n_sod, len(target))])
    sel = sel[torch.randperm(len(sel), generator=gen)].cuda()
    # targets 0 / 1: the network's output is the probability that the
    # Lax-Wendroff update lands closer, and phi = min(1, 1.25 y) takes the
    # full Lax-Wendroff update from a probability of 0.8 on
    fx, tx = feat[sel].contiguous(), target[sel].contiguous()
    cfg, _ = W.sod3d(n=128, ny=8, nz=8, seed=23)
    ctx = lp.Context(cfg)
    ctx.mlp_init(7)
    losses = ctx.mlp_train(fx, tx, epochs=40, batch=2048, lr=3e-3)
    say("loss by epoch", np.round(losses[[0, 9, 19, 39]], 4))
    assert losses[-1] < losses[0]
    _ACC["params"] = ctx.mlp_get()
    ctx.close()
    return _ACC["params"]


def test_network_trained_on_accuracy_targets(lp, oracle_lib):
    """The network trained to reproduce accuracy, not the quotient estimator:
    its targets say which pure update (upwind or Lax-Wendroff) brings each
    step closer to the exact solution, harvested along Sod tubes (seeds 21, 22)
    and jittered Yee vortices at dx 0.25 and 0.3.  On resolutions and tubes
    it has not seen, it must beat the quotient estimator's L2 error of P and
    u on the Yee vortex at dx 0.2 (t = 8) and stay within 1.15x of its L1
    error of rho and P on a Sod tube (seed 23, t = 0.1), deciding most
    particles itself."""
    params = _accuracy_network(lp, oracle_lib)
    cfg, st = W.sod3d(n=128, ny=8, nz=8, seed=23)
    sod = {}
    for name, kw in (("plain", {}), ("mlp", {"estimator": "mlp", "params": params})):
        out, info, ok = _sod_run(lp, cfg, st, 0.1, **kw)
        assert ok, name
        sod[name] = (_sod_error(out), info)
        say("unseen Sod, %-5s L1 rho %.5f  L1 p %.5f  network decided %d" % (
            name, sod[name][0][0], sod[name][0][1], info["n_mlp"]))
    assert sod["mlp"][1]["n_mlp"] > 0.5 * st["V"].shape[0]
    assert sod["mlp"][0][0] <= 1.15 * sod["plain"][0][0] and sod["mlp"][0][1] <= 1.15 * sod["plain"][0][1]
    yee = {}
    for name, kw in (("plain", {}), ("mlp", {"estimator": "mlp", "params": params}),
                     ("phi=1", {"estimator": "injected", "phi": 1.0})):
        yee[name] = _yee_l2(lp, oracle_lib, 0.2, 8.0, **kw)
        say("Yee dx 0.2, t = 8, %-5s L2 P %.5f  L2 u %.5f  network decisions %d" % ((name,) + yee[name]))
    assert yee["mlp"][0] < 0.5 * yee["plain"][0] and yee["mlp"][1] < 0.5 * yee["plain"][1]
    assert yee["mlp"][2] > 0


def test_sedov_blast_with_the_accuracy_network(lp, oracle_lib):
    """The blast (64 x 32 x 32, Gaussian deposit) with the network trained on
    accuracy labels as the estimator: 50 graph-replayed mixed steps with every
    V and P positive, mass unchanged, the network deciding most particles,
    and the densest particle's radius within 15% of the self-similar blast
    radius, as the oracle's quotient-estimator run is pinned."""
    params = _accuracy_network(lp, oracle_lib)
    cfg, st = W.sedov3d(nx=64)
    h = 2.0 / 64
    xc = np.array([32.5, 16.5, 16.5]) * h
    for name, kw in (("quotient", {}), ("network", {"estimator": "mlp"})):
        ctx = lp.Context(cfg, precision="mixed", refine_cond=1e3, **kw)
        if name == "network":
            ctx.mlp_set(params)
        dev = lp.state_to_device(st)
        m0 = ctx.conservation(dev)[0]
        n_mlp = 0
        for _ in range(5):
            ctx.run(dev, 10)
            assert ctx.check() == lp.OK, (name, lp.lib().lp_last_error(ctx._h))
            n_mlp += ctx.info()["n_mlp"]
        info = ctx.info()
        out = lp.state_to_host(dev)
        r = np.sqrt(((out["x"] - xc) ** 2).sum(axis=1))
        R, R0 = r[np.argmax(1.0 / out["V"])], W.sedov_radius(info["t"])
        say("sedov 64x32x32, %-8s t %.4f: radius of the densest particle %.4f, self-similar %.4f; "
            "limited %d, network decisions in the last step of each run: %d" % (name, info["t"], R, R0,
                                                                               info["n_limited"], n_mlp))
        assert ctx.conservation(dev)[0] == m0
        assert out["P"].min() > 0.0 and out["V"].min() > 0.0
        assert R0 > 4 * h and abs(R / R0 - 1.0) < 0.15, name
        if name == "network":
            assert info["n_mlp"] > 0.5 * st["V"].shape[0]
        ctx.close()
