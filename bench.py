"""Throughput of the LP time step on one MI355X.

Workload: the 3D expansion into vacuum -- 2,097,152 equal-mass particles
rejection-sampled from rho = exp(-|x|^2/0.05) (spacing varies 8x), kappa 2.2,
CFL 0.2, free boundary -- one time step = neighbour search + GFD fits + blended
update + mover for every particle.  Prints one JSON line: particle-updates/s of
the mixed-precision step (FP32 fits, one FP64-residual refinement step for the
fits whose condition estimate exceeds --refine-cond, FP64 for ill-conditioned
stencils and the state), the FP64 step, the mixed step refining every fit, the
FP32 step without refinement and the learned-estimator step next to it, the
relative L1 error of each against the CPU reference, the roofline of the
dominant kernel (timed with HIP events on the library's stream) and the CPU
reference's own throughput on the host cores.
"""
import argparse
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "particle-updates/s at 2M particles, mixed vs FP64 step; L1 err vs oracle"
PEAK_ALU_TFLOPS = 78.6   # 256 CU x 4 SIMD x 16 lanes x 2 flop x 2.4 GHz (FP64, and FP32 without packed math)
PEAK_HBM_GBS = 8000.0
PEAK_BF16_TFLOPS = 2500.0  # dense BF16 matrix-core peak
MLP_FLOPS = 20 * 16 * 16 * 16 * 2 / 16.0  # 20 MFMA 16x16x16 per tile of 16 particles


def fit_flops(k_lw, dim=3):
    """Algorithmic flops of one particle's second-order least-squares fit over a
    stencil of k_lw rows: row assembly 20k, Householder factorisation
    2kn^2 - 2n^3/3 and R right-hand sides R(4kn - 2n^2) + Rn^2 (n unknowns)."""
    n, R = (9, 5) if dim == 3 else (5, 4)
    k = np.asarray(k_lw, dtype=np.float64)
    return 20 * k + 2 * k * n * n - 2.0 * n ** 3 / 3 + R * (4 * k * n - 2 * n * n) + R * n * n


def gfd3_flops(k_lw, dim=3):
    """Algorithmic flops of one particle's third-order least-squares fit
    (lp_gfd3) over k_lw rows: row assembly 40k, Householder factorisation
    2kn^2 - 2n^3/3 and R right-hand sides R(4kn - 2n^2) + Rn^2, n = 19 (3D) or
    9 (2D) unknowns, R = 5 fields."""
    n, R = (19, 5) if dim == 3 else (9, 4)
    k = np.asarray(k_lw, dtype=np.float64)
    return 40 * k + 2 * k * n * n - 2.0 * n ** 3 / 3 + R * (4 * k * n - 2 * n * n) + R * n * n


def update_flops(dim=3):
    """Half-ball fits (2D fits of 8 rows, D unknowns, 3 right-hand sides) plus
    estimator, rates, blend and mover."""
    return (2800.0 if dim == 3 else 1200.0) + 300.0


def cells_bytes(n):
    """Algorithmic HBM bytes of the prep and cell stages per particle: read
    x, V, m (40 B), write h, r (16 B); Morton key and slot (8 B written, 8 B
    read back); the cell-order scatter reads 10 FP64 values and writes them
    with the 64-byte gather record (80 + 80 + 64 B)."""
    return float(n) * (40 + 16 + 16 + 80 + 80 + 64)


def search_bytes(count):
    """Algorithmic HBM bytes of the neighbour search: read position, radius and
    id of every particle once (36 B), write its list and count (4k + 4 B)."""
    k = np.asarray(count, dtype=np.float64)
    return 40.0 + 4.0 * k


def cpu_model():
    """The host CPU's model name (from /proc/cpuinfo), or None."""
    try:
        with open("/proc/cpuinfo") as fh:
            for line in fh:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return None


def source_hash():
    """Hash of the device sources (every file of csrc/ but lp_api.hip, the
    host-only entry points): HBM counters committed under profiles/ are only
    reported while the kernels they were taken on are unchanged."""
    import hashlib
    h = hashlib.sha256()
    src = os.path.join(ROOT, "paper_2206_11998_amd", "csrc")
    for f in sorted(os.listdir(src)):
        if f == "lp_api.hip":
            continue
        with open(os.path.join(src, f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()[:16]


def committed_traffic(kernel, precision):
    """HBM bytes per launch (FETCH_SIZE + WRITE_SIZE, copy-calibrated) of the
    search / fit / update kernel, from the rocprofv3 counter summary of the
    same workload and precision in profiles/; None when there is none or it
    was taken on other kernel sources."""
    path = os.path.join(ROOT, "profiles", "vacuum3d_2M_%s_step_traffic.json" % precision)
    if not os.path.exists(path):
        return None
    with open(path) as fh:
        d = json.load(fh)
    if d.get("source_hash") != source_hash() or kernel not in d.get("kernels", {}):
        return None
    v = d["kernels"][kernel]
    return v["read_bytes"] + v["written_bytes"]


def gfd3_leg(lp, torch, cfg, st, log, no_cpu):
    """lp_gfd3 (third-order derivatives of V, u, P) on the workload's particles:
    the fit kernel timed by the library's stage events over 3 calls, its FP64
    ALU roofline, and the oracle's third-order operator on the central
    particles beside it (on that sample the GPU result is compared too)."""
    n = st["V"].shape[0]
    h = (st["m"] * st["V"]) ** (1.0 / 3.0)
    r_np = cfg["kappa"] * h
    fields_np = [st["V"], st["u"][:, 0], st["u"][:, 1], st["u"][:, 2], st["P"]]

    def dev(a):
        return torch.from_numpy(np.ascontiguousarray(a, dtype=np.float64)).cuda()

    ctx = lp.Context(cfg)
    x = [dev(st["x"][:, a]) for a in range(3)]
    r = dev(r_np)
    f = [dev(v) for v in fields_np]
    ctx.gfd3(x, r, f)  # warm-up (workspace, tables)
    torch.cuda.synchronize()
    calls = 3
    ctx.profile(True)
    t1 = time.perf_counter()
    for _ in range(calls):
        deriv, status = ctx.gfd3(x, r, f)
    torch.cuda.synchronize()
    wall = (time.perf_counter() - t1) / calls
    prof = ctx.profile_read()
    ctx.profile(False)
    count, _, _ = ctx.neighbors(x, r)
    k_lw = np.minimum(count.cpu().numpy(), 54)
    flops = float(gfd3_flops(k_lw).sum())
    fit_ms = prof["fit"][0] / max(prof["fit"][1], 1)
    stat = np.bincount(status.cpu().numpy(), minlength=4)
    achieved = flops / (fit_ms * 1e-3) / 1e12
    res = {"particles": n, "fields": 5, "calls": calls, "ms_per_call": wall * 1e3,
           "stages_ms_per_call": {k: v[0] / max(v[1], 1) for k, v in prof.items() if v[1]},
           "status_counts": {"cubic": int(stat[0]), "quadratic": int(stat[1]), "linear": int(stat[2]),
                             "none": int(stat[3])},
           "mean_stencil": float(k_lw.mean()),
           "roofline": {"bound": "alu", "achieved": achieved, "peak": PEAK_ALU_TFLOPS, "unit": "TFLOP/s",
                        "frac": achieved / PEAK_ALU_TFLOPS, "traffic": committed_traffic("gfd3", "mixed"),
                        "algorithmic_flops_per_launch": flops, "avg_launch_ms": fit_ms,
                        "kernel": "k_gfd3 (third-order fits)"},
           "cpu_baseline": None}
    del deriv, status
    log("gfd3: %.2f ms per call (fit kernel %.2f ms), %.3f TFLOP/s" % (wall * 1e3, fit_ms, achieved))
    if not no_cpu:
        try:
            import oracle
            # the particles of a central cube, about 200k of them, repeated
            # until 3 s of CPU time have elapsed (at most 8 times)
            xs = st["x"]
            half = np.sort(np.abs(xs).max(axis=1))[min(200_000, n) - 1]
            sel = np.flatnonzero(np.abs(xs).max(axis=1) <= half)
            xs_s, r_s = xs[sel], r_np[sel]
            f_s = [v[sel] for v in fields_np]
            reps, cpu_total = 0, 0.0
            while reps == 0 or (cpu_total < 3.0 and reps < 8):
                t1 = time.perf_counter()
                ref, rst, rs = oracle.gfd3(cfg, xs_s, r_s, f_s)
                cpu_total += time.perf_counter() - t1
                reps += 1
            cpu_t = cpu_total / reps
            got, gst = ctx.gfd3([dev(xs_s[:, a]) for a in range(3)], dev(r_s), [dev(v) for v in f_s])
            got, gst = got.cpu().numpy(), gst.cpu().numpy()
            worst = 0.0
            for q in range(ref.shape[0]):
                for c in range(ref.shape[1]):
                    worst = max(worst, float(np.abs(got[q, c] - ref[q, c]).sum() / max(np.abs(ref[q, c]).sum(),
                                                                                       1e-300)))
            res["cpu_baseline"] = {"value": len(sel) / cpu_t, "unit": "particles/s", "cores": oracle.num_threads(),
                                   "kind": "oracle",
                                   "sample": "lp_gfd3 of the %d particles with |x|_inf <= %.4f (their neighbourhoods "
                                             "limited to the sample), mean of %d calls" % (len(sel), half, reps)}
            res["sample_parity"] = {"status_equal": bool(np.array_equal(gst, rst)),
                                    "max_column_rel_l1": worst}
            log("gfd3 oracle: %d particles in %.2fs; sample parity %s" % (len(sel), cpu_t, res["sample_parity"]))
        except Exception as exc:
            log("gfd3 oracle unavailable:", repr(exc))
    ctx.close()
    return res


def openbc_leg(lp, torch, cfg, st, log, no_cpu):
    """lp_outflow on the workload's particles with the x-high face moved to 0
    (an outflow face through the middle of the cloud; about half the
    particles leave), lp_reservoir_inflow at that face, and lp_inflow_layer
    of a 256 x 256 layer with that state after the kept particles.  The
    compaction's algorithmic HBM bytes: every per-particle array read once
    (x, u, V, P, m: 72 B; phi, flags: 5 B) and the kept part written once."""
    n = st["V"].shape[0]
    ocfg = dict(cfg, box_hi=[0.0] + list(cfg["box_hi"][1:]))
    ctx = lp.Context(ocfg)
    src = lp.state_to_device(st)
    dev = {k: ([t.clone() for t in v] if isinstance(v, list) else v.clone()) for k, v in src.items()}
    ctx.outflow(dev, 0, 1)  # warm-up (workspace)
    times, kept = [], 0
    for _ in range(5):
        for k, v in src.items():
            if isinstance(v, list):
                for a, t in enumerate(v):
                    dev[k][a].copy_(t)
            else:
                dev[k].copy_(v)
        torch.cuda.synchronize()
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record()
        kept = ctx.outflow(dev, 0, 1)
        e1.record()
        torch.cuda.synchronize()
        times.append(e0.elapsed_time(e1))
    ms = float(np.median(times))
    per = 72.0 + 5.0
    alg = per * n + per * kept
    achieved = alg / (ms * 1e-3) / 1e9
    res = {"particles": n, "kept": int(kept), "outflow_ms": ms,
           "roofline": {"bound": "hbm", "achieved": achieved, "peak": PEAK_HBM_GBS, "unit": "GB/s",
                        "frac": achieved / PEAK_HBM_GBS, "traffic": None, "algorithmic_bytes_per_call": alg,
                        "note": "one call: keep flags, scan, one sync, one gather and one copy back over all arrays"}}
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record()
    inflow = ctx.reservoir_inflow(src, 0, 1, 0.02, 2.0, 1.5)  # the layer -0.02 < x <= 0 of the moved face
    e1.record()
    torch.cuda.synchronize()
    res["reservoir_inflow"] = {"ms": e0.elapsed_time(e1), "p_in": float(inflow[0]), "rho_in": float(inflow[1]),
                               "u_in": float(inflow[2]), "averaged": int(inflow[3])}
    # one 256 x 256 lattice layer with that state, appended after the kept particles (77 B written each)
    cap = int(kept) + 256 * 256
    h = (cfg["box_hi"][1] - cfg["box_lo"][1]) / 256
    args = (0, 0, h, 0.5 * h, float(inflow[1]), float(inflow[0]), float(inflow[2]))
    ctx.inflow_layer(dev, kept, *args)  # warm-up
    lt = []
    for _ in range(5):
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record()
        n_new = ctx.inflow_layer({k: ([t[:cap] for t in v] if isinstance(v, list) else v[:cap])
                                  for k, v in dev.items()}, kept, *args)
        e1.record()
        torch.cuda.synchronize()
        lt.append(e0.elapsed_time(e1))
    lms = float(np.median(lt))
    res["inflow_layer"] = {"particles": int(n_new - kept), "ms": lms,
                           "achieved_gbs": 77.0 * (n_new - kept) / (lms * 1e-3) / 1e9}
    log("outflow: %d of %d kept in %.3f ms (%.0f GB/s algorithmic); inflow layer of %d in %.3f ms"
        % (kept, n, ms, achieved, n_new - kept, lms))
    res["run_open"] = run_open_leg(lp, torch, cfg, st, log)
    if not no_cpu:
        try:
            import oracle
            t1 = time.perf_counter()
            ref = oracle.outflow(ocfg, st, 0, 1)
            cpu_t = time.perf_counter() - t1
            res["cpu_baseline"] = {"value": n / cpu_t, "unit": "particles/s", "cores": 1, "kind": "oracle",
                                   "sample": "lp_outflow of all %d particles, one call (single-threaded loop)" % n}
            res["parity"] = {"kept_equal": len(ref["V"]) == kept}
        except Exception as exc:
            log("open-boundary oracle unavailable:", repr(exc))
    ctx.close()
    return res


def run_open_leg(lp, torch, cfg, st, log, steps=20):
    """lp_run_open on the workload with an outflow face at x = 0.2 (a cap of
    the cloud leaves in the first step, then what the expansion carries across
    the face every step): the mixed step with the deletions inside the
    graph-replayed steps and the compaction at the end of the call.  Timed:
    one call of `steps` steps (its planning step, capture and compaction
    included) after a one-step call that removes the cap."""
    n = st["V"].shape[0]
    cap = n + 65536
    full = {"x": np.zeros((cap, 3)), "u": np.zeros((cap, 3)), "V": np.ones(cap), "P": np.ones(cap),
            "m": np.zeros(cap)}
    for k in full:
        full[k][:n] = st[k]
    ocfg = dict(cfg, box_hi=[0.2] + list(cfg["box_hi"][1:]))
    ctx = lp.Context(ocfg, precision="mixed", refine_cond=1e3)
    dev = lp.state_to_device(full)
    n1 = ctx.run_open(dev, n, 1, out_hi_mask=1)
    i0 = ctx.info()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    n2 = ctx.run_open(dev, n1, steps, out_hi_mask=1)
    torch.cuda.synchronize()
    ms = (time.perf_counter() - t0) * 1e3
    i1 = ctx.info()
    status = ctx.check()
    ctx.close()
    out = {"steps": steps, "ms_per_step": ms / steps, "n_before": int(n1), "n_after": int(n2),
           "captures": int(i1["n_captures"] - i0["n_captures"]),
           "list_builds": int(i1["n_list_builds"] - i0["n_list_builds"]), "status": int(status),
           "note": "outflow face x >= 0.2 inside lp_run_open (mixed, refine_cond 1e3); one call, planning "
                   "step and final compaction included"}
    log("lp_run_open: %d steps in %.2f ms (%.3f ms/step), %d -> %d particles, %d capture(s), %d list builds"
        % (steps, ms, ms / steps, n1, n2, out["captures"], out["list_builds"]))
    return out


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20, help="timed steps (lp_run: graph-replayed steps)")
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--n", type=int, default=2_097_152)
    ap.add_argument("--precision", choices=["both", "all", "mixed", "mixed_all", "fp64", "fp32", "mlp"],
                    default="all",
                    help="mixed: FP32 fits, the FP64-residual refinement step where the condition estimate "
                         "exceeds --refine-cond; mixed_all: the refinement step for every fit; fp32: no "
                         "refinement; mlp: mixed with the learned estimator (trained first, untimed); "
                         "both: mixed then fp64; all: mixed, fp64, mixed_all, fp32, mlp")
    ap.add_argument("--refine-cond", type=float, default=1e3,
                    help="condition-estimate threshold of the refinement step (mixed, mlp); the estimate "
                         "bounds cond(A)^2, so unrefined fits carry a relative error of at most about "
                         "refine_cond * 2^-24")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--sample", type=int, default=0, help="particles in the CPU-reference sample (0: all)")
    ap.add_argument("--search-mode", type=int, default=None, help="override the neighbour-search mode (0/1)")
    ap.add_argument("--search-group", type=int, default=None)
    ap.add_argument("--max-nb", type=int, default=None, help="override the neighbour-list capacity")
    ap.add_argument("--solve-block", type=int, default=None)
    ap.add_argument("--list-skin", type=int, default=None,
                    help="neighbour-list reuse skin in per mille of r (0: a full search every step)")
    ap.add_argument("--search-cap", type=int, default=None,
                    help="list slots per particle in LDS for the search and filter kernels (0: from the last step)")
    ap.add_argument("--solve-mode", type=int, default=None, help="0 direct, 1 work queue, 2 persistent work queue")
    ap.add_argument("--no-autotune", action="store_true", help="keep the default launch shapes")
    ap.add_argument("--no-openbc", action="store_true",
                    help="skip the open-boundary calls (lp_outflow, lp_reservoir_inflow) on the same particles")
    ap.add_argument("--no-gfd3", action="store_true",
                    help="skip the third-order derivative operator (lp_gfd3) on the same particles")
    ap.add_argument("--copy-calibration", action="store_true",
                    help="only run 5 device copies of 1 GiB (HBM counter calibration) and exit")
    args = ap.parse_args()
    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) != 1:
        print("bench.py: this build measures one GPU only (the multi-GPU split is described, not built)",
              file=sys.stderr)
        sys.exit(2)

    import torch
    from paper_2206_11998_amd import lp, workloads as W

    if args.copy_calibration:
        a = torch.ones(1 << 27, dtype=torch.float64, device="cuda")
        b = torch.empty_like(a)
        for _ in range(5):
            b.copy_(a)
        torch.cuda.synchronize()
        print(json.dumps({"copy_bytes_read": a.numel() * 8, "copy_bytes_written": b.numel() * 8, "copies": 5}))
        return

    def log(*a):
        print("[bench]", *a, file=sys.stderr, flush=True)

    t0 = time.time()
    cfg, st = W.vacuum3d(n_particles=args.n)
    if args.max_nb:
        cfg["max_nb"] = args.max_nb
    n = st["V"].shape[0]
    log("workload generated: %d particles in %.1fs" % (n, time.time() - t0))
    rng = np.random.default_rng(1234)
    sample = (np.arange(n) if args.sample <= 0 or args.sample >= n
              else np.sort(rng.choice(n, size=args.sample, replace=False)))

    precisions = {"both": ["mixed", "fp64"], "all": ["mixed", "fp64", "mixed_all", "fp32", "mlp"]}.get(
        args.precision, [args.precision])
    mlp_params = None
    mlp_train = None
    if "mlp" in precisions:
        # the learned estimator's weights: trained on the GPU, before and
        # outside the timed region, on (inputs, quotient-estimator phi) of this
        # workload's particles, limited and unlimited ones in equal numbers
        t_tr = time.time()
        hctx = lp.Context(cfg)
        hdev = lp.state_to_device(st)
        feat, phi, valid = hctx.features(hdev)
        keep = valid.bool()
        feat, phi = feat[keep], phi[keep]
        lim = torch.nonzero(phi < 1.0).flatten()
        unl = torch.nonzero(phi >= 1.0).flatten()
        g = torch.Generator(device="cuda").manual_seed(3)
        m = min(len(lim), len(unl), 500_000)
        sel = torch.cat([lim[torch.randperm(len(lim), generator=g, device="cuda")[:m]],
                         unl[torch.randperm(len(unl), generator=g, device="cuda")[:m]]])
        sel = sel[torch.randperm(len(sel), generator=g, device="cuda")]
        fx, tx = feat[sel].contiguous(), (phi[sel] / 1.25).contiguous()  # the step uses min(1, 1.25 y)
        hctx.mlp_init(7)
        losses = hctx.mlp_train(fx, tx, epochs=8, batch=8192, lr=3e-3)
        _, y = hctx.mlp_forward(fx)
        agree = float((torch.abs(torch.clamp(1.25 * y, max=1.0) - 1.25 * tx) < 0.1).float().mean())
        mlp_params = hctx.mlp_get()
        mlp_train = {"samples": int(len(sel)), "epochs": 8, "final_loss": float(losses[-1]),
                     "within_0.1_of_plain_phi": agree, "seconds": time.time() - t_tr}
        log("learned estimator trained:", mlp_train)
        hctx.close()
        del hdev, feat, phi, fx, tx, y
    results = {}
    first_step = {}
    def tuned(ctx):
        if args.solve_mode is not None:
            ctx.set_tuning(lp.TUNE_SOLVE_MODE, args.solve_mode)
        if args.search_mode is not None:
            ctx.set_tuning(lp.TUNE_SEARCH_MODE, args.search_mode)
        if args.search_group is not None:
            ctx.set_tuning(lp.TUNE_SEARCH_GROUP, args.search_group)
        if args.solve_block is not None:
            ctx.set_tuning(lp.TUNE_SOLVE_BLOCK, args.solve_block)
        if args.list_skin is not None:
            ctx.set_tuning(lp.TUNE_LIST_SKIN, args.list_skin)
        if args.search_cap is not None:
            ctx.set_tuning(lp.TUNE_SEARCH_CAP, args.search_cap)
        return ctx

    for prec in precisions:
        ctx = lp.Context(cfg, precision="fp64" if prec == "fp64" else "mixed", refine=prec != "fp32",
                         refine_cond=args.refine_cond if prec in ("mixed", "mlp") else 0.0,
                         estimator="mlp" if prec == "mlp" else "plain")
        if prec == "mlp":
            ctx.mlp_set(mlp_params)
        dev = lp.state_to_device(st)
        tuning = None
        if not args.no_autotune:
            # tuned on the state a few steps in, where the cloud moves as in the
            # timed steps (from rest, the estimator and the lists see a different load)
            t_at = time.time()
            for _ in range(6):
                ctx.step(dev)
            tuning, at_ms = ctx.autotune(dev, reps=6)
            log(prec, "autotune chose %s (%.3f ms/step) in %.1fs" % (tuning, at_ms, time.time() - t_at))
            dev = lp.state_to_device(st)
            ctx.set_time(0.0)
        ctx = tuned(ctx)
        tuning = {name: ctx.get_tuning(q) for q, name in enumerate(lp.TUNE_NAMES)}
        # one step from the initial state for the accuracy check
        ctx.step(dev)
        if ctx.check() != lp.OK:
            raise RuntimeError(lp.lib().lp_last_error(ctx._h).decode())
        first_step[prec] = {k: (v[sample] if v.ndim == 1 else v[sample]) for k, v in lp.state_to_host(dev).items()}
        dt0 = ctx.info()["dt"]
        # per-kernel times: eager steps with HIP events around every stage,
        # recorded by the library on the stream it launches on
        dev = lp.state_to_device(st)
        ctx.set_time(0.0)
        for _ in range(args.warmup):
            ctx.step(dev)
        ctx.profile(True)
        for _ in range(args.steps):
            ctx.step(dev)
        prof = ctx.profile_read()
        ctx.profile(False)
        # timed run from the initial state: lp_run, the multi-step entry point
        # (one planning step, then graph replays of the captured step)
        dev = lp.state_to_device(st)
        ctx.set_time(0.0)
        ctx.run(dev, args.warmup)
        torch.cuda.synchronize()
        t_start = time.perf_counter()
        ctx.run(dev, args.steps)
        torch.cuda.synchronize()
        elapsed = time.perf_counter() - t_start
        status = ctx.check()
        info = ctx.info()
        log(prec, "steps %d in %.3fs -> %.3f ms/step; stages %s; info %s" % (
            args.steps, elapsed, 1e3 * elapsed / args.steps,
            {k: "%.3f ms" % (v[0] / max(v[1], 1)) for k, v in prof.items()}, info))
        results[prec] = {"elapsed": elapsed, "prof": prof, "status": status, "info": info, "dt0": dt0,
                         "tuning": tuning}
        del dev
        ctx.close()

    # stencil sizes for the algorithmic work (state at the start of the timed run)
    ctx = lp.Context(cfg)
    d = lp.state_to_device(st)
    h = (st["m"] * st["V"]) ** (1.0 / 3.0)
    r = torch.from_numpy(cfg["kappa"] * h).cuda()
    count, _, _ = ctx.neighbors(d["x"], r)
    count = count.cpu().numpy()
    k_lw = np.minimum(count, 54)
    work = {"search": float(search_bytes(count).sum()), "fit": float(fit_flops(k_lw).sum()),
            "update": float(update_flops() * n), "mlp": float(MLP_FLOPS * n), "cells": cells_bytes(n)}
    ctx.close()
    del d

    # CPU reference on the sample: one step of the same input
    l1 = {}
    cpu = None
    try:
        import oracle
        # the same step repeated until about 8 s of CPU time have elapsed (at most 8 times)
        reps, cpu_total = 0, 0.0
        while reps == 0 or (cpu_total < 8.0 and reps < 8):
            t1 = time.perf_counter()
            ref, rinfo = oracle.step_subset(cfg, st, sample)
            cpu_total += time.perf_counter() - t1
            reps += 1
        cpu_time = cpu_total / reps
        threads = oracle.num_threads()
        log("cpu reference: %d particles in %.2fs (mean of %d) with %d threads (status %d)" % (
            len(sample), cpu_time, reps, threads, rinfo["status"]))
        cpu = {"value": len(sample) / cpu_time, "unit": "particle-updates/s", "cores": threads, "kind": "oracle",
               "sample": "one step of %d particles of the %d-particle workload (global dt and bucket grid over "
                         "all particles included), timed %d times, mean" % (len(sample), n, reps),
               "cpu_model": cpu_model(), "host_threads": os.cpu_count()}
        # the same oracle on one thread, on the 100,000 particles nearest the centre (one step)
        try:
            sub = np.argsort((st["x"] ** 2).sum(axis=1))[:100_000]
            oracle.set_num_threads(1)
            t1 = time.perf_counter()
            oracle.step_subset(cfg, st, np.sort(sub))
            t1 = time.perf_counter() - t1
            cpu["single_thread"] = {"value": len(sub) / t1, "unit": "particle-updates/s", "cores": 1,
                                    "sample": "one step of the 100,000 particles nearest the centre (the densest, "
                                              "longest lists) of the same workload"}
            log("cpu reference, one thread: %d particles in %.2fs" % (len(sub), t1))
        finally:
            oracle.set_num_threads(threads)
        cvmax = np.sqrt(cfg["gamma"] * st["P"] * st["V"]).max()
        for prec, got in first_step.items():
            e = {}
            for key in ("V", "P", "u", "x"):
                a, b = got[key], ref[key]
                den = np.abs(b).sum()
                if key == "u":
                    den = max(den, b.size * 1e-12 * cvmax)
                e[key] = float(np.abs(a - b).sum() / den)
            l1[prec] = e
        if args.no_cpu_baseline:
            cpu = None
    except Exception as exc:  # the reference is optional on hosts without gcc
        log("cpu reference unavailable:", repr(exc))

    def fused(precision):
        """FP32 fits refined where ill-conditioned (or not at all) run with the
        update in one kernel (k_fit_finish); FP64 and always-refined fits
        keep the fit and update kernels apart."""
        return precision == "fp32" or (precision in ("mixed", "mlp") and args.refine_cond > 0)

    def kernel_rooflines(prof, precision):
        out = {}
        for name, bound in (("search", "hbm"), ("fit", "alu"), ("update", "alu"), ("mlp", "mfma")):
            ms, cnt = prof[name]
            if cnt == 0 or (name == "update" and fused(precision)):
                continue
            avg = ms / max(cnt, 1)
            if name == "fit" and fused(precision):
                # the fit stage holds the fused kernel (and the refinement of
                # the queued fits, which updates those particles)
                name, wk = "fit+update", work["fit"] + work["update"]
            else:
                wk = work[name]
            if bound == "hbm":
                achieved = wk / (avg * 1e-3) / 1e9 if avg > 0 else None
                peak, unit, per = PEAK_HBM_GBS, "GB/s", "algorithmic_bytes_per_launch"
            elif bound == "mfma":
                achieved = wk / (avg * 1e-3) / 1e12 if avg > 0 else None
                peak, unit, per = PEAK_BF16_TFLOPS, "TFLOP/s", "algorithmic_flops_per_launch"
            else:
                achieved = wk / (avg * 1e-3) / 1e12 if avg > 0 else None
                peak, unit, per = PEAK_ALU_TFLOPS, "TFLOP/s", "algorithmic_flops_per_launch"
            out[name] = {"bound": bound, "achieved": achieved, "peak": peak, "unit": unit,
                         "frac": achieved / peak if achieved else None,
                         "traffic": committed_traffic(name, precision), per: wk,
                         "avg_launch_ms": avg}
        return out

    def step_roofline(prof, ms_step):
        """The whole step against its roofline: each stage's algorithmic
        minimum time (bytes / HBM peak or flops / ALU or MFMA peak), summed,
        over the measured time per step."""
        terms = {"prep+cells": work["cells"] / (PEAK_HBM_GBS * 1e9) * 1e3,
                 "search": work["search"] / (PEAK_HBM_GBS * 1e9) * 1e3,
                 "fit": work["fit"] / (PEAK_ALU_TFLOPS * 1e12) * 1e3,
                 "update": work["update"] / (PEAK_ALU_TFLOPS * 1e12) * 1e3}
        if prof.get("mlp", (0, 0))[1]:
            terms["mlp"] = work["mlp"] / (PEAK_BF16_TFLOPS * 1e12) * 1e3
        floor = sum(terms.values())
        return {"floor_ms": floor, "measured_ms": ms_step, "frac": floor / ms_step,
                "terms_ms": terms}

    main_prec = precisions[0]
    res = results[main_prec]
    ms_step = 1e3 * res["elapsed"] / args.steps
    value = n * args.steps / res["elapsed"]
    kr = kernel_rooflines(res["prof"], main_prec)
    dominant = max(kr, key=lambda k: kr[k]["avg_launch_ms"])
    top = dict(kr[dominant])
    top["kernel"] = {"search": "k_search (neighbour lists)", "fit": "k_lw_fit (second-order fits)",
                     "update": "k_finish (half-ball fits, estimator, update, mover)",
                     "fit+update": "k_fit_finish (second-order fit, half-ball fits, estimator, update, mover)",
                     "mlp": "k_mlp_apply (network estimator, update, mover)"}[dominant]
    out = {
        "metric": METRIC,
        "value": value,
        "unit": "particle-updates/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms_step,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64" if main_prec == "fp64" else "f32+f64",
        "data": "synthetic",
        "config": {"workload": "vacuum3d: %d equal-mass particles rejection-sampled from rho=exp(-r^2/0.05) "
                               "in the ball rho>=1/512, p=rho^1.4, kappa 2.2, CFL 0.2, free boundary" % n,
                   "n_particles": n, "precision": main_prec, "mean_lw_stencil": float(k_lw.mean()),
                   "refine_cond": args.refine_cond if main_prec in ("mixed", "mlp") else None,
                   "refined_fits_per_step": res["info"].get("n_refined")},
        "roofline": top,
        "step_roofline": step_roofline(res["prof"], ms_step),
        "kernels": kr,
        "cpu_baseline": cpu,
        "stages_ms_per_step": {k: v[0] / max(v[1], 1) for k, v in res["prof"].items()},
        "tuning": res["tuning"],
        "l1_vs_oracle": l1,
    }
    if not args.no_gfd3:
        out["gfd3"] = gfd3_leg(lp, torch, cfg, st, log, args.no_cpu_baseline)
    if not args.no_openbc:
        out["open_boundary"] = openbc_leg(lp, torch, cfg, st, log, args.no_cpu_baseline)
    for prec in precisions[1:]:
        r2 = results[prec]
        out[prec] = {"value": n * args.steps / r2["elapsed"], "ms_per_step": 1e3 * r2["elapsed"] / args.steps,
                     "kernels": kernel_rooflines(r2["prof"], prec), "tuning": r2["tuning"],
                     "step_roofline": step_roofline(r2["prof"], 1e3 * r2["elapsed"] / args.steps),
                     "refined_fits_per_step": r2["info"].get("n_refined"),
                     "stages_ms_per_step": {k: v[0] / max(v[1], 1) for k, v in r2["prof"].items()}}
        if prec == "mlp":
            out[prec]["learned_estimator"] = dict(mlp_train, n_network=r2["info"]["n_mlp"],
                                                  n_fallback=r2["info"]["n_mlp_plain"])
    print(json.dumps(out))


if __name__ == "__main__":
    main()
