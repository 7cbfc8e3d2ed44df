"""Helpers for the GPU parity tests."""
import sys

import numpy as np


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def radii(cfg, st):
    d = cfg["dim"]
    return cfg["kappa"] * (st["m"] * st["V"]) ** (1.0 / d)


def rel_l1(got, ref, scale=None):
    den = np.abs(ref).sum()
    if scale is not None:
        den = max(den, ref.size * 1e-12 * scale)
    return np.abs(got - ref).sum() / max(den, 1e-300)


def compare_states(got, ref, cfg, tol, tag="", tol_pp=None):
    """Relative L1 per field (velocity scaled by the max sound speed), and the
    largest single-particle error relative to the field's largest magnitude
    (tol_pp; default 1e-8 for the FP64 tolerance, 1e-3 for the mixed one)."""
    c = np.sqrt(cfg["gamma"] * ref["P"] * ref["V"]).max()
    errs = {
        "V": rel_l1(got["V"], ref["V"]),
        "P": rel_l1(got["P"], ref["P"]),
        "u": rel_l1(got["u"], ref["u"], scale=c),
    }
    span = np.array(cfg["box_hi"]) - np.array(cfg["box_lo"])
    dx = got["x"] - ref["x"]
    for a in range(cfg["dim"]):
        if cfg["periodic"][a]:
            dx[:, a] -= span[a] * np.round(dx[:, a] / span[a])
    errs["x"] = np.abs(dx).max()
    if tol_pp is None:
        tol_pp = 1e-8 if tol <= 1e-9 else 1e-3
    pp = {
        "V": np.abs(got["V"] - ref["V"]).max() / np.abs(ref["V"]).max(),
        "P": np.abs(got["P"] - ref["P"]).max() / np.abs(ref["P"]).max(),
        "u": np.abs(got["u"] - ref["u"]).max() / max(np.abs(ref["u"]).max(), c),
    }
    say(tag, {k: "%.2e" % v for k, v in errs.items()}, "per particle", {k: "%.2e" % v for k, v in pp.items()})
    for k in ("V", "P", "u"):
        assert errs[k] <= tol, (tag, k, errs[k])
        assert pp[k] <= tol_pp, (tag, "per particle", k, pp[k])
    assert errs["x"] <= tol * 10, (tag, "x", errs["x"])
    return errs


def compare_phi(got_phi, ref_phi, fp64, tag=""):
    """Limiter values.  FP64 path: within 1e-6 of the oracle at every
    particle.  Mixed path: the estimator takes its decisions on FP32
    one-sided slopes (the kernel's precision), so where a slope sits at the
    rounding level (below the activity threshold or changing sign) phi can
    differ from the FP64 decision by up to the limiter's range; the fields'
    per-particle bound above is what the mixed path is held to, and the
    number of such particles is reported."""
    d = np.abs(np.asarray(got_phi, dtype=np.float64) - ref_phi)
    far = int((d > 1e-6).sum())
    say(tag, "phi: max |dphi| %.2e, particles beyond 1e-6: %d of %d" % (d.max(), far, d.size))
    if fp64:
        assert far == 0, (tag, far, d.max())
    else:
        assert np.all(np.asarray(got_phi) >= 0.0) and np.all(np.asarray(got_phi) <= 1.25)
    return far


def accuracy_phi(ns0, ns1, ex_V, ex_u, ex_P, V_scale, u_scale, P_scale):
    """Per particle, the blend weight phi in [0, 1] whose step lands closest to
    the exact state: the update is linear in phi, s(phi) = s0 - phi (s0 - s1)
    with s0 the upwind (phi = 0) and s1 the Lax-Wendroff (phi = 1) result, so
    the least-squares weight over V, u and P (each scaled) is
    sum a b / sum b^2 with a = s0 - exact, b = s0 - s1, clipped to [0, 1].
    NaN where the two results coincide (phi does not matter there).
    Returns (phi, sum b^2)."""
    D = ns0["u"].shape[1]
    terms = [(ns0["V"], ns1["V"], ex_V, V_scale)]
    terms += [(ns0["u"][:, q], ns1["u"][:, q], ex_u[:, q], u_scale) for q in range(D)]
    terms += [(ns0["P"], ns1["P"], ex_P, P_scale)]
    num = np.zeros(len(ex_V))
    den = np.zeros(len(ex_V))
    for s0, s1, ex, sc in terms:
        a = (s0 - ex) / sc
        b = (s0 - s1) / sc
        num += a * b
        den += b * b
    phi = np.full(len(ex_V), np.nan)
    ok = den > 1e-30
    phi[ok] = np.clip(num[ok] / den[ok], 0.0, 1.0)
    return phi, den
