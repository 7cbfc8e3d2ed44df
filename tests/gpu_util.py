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


def compare_states(got, ref, cfg, tol, tag=""):
    """Relative L1 per field (velocity scaled by the max sound speed)."""
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
    say(tag, {k: "%.2e" % v for k, v in errs.items()})
    for k in ("V", "P", "u"):
        assert errs[k] <= tol, (tag, k, errs[k])
    assert errs["x"] <= tol * 10, (tag, "x", errs["x"])
    return errs
