"""Plain numpy definitions used to pin the oracle (no shared code with it)."""
import numpy as np


def min_image(d, L):
    half = 0.5 * L
    return np.where(d > half, d - L, np.where(d < -half, d + L, d))


def brute_neighbors(cfg, x, r):
    """All-pairs definition: N(i) = {j != i : d2 < r_i^2}, ordered by (d2, j).

    d2 = ((dx*dx) + (dy*dy)) + (dz*dz) evaluated elementwise in IEEE binary64."""
    n, D = x.shape
    out = []
    for i in range(n):
        dx = []
        for a in range(D):
            d = x[:, a] - x[i, a]
            if cfg["periodic"][a]:
                d = min_image(d, cfg["box_hi"][a] - cfg["box_lo"][a])
            dx.append(d)
        d2 = dx[0] * dx[0] + dx[1] * dx[1]
        if D == 3:
            d2 = d2 + dx[2] * dx[2]
        mask = d2 < r[i] * r[i]
        mask[i] = False
        j = np.nonzero(mask)[0]
        order = np.lexsort((j, d2[j]))
        out.append(j[order].astype(np.int32))
    return out
