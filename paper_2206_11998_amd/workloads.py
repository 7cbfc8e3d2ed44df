"""Seeded synthetic particle workloads (initial conditions only).

This module builds particle sets and their initial states; it holds none of
the method's arithmetic (no smoothing lengths, radii, time steps, fits or
updates), so it can feed both the GPU library and the CPU oracle.  Every
generator is deterministic in its seed (numpy PCG64).

Workloads (γ = 1.4 everywhere):

* ``pulse2d``   -- 2D pressure pulse, 64x64 jittered lattice on the periodic
  unit square, ρ = 1, u = 0, p = 1 + 0.1 exp(-|x - ½|²/0.01), κ = 2.5.
* ``sod3d``     -- 3D Sod shock tube on a jittered n³ lattice of [0,1]³,
  (ρ, p) = (1, 1) for x < ½ and (0.125, 0.1) otherwise, mirror walls at
  x = 0, 1, periodic in y and z, κ = 2.1.
* ``vacuum3d``  -- 3D expansion into vacuum: equal-mass particles
  rejection-sampled from ρ = exp(-|x|²/0.05) inside the ball of radius
  √(0.05 ln 512), so ρ spans 512x and the particle spacing exactly 8x,
  p = ρ^γ, u = 0, free boundary, κ = 2.2.
* ``sedov3d``   -- 3D Sedov-type blast: jittered 2:1:1 lattice on
  [0,2]x[0,1]², ρ = 1, p = 1e-5, energy 1 deposited as internal energy
  around the centre (a Gaussian of width 2h by default, or the literal 27
  lattice particles), periodic, κ = 2.1, CFL 0.1.
* ``yee_vortex`` -- 2D Yee vortex (Sec. 2.3): an isentropic vortex of strength
  β = 5 in the free stream (u, v, ρ, p) = (1, 0, 1, 1), on an almost hexagonal
  lattice of the periodic square [-5, 5]², κ = 3.5 with every neighbour in
  the second-order fit; ``yee_exact`` is its exact solution, the initial state
  convected with the free stream.
* ``vacuum_slab`` -- a uniform gas slab (ρ, p) = (1, 1) at rest on
  x ∈ [-½, ½], periodic across, expanding into vacuum on both x faces.
* ``shear3d``   -- 3D shear layer: jittered n³ lattice of [0,1]³, periodic in
  x, z, mirror walls at y = 0, 1, u_x = 0.5 tanh((y-½)/0.025),
  u_y = 0.01 sin(2πx) exp(-((y-½)/0.05)²), ρ = 1.5 + 0.5 tanh((y-½)/0.025),
  p = 2.5, κ = 2.1.

Lattice particles sit at (i + ½)h plus a uniform jitter in (-0.2h, 0.2h) per
coordinate; lattice masses are m = ρ(x) h^D so that every particle carries its
own cell's mass.  The 2D workload runs at CFL 0.5; the 3D ones at CFL 0.2
(the blended scheme's upwind part sums the 1D rates over the axes, which
lowers its stable CFL number on scattered particles).  The Sod interface is
spread over one particle spacing by a tanh profile.
"""
from __future__ import annotations

import math

import numpy as np

GAMMA = 1.4


def base_config(name, dim, kappa, box_lo, box_hi, periodic, wall_lo=None, wall_hi=None, vacuum=False,
                cfl=0.5, **extra):
    d = dim
    cfg = {
        "name": name, "dim": d, "gamma": GAMMA, "cfl": cfl, "kappa": kappa,
        "box_lo": list(box_lo), "box_hi": list(box_hi), "periodic": list(periodic),
        "wall_lo": list(wall_lo or [False] * d), "wall_hi": list(wall_hi or [False] * d),
        "vacuum": bool(vacuum), "max_nb": 128, "lw_cap": 0, "uw_cap": 0,
        "est_eps": 1e-5, "cond_max": 1e12, "uw_cond_max": 1e2,
    }
    cfg.update(extra)
    return cfg


def jittered_lattice(shape, h, jitter=0.2, seed=0, origin=None):
    """Points at (i + ½)h + U(-jitter h, jitter h) per coordinate, C order over shape."""
    rng = np.random.Generator(np.random.PCG64(seed))
    d = len(shape)
    grids = np.meshgrid(*[np.arange(s, dtype=np.float64) for s in shape], indexing="ij")
    idx = np.stack([g.reshape(-1) for g in grids], axis=1)
    x = (idx + 0.5) * h
    if jitter:
        x = x + rng.uniform(-jitter * h, jitter * h, size=x.shape)
    if origin is not None:
        x = x + np.asarray(origin, dtype=np.float64)[None, :d]
    return np.ascontiguousarray(x), idx.astype(np.int64)


def _state(x, rho, u, p, m):
    return {"x": np.ascontiguousarray(x, dtype=np.float64),
            "u": np.ascontiguousarray(u, dtype=np.float64),
            "V": np.ascontiguousarray(1.0 / rho, dtype=np.float64),
            "P": np.ascontiguousarray(p, dtype=np.float64),
            "m": np.ascontiguousarray(m, dtype=np.float64)}


def pulse2d(n=64, seed=0, jitter=0.2, steps=10):
    h = 1.0 / n
    x, _ = jittered_lattice((n, n), h, jitter, seed)
    rho = np.ones(x.shape[0])
    r2 = ((x - 0.5) ** 2).sum(axis=1)
    p = 1.0 + 0.1 * np.exp(-r2 / 0.01)
    u = np.zeros_like(x)
    m = rho * h * h
    cfg = base_config("pulse2d", 2, 2.5, [0.0, 0.0], [1.0, 1.0], [True, True], steps=steps)
    return cfg, _state(x, rho, u, p, m)


def sod3d(n=64, seed=1, jitter=0.2, ny=None, nz=None, t_end=0.1, smooth=1.0):
    """Sod tube along x; ny, nz (default n) set the periodic cross-section in cells of h = 1/n.

    The initial jump at x = ½ is spread over ``smooth`` particle spacings by a
    tanh profile (0 gives the sharp jump)."""
    ny = n if ny is None else ny
    nz = n if nz is None else nz
    h = 1.0 / n
    x, _ = jittered_lattice((n, ny, nz), h, jitter, seed)
    if smooth > 0.0:
        w = 0.5 * (1.0 + np.tanh((x[:, 0] - 0.5) / (smooth * h)))
    else:
        w = (x[:, 0] >= 0.5).astype(np.float64)
    rho = 1.0 + (0.125 - 1.0) * w
    p = 1.0 + (0.1 - 1.0) * w
    u = np.zeros_like(x)
    m = rho * h ** 3
    cfg = base_config("sod3d", 3, 2.1, [0.0, 0.0, 0.0], [1.0, ny * h, nz * h], [False, True, True],
                      wall_lo=[True, False, False], wall_hi=[True, False, False], t_end=t_end, cfl=0.2)
    return cfg, _state(x, rho, u, p, m)


def morton_keys(x, lo, side, bits):
    """Morton (Z-order) key of each point on a 2^bits grid over the cube [lo, lo + side)^D."""
    d = x.shape[1]
    c = np.clip(((x - lo) / side * (1 << bits)).astype(np.int64), 0, (1 << bits) - 1)
    key = np.zeros(x.shape[0], dtype=np.int64)
    for b in range(bits):
        for a in range(d):
            key |= ((c[:, a] >> b) & 1) << (d * b + a)
    return key


def vacuum_ball_radius(a=0.05, ratio=512.0):
    return math.sqrt(a * math.log(ratio))


def vacuum3d(n_particles=2_097_152, seed=2, a=0.05, steps=20, box=1.0):
    """Equal-mass particles rejection-sampled from ρ = exp(-|x|²/a) in the ball where ρ ≥ 1/512."""
    R = vacuum_ball_radius(a)
    rng = np.random.Generator(np.random.PCG64(seed))
    chunks = []
    have = 0
    while have < n_particles:
        m = max(4096, int(1.3 * (n_particles - have) / 0.11) + 1024)
        c = rng.uniform(-R, R, size=(m, 3))
        r2 = (c * c).sum(axis=1)
        keep = (r2 <= R * R) & (rng.uniform(0.0, 1.0, size=m) < np.exp(-r2 / a))
        c = c[keep]
        chunks.append(c)
        have += c.shape[0]
    x = np.concatenate(chunks, axis=0)[:n_particles]
    # store the particles along a space-filling (Morton) curve, as an LP code
    # keeps its particle array (paper, Sec. 2.2)
    x = x[np.argsort(morton_keys(x, -R, 2.0 * R, 10), kind="stable")]
    r2 = (x * x).sum(axis=1)
    rho = np.exp(-r2 / a)
    z = R / math.sqrt(a)
    total = 4.0 * math.pi * a ** 1.5 * (math.sqrt(math.pi) / 4.0 * math.erf(z) - 0.5 * z * math.exp(-z * z))
    m = np.full(n_particles, total / n_particles)
    p = rho ** GAMMA
    u = np.zeros_like(x)
    cfg = base_config("vacuum3d", 3, 2.2, [-box, -box, -box], [box, box, box], [False, False, False],
                      vacuum=True, steps=steps, cfl=0.2, max_nb=256)
    return cfg, _state(x, rho, u, p, m)


def sedov3d(nx=256, seed=3, jitter=0.2, p_bg=1e-5, energy=1.0, steps=50, deposit="gauss", sigma=2.0):
    """Sedov-type blast on a jittered 2:1:1 lattice of [0,2]x[0,1]^2 (h = 2/nx),
    rho = 1, background pressure p_bg, periodic.  The energy is internal energy
    around the lattice centre (index (nx/2, nx/4, nx/4)):

    - deposit="gauss" (default): specific energy proportional to
      exp(-|x - x_c|^2 / (2 (sigma h)^2)) over every particle, scaled so that
      the total is `energy`; sigma = 2 smoothing lengths.
    - deposit="block27": the literal 3x3x3 block of lattice particles around
      the centre.  Its first step drives V or P below zero next to the block
      (a pressure ratio of 3e9 between neighbours), in the oracle as on the GPU.

    Time step at CFL 0.1 and lists up to 256 entries: the hot core's radius
    grows with its volume and reaches into the compressed shell."""
    ny = nz = nx // 2
    h = 2.0 / nx
    x, idx = jittered_lattice((nx, ny, nz), h, jitter, seed)
    rho = np.ones(x.shape[0])
    m = rho * h ** 3
    p = np.full(x.shape[0], p_bg)
    c = np.array([nx // 2, ny // 2, nz // 2])
    if deposit == "block27":
        hot = np.all(np.abs(idx - c[None, :]) <= 1, axis=1)
        e = energy / (27.0 * m[hot])
        p[hot] = (GAMMA - 1.0) * rho[hot] * e
    else:
        xc = (c + 0.5) * h
        w = np.exp(-((x - xc[None, :]) ** 2).sum(axis=1) / (2.0 * (sigma * h) ** 2))
        e = energy * w / (m * w).sum()
        p = p + (GAMMA - 1.0) * rho * e
    u = np.zeros_like(x)
    cfg = base_config("sedov3d", 3, 2.1, [0.0, 0.0, 0.0], [2.0, 1.0, 1.0], [True, True, True], steps=steps,
                      cfl=0.1, max_nb=256)
    return cfg, _state(x, rho, u, p, m)


def sedov_radius(t, energy=1.0, rho0=1.0, xi0=1.033):
    """Self-similar blast-wave radius xi0 (E t^2 / rho0)^(1/5); xi0 = 1.033 is
    Taylor's constant for gamma = 1.4 in three dimensions."""
    return xi0 * (energy * t * t / rho0) ** 0.2


def shear3d(n=256, seed=4, jitter=0.2, steps=100):
    h = 1.0 / n
    x, _ = jittered_lattice((n, n, n), h, jitter, seed)
    y = x[:, 1]
    t = np.tanh((y - 0.5) / 0.025)
    u = np.zeros_like(x)
    u[:, 0] = 0.5 * t
    u[:, 1] = 0.01 * np.sin(2.0 * math.pi * x[:, 0]) * np.exp(-((y - 0.5) / 0.05) ** 2)
    rho = 1.5 + 0.5 * t
    p = np.full(x.shape[0], 2.5)
    m = rho * h ** 3
    cfg = base_config("shear3d", 3, 2.1, [0.0, 0.0, 0.0], [1.0, 1.0, 1.0], [True, False, True],
                      wall_lo=[False, True, False], wall_hi=[False, True, False], steps=steps, cfl=0.2)
    return cfg, _state(x, rho, u, p, m)


def uniform_box(dim, n, seed=5, jitter=0.2, periodic=True, kappa=None, rho=1.0, p=1.0, u0=None):
    """Jittered lattice with a constant state (optionally a constant velocity)."""
    h = 1.0 / n
    x, _ = jittered_lattice((n,) * dim, h, jitter, seed)
    N = x.shape[0]
    u = np.zeros_like(x)
    if u0 is not None:
        u[:] = np.asarray(u0, dtype=np.float64)[None, :dim]
    rr = np.full(N, rho)
    cfg = base_config("uniform%dd" % dim, dim, kappa or (2.5 if dim == 2 else 2.1), [0.0] * dim, [1.0] * dim,
                      [periodic] * dim, cfl=0.5 if dim == 2 else 0.2)
    return cfg, _state(x, rr, u, np.full(N, p), rr * h ** dim)


def smooth_wave(dim, n, seed=6, jitter=0.2, amp=1e-2):
    """Jittered periodic lattice with a smooth, fully 3D (or 2D) acoustic perturbation."""
    h = 1.0 / n
    x, _ = jittered_lattice((n,) * dim, h, jitter, seed)
    N = x.shape[0]
    ph = 2.0 * math.pi * x
    s = np.sin(ph[:, 0])
    for a in range(1, dim):
        s = s + 0.5 * np.cos(ph[:, a] + 0.3 * a)
    rho = 1.0 + amp * s
    p = 1.0 + GAMMA * amp * s
    u = np.zeros_like(x)
    for a in range(dim):
        u[:, a] = amp * np.sin(ph[:, (a + 1) % dim] + 0.7 * a)
    cfg = base_config("wave%dd" % dim, dim, 2.5 if dim == 2 else 2.1, [0.0] * dim, [1.0] * dim, [True] * dim,
                      cfl=0.5 if dim == 2 else 0.2)
    return cfg, _state(x, rho, u, p, rho * h ** dim)


WORKLOADS = {
    "pulse2d": pulse2d,
    "sod3d": sod3d,
    "vacuum3d": vacuum3d,
    "sedov3d": sedov3d,
    "shear3d": shear3d,
}


def vacuum_slab(n, dim=3, nt=4, seed=11, jitter=0.2, kappa=2.2):
    """Uniform gas (ρ, p) = (1, 1) at rest on a jittered lattice of spacing
    h = 1/n filling x ∈ [-½, ½] and nt cells across (periodic on the other
    axes), free boundary (vacuum) on both x faces.  Masses m = h^dim."""
    h = 1.0 / n
    x, _ = jittered_lattice((n,) + (nt,) * (dim - 1), h, jitter, seed)
    x[:, 0] -= 0.5
    N = x.shape[0]
    cfg = base_config("vacuum_slab", dim, kappa, [-4.0] + [0.0] * (dim - 1), [4.0] + [nt * h] * (dim - 1),
                      [False] + [True] * (dim - 1), vacuum=True, cfl=0.2)
    return cfg, _state(x, np.ones(N), np.zeros((N, dim)), np.ones(N), np.full(N, h ** dim))


def yee_exact(x, t, beta=5.0, half=5.0, center=(0.0, 0.0)):
    """Yee vortex at time t: the initial vortex convected by the free stream
    (1, 0), its centre wrapped into the periodic square [-half, half]^2 and
    offsets taken to the nearest image (the vortex is below e^-12 of its
    amplitude at distance 5).  Returns (rho, u (N x 2), p).

    T = 1 - (gamma-1) beta^2 / (8 gamma pi^2) exp(1 - r^2), rho = T^(1/(gamma-1)),
    (u, v) = (1, 0) + beta/(2 pi) exp((1 - r^2)/2) (-(y - y0), x - x0), p = rho^gamma."""
    L = 2.0 * half
    xc = np.array([center[0] + t, center[1]])
    xc = (xc + half) % L - half
    d = x[:, :2] - xc
    d -= L * np.round(d / L)
    r2 = (d * d).sum(axis=1)
    T = 1.0 - (GAMMA - 1.0) * beta ** 2 / (8.0 * GAMMA * math.pi ** 2) * np.exp(1.0 - r2)
    rho = T ** (1.0 / (GAMMA - 1.0))
    a = beta / (2.0 * math.pi) * np.exp(0.5 * (1.0 - r2))
    u = np.stack([1.0 - a * d[:, 1], a * d[:, 0]], axis=1)
    return rho, u, rho ** GAMMA


def yee_vortex(dx, beta=5.0, half=5.0, jitter=0.0, seed=7, kappa=3.5, lw_cap=64):
    """2D Yee vortex on an almost hexagonal lattice of the periodic square
    [-half, half]^2: nx = L/dx columns, an even number of rows spaced as close
    to dx sqrt(3)/2 as the box allows, alternate rows shifted by dx/2 (the
    rows of a periodic square cannot be exactly sqrt(3)/2 apart); optional
    uniform jitter of +-jitter*dx.  Masses m = rho dx dy.

    Stencil: radius kappa = 3.5 smoothing lengths (about 44 neighbours on the
    lattice) with every neighbour in the second-order fit (lw_cap 64).  The
    vortex shears the particle set until neighbours come within 0.15 h and
    leave angular gaps past 130 degrees; with 18 neighbours (kappa 2.5) the
    second-order update loses stability there, with 44 it stays stable to
    t = 8 at every resolution of the paper's tables."""
    L = 2.0 * half
    nx = max(2, int(round(L / dx)))
    ddx = L / nx
    ny = max(2, int(round(L / (ddx * math.sqrt(3.0) / 2.0))))
    ny += ny % 2
    ddy = L / ny
    j, i = np.meshgrid(np.arange(ny), np.arange(nx), indexing="ij")
    x = np.stack([-half + (i + 0.5 + 0.5 * (j % 2)) * ddx, -half + (j + 0.5) * ddy], axis=-1).reshape(-1, 2)
    if jitter > 0.0:
        rng = np.random.default_rng(seed)
        x += rng.uniform(-jitter, jitter, size=x.shape) * np.array([ddx, ddy])
    x = (x + half) % L - half
    rho, u, p = yee_exact(x, 0.0, beta, half)
    m = rho * ddx * ddy
    cfg = base_config("yee2d", 2, kappa, [-half, -half], [half, half], [True, True], beta=beta)
    cfg["lw_cap"] = lw_cap
    return cfg, _state(x, rho, u, p, m)


def yee_vortex3d(dx, beta=5.0, half=5.0, z_div=8, kappa=2.2, jitter=0.0, seed=7):
    """The Yee vortex extruded along z (the 3D variant of Sec. 2.3): the 2D
    lattice of yee_vortex repeated in nz layers over the periodic z extent
    L / z_div (L = 2 half; a periodic extent must be the largest one over a
    power of two), nz = round(L / z_div / dx) layers at (k + 1/2) dz.  The
    state does not depend on z and the z velocity is 0; masses m = rho dx dy dz.
    Particles are stored layer by layer.  With jitter > 0 every particle
    moves by up to +-jitter of the spacing per axis, independently in each
    layer, and takes the exact state at its new position: no two neighbours
    are then at exactly equal distance."""
    _, st2 = yee_vortex(dx, beta, half)
    L = 2.0 * half
    lz = L / z_div
    nz = max(2, int(round(lz / dx)))
    dz = lz / nz
    n2 = st2["V"].shape[0]
    z = np.repeat((np.arange(nz) + 0.5) * dz, n2)
    st = {"x": np.concatenate([np.tile(st2["x"], (nz, 1)), z[:, None]], axis=1),
          "u": np.concatenate([np.tile(st2["u"], (nz, 1)), np.zeros((nz * n2, 1))], axis=1),
          "V": np.tile(st2["V"], nz), "P": np.tile(st2["P"], nz), "m": np.tile(st2["m"], nz) * dz}
    if jitter > 0.0:
        rng = np.random.default_rng(seed)
        area = st2["m"][0] * st2["V"][0]          # dx dy of the 2D lattice
        hx = L / max(2, int(round(L / dx)))
        x = st["x"] + rng.uniform(-jitter, jitter, size=st["x"].shape) * np.array([hx, area / hx, dz])
        x[:, :2] = (x[:, :2] + half) % L - half
        x[:, 2] %= lz
        rho, u, p = yee_exact(x, 0.0, beta, half)
        st = {"x": x, "u": np.concatenate([u, np.zeros((x.shape[0], 1))], axis=1), "V": 1.0 / rho, "P": p,
              "m": rho * area * dz}
    cfg = base_config("yee3d", 3, kappa, [-half, -half, 0.0], [half, half, lz], [True, True, True], beta=beta)
    return cfg, {k: np.ascontiguousarray(v) for k, v in st.items()}
