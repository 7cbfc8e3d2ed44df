"""Pin P1: the oracle's bucket-grid neighbour search equals the all-pairs
definition (Sec. 2.2, step 3) bit for bit, including order by (d2, id)."""
import numpy as np
import pytest

from paper_2206_11998_amd import workloads as W
from tests.brute import brute_neighbors


def _radii(cfg, st):
    d = cfg["dim"]
    h = (st["m"] * st["V"]) ** (1.0 / d)
    return cfg["kappa"] * h


def _check(oracle_lib, cfg, x, r, max_nb=256):
    count, idx, status = oracle_lib.neighbors(cfg, x, r, max_nb=max_nb)
    assert status == 0
    ref = brute_neighbors(cfg, x, r)
    for i in range(x.shape[0]):
        assert count[i] == len(ref[i]), i
        assert np.array_equal(idx[i, :count[i]], ref[i]), i
    return count


def test_pulse2d_whole(oracle_lib):
    cfg, st = W.pulse2d()
    c = _check(oracle_lib, cfg, st["x"], _radii(cfg, st))
    assert 15 <= c.min() and c.max() <= 26


def test_periodic_3d_lattice(oracle_lib):
    cfg, st = W.uniform_box(3, 10, seed=11)
    _check(oracle_lib, cfg, st["x"], _radii(cfg, st))


def test_exact_lattice_ties(oracle_lib):
    # unjittered lattice: many equal distances, so the id tie-break decides the order
    cfg, st = W.uniform_box(3, 8, jitter=0.0)
    count = _check(oracle_lib, cfg, st["x"], _radii(cfg, st))
    assert np.all(count == count[0])


def test_variable_radius_free_space(oracle_lib):
    cfg, st = W.vacuum3d(n_particles=3000, seed=7)
    _check(oracle_lib, cfg, st["x"], _radii(cfg, st), max_nb=3000)


def test_radius_on_a_distance_is_excluded(oracle_lib):
    # d2 == r^2 exactly is not a neighbour (strict inequality)
    cfg = W.base_config("t", 2, 1.0, [0.0, 0.0], [10.0, 10.0], [False, False])
    x = np.array([[1.0, 1.0], [1.5, 1.0], [1.0, 2.0], [1.25, 1.0]])
    r = np.array([0.5, 0.1, 0.1, 0.1])
    count, idx, st = oracle_lib.neighbors(cfg, x, r, max_nb=8)
    assert count[0] == 1 and idx[0, 0] == 3


def test_capacity_reported(oracle_lib):
    cfg, st = W.uniform_box(2, 16)
    r = _radii(cfg, st) * 3.0
    count, idx, status = oracle_lib.neighbors(cfg, st["x"], r, max_nb=16)
    assert status == oracle_lib.E_CAPACITY and count.max() > 16
