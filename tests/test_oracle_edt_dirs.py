"""Oracle pins: EDT (lookup table of Sec. III-A, MinDistToObstacle) and the
direction table.

EDT pins: brute force over every occupied cell on micro-maps, and
scipy.ndimage.distance_transform_edt (an exact EDT to the nearest zero, the
same definition) at workload scale, compared through the feature indices so
the squared distance is exact.
Direction pins: axis directions, unit length, angle accuracy, and grid
independence of a direction (same reduced turn fraction -> same vector).
"""
import math

import numpy as np
import pytest
from scipy import ndimage

import oracle
from synth import make_micro, rasterize, rooms_map, warehouse_map


@pytest.mark.parametrize("seed", range(8))
def test_edt_separable_equals_brute(seed):
    occ = make_micro(seed, 23 + seed, 17 + 2 * seed, n_boxes=3 + seed % 3,
                     p_unknown=0.1 if seed % 2 else 0.0)
    a = oracle.edt(occ, brute=True)
    b = oracle.edt(occ)
    assert (a == b).all()
    assert (a[occ >= 65] == 0).all()
    assert (a[occ < 65] > 0).all()


def test_edt_single_obstacle_closed_form():
    occ = np.zeros((9, 13), dtype=np.int8)
    occ[4, 6] = 100
    k = oracle.edt(occ)
    yy, xx = np.mgrid[0:9, 0:13]
    assert (k == (xx - 6) ** 2 + (yy - 4) ** 2).all()


def test_edt_empty_map():
    k = oracle.edt(np.zeros((5, 7), dtype=np.int8))
    assert (k == -1).all()


def test_edt_unknown_cells_are_not_obstacles():
    occ = np.zeros((5, 9), dtype=np.int8)
    occ[2, 0] = 100
    occ[2, 4] = -1
    k = oracle.edt(occ)
    assert k[2, 4] == 16 and k[2, 8] == 64


def _scipy_k(occ):
    _, idx = ndimage.distance_transform_edt(occ < 65, return_indices=True)
    yy, xx = np.mgrid[0:occ.shape[0], 0:occ.shape[1]]
    return (yy - idx[0]).astype(np.int64) ** 2 + (xx - idx[1]).astype(np.int64) ** 2


def test_edt_matches_scipy_rooms():
    occ = rasterize(rooms_map(np.random.default_rng([1, 0])))
    assert (oracle.edt(occ) == _scipy_k(occ)).all()


def test_edt_matches_scipy_warehouse_500():
    occ = rasterize(warehouse_map(np.random.default_rng([7, 0]), 500, 500))
    assert (oracle.edt(occ) == _scipy_k(occ)).all()


@pytest.mark.parametrize("Ng", [360, 480, 1440, 2880, 5760])
def test_dirs_axes_and_length(Ng):
    U = oracle.dirs(Ng).astype(np.int64)
    s = 1 << 20
    assert tuple(U[0]) == (s, 0)
    assert tuple(U[Ng // 4]) == (0, s)
    assert tuple(U[Ng // 2]) == (-s, 0)
    assert tuple(U[3 * Ng // 4]) == (0, -s)
    n = np.sqrt((U.astype(np.float64) ** 2).sum(1))
    assert np.abs(n - s).max() <= 1.0
    ang = np.arctan2(U[:, 1], U[:, 0])
    ref = 2 * np.pi * np.arange(Ng) / Ng
    err = np.abs((ang - ref + np.pi) % (2 * np.pi) - np.pi)
    assert err.max() < 1.5e-6


def test_dirs_grid_independent():
    a = oracle.dirs(480)
    b = oracle.dirs(1440)
    c = oracle.dirs(2880)
    assert (b[::3] == a).all()
    assert (c[::2] == b).all()


@pytest.mark.parametrize("Ng", [480, 1440])
def test_dirs_quarter_turn_symmetry(Ng):
    # for these grids the rounded table is exactly symmetric under a quarter
    # turn, which the rotation tests of the ray cast and TAM rely on
    U = oracle.dirs(Ng)
    q = Ng // 4
    rot = np.stack([-U[:, 1], U[:, 0]], 1)
    assert (np.roll(U, -q, axis=0) == rot).all()
