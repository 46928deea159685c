"""Dense sweeps through the C ABI (Sec. IV Case 1: Fig. 7's SMAD map over
positions and Fig. 8's metrics over a translation x rotation lattice).

Bars:
  * coarse map over every feasible cell of plain-small: bit-exact against
    the oracle on a seeded 5 % sample (plus the cell of the true pose), the
    order the stable ascending (score, index) permutation;
  * fine metrics at explicit poses (a 0.1 m x 10 deg lattice of 15 x 36
    poses around the truth, and random poses including the map's corner
    cells): within 1e-4 relative + 1e-7 of the oracle's TAM on the Ng grid;
  * cells outside the map and heading indices outside [0, Ng) are refused.
"""
import math
import sys

import numpy as np
import pytest

import oracle
import paper_2511_01219_amd as reloc
from synth import make_config

pytestmark = pytest.mark.gpu

V_RTOL, V_ATOL = 1e-4, 1e-7


def _case(msg):
    print("[gpu case] " + msg, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def world():
    w = make_config(1)
    k = oracle.edt(w.occ)
    ctx = reloc.Context(0)
    m = ctx.load_map(w.occ, w.resolution, w.origin)
    yield w, k, ctx, m
    ctx.unload_map(m)
    ctx.close()


def _scan(w):
    return dict(ranges=w.ranges, angle_min=w.angle_min, angle_increment=w.angle_increment,
                range_min=w.range_min, range_max=w.range_max)


def test_coarse_map_all_free_cells(world):
    w, k, ctx, m = world
    F = (w.occ >= 0) & (w.occ < 65) & (k >= 18)
    ys, xs = np.nonzero(F)
    cells = np.stack([xs, ys], 1).astype(np.int32)
    n = len(cells)
    _case("coarse map over %d free cells" % n)
    sid = ctx.set_hypotheses(m, cells)
    rid = ctx.prepare(m, sid, **_scan(w), n_theta=360, batch_k=10)
    sc, sh, order, st = ctx.coarse_scores(rid, n)
    assert st["n_hyp"] == n and st["rays"] == n * 480
    assert (order == np.lexsort((np.arange(n), sc))).all()
    true_cell = np.floor((np.asarray(w.pose[:2]) - np.asarray(w.origin)) / w.resolution)
    near = int(np.argmin(np.abs(cells - true_cell).sum(1)))
    sub = np.unique(np.append(np.random.default_rng([1, 7]).choice(n, n // 20, replace=False),
                              near))
    pr = oracle.prep(w.ranges, w.angle_min, w.angle_increment, w.resolution,
                     range_min=w.range_min, range_max=w.range_max, n_theta=360)
    _, zhat = oracle.raycast(w.occ, cells[sub], pr["Ns"], pr["Ng"], w.resolution, w.range_max,
                             threads=16)
    ref, ram = oracle.smad(zhat, pr, threads=16)
    assert (sc[sub].view(np.uint64) == ref.view(np.uint64)).all()
    assert (sh[sub] == ram).all()
    # a smaller buffer than the set is refused
    with pytest.raises(reloc.RelocError):
        ctx.coarse_scores(rid, n - 1)
    ctx.release(rid)
    ctx.free_hypotheses(sid)


@pytest.mark.parametrize("n", [1, 300, 512, 513, 1023, 1024, 1025, 4097, 65536, 65537, 200000,
                               262145])
def test_order_with_ties_across_tiles(world, n):
    """The stable SMAD order at sizes around the 512-key limit of the
    ranked small tiles and the 1024-key tiles of the sort, and around the
    runs of its merge levels, with many exact ties (37 cells repeated, so equal scans give
    equal SMAD): the order is the stable one (ties by index) of the returned
    scores; with no coarse metric (every key zero) it is the identity."""
    w, k, ctx, m = world
    F = (w.occ >= 0) & (w.occ < 65) & (k >= 18)
    ys, xs = np.nonzero(F)
    rng = np.random.default_rng([n, 3])
    few = rng.choice(len(xs), 37, replace=False)
    pick = rng.choice(few, n)
    cells = np.stack([xs[pick], ys[pick]], 1).astype(np.int32)
    sid = ctx.set_hypotheses(m, cells)
    for cm in (0, 3):
        _case("order with ties: n %d, coarse metric %d" % (n, cm))
        rid = ctx.prepare(m, sid, **_scan(w), n_theta=360, batch_k=10, coarse_metric=cm)
        sc, sh, order, st = ctx.coarse_scores(rid, n)
        assert (order == np.lexsort((np.arange(n), sc))).all()
        if cm == 3:
            assert (order == np.arange(n)).all()
        else:
            assert len(np.unique(sc)) <= 37
        ctx.release(rid)
    ctx.free_hypotheses(sid)


def _fine_prep(w, Ng):
    return oracle.prep(w.ranges, w.angle_min, w.angle_increment, w.resolution,
                       range_min=w.range_min, range_max=w.range_max, n_theta=Ng)


@pytest.mark.parametrize("fine", [0, 2])
def test_translation_rotation_lattice(world, fine):
    w, k, ctx, m = world
    cells = np.array([[10, 10]], np.int32)
    sid = ctx.set_hypotheses(m, cells)
    rid = ctx.prepare(m, sid, **_scan(w), n_theta=360, batch_k=10, fine_metric=fine)
    Ng = 1440
    c0 = np.floor((np.asarray(w.pose[:2]) - np.asarray(w.origin)) / w.resolution).astype(int)
    g0 = int(round(w.pose[2] * Ng / (2 * math.pi))) % Ng
    xy, g = [], []
    for t in range(-7, 8):                 # 0.1 m steps along x (2 cells)
        for j in range(36):                # 10 degree steps (40 direction steps)
            xy.append((c0[0] + 2 * t, c0[1]))
            g.append((g0 + 40 * j) % Ng)
    xy = np.array(xy, np.int32)
    g = np.array(g, np.int32)
    _case("pose lattice 15 x 36, fine metric %d" % fine)
    v, ms = ctx.score_poses(rid, xy, g)
    assert len(v) == 540 and ms > 0
    ref = oracle.tam(k, w.resolution, _fine_prep(w, Ng), xy, g, threads=16)[:, oracle.FINE_COL[fine]]
    assert (np.abs(v.astype(np.float64) - ref) <= V_RTOL * np.abs(ref) + V_ATOL).all()
    ctx.release(rid)
    ctx.free_hypotheses(sid)


@pytest.mark.parametrize("n", [1, 17, 333])
@pytest.mark.parametrize("fine", [0, 1, 3])
def test_random_poses(world, n, fine):
    w, k, ctx, m = world
    H, W = w.occ.shape
    sid = ctx.set_hypotheses(m, np.array([[10, 10]], np.int32))
    rid = ctx.prepare(m, sid, **_scan(w), n_theta=360, batch_k=10, fine_metric=fine)
    rng = np.random.default_rng([n, fine])
    xy = np.stack([rng.integers(0, W, n), rng.integers(0, H, n)], 1).astype(np.int32)
    xy[0] = (0, 0)
    if n > 1:
        xy[1] = (W - 1, H - 1)
    g = rng.integers(0, 1440, n).astype(np.int32)
    _case("score %d random poses, fine %d" % (n, fine))
    v, _ = ctx.score_poses(rid, xy, g)
    ref = oracle.tam(k, w.resolution, _fine_prep(w, 1440), xy, g)[:, oracle.FINE_COL[fine]]
    assert (np.abs(v.astype(np.float64) - ref) <= V_RTOL * np.abs(ref) + V_ATOL).all()
    ctx.release(rid)
    ctx.free_hypotheses(sid)


@pytest.mark.parametrize("fine", [0, 1, 2, 3])
def test_random_poses_far_cells(world, fine):
    """Every fine metric at random poses of an open hall, where most
    endpoints lie 128 or more cells from any obstacle (the escape path of
    the TAM planes, in the full-sum class too), against the oracle."""
    _, _, ctx, _ = world
    W, H = 700, 600
    occ = np.zeros((H, W), np.int8)
    occ[0, :] = occ[H - 1, :] = 100
    occ[:, 0] = occ[:, W - 1] = 100
    occ[280:300, 150:200] = 100
    k = oracle.edt(occ)
    m = ctx.load_map(occ, 0.05)
    sid = ctx.set_hypotheses(m, np.array([[350, 300]], np.int32))
    inc = 2 * math.pi / 360
    z = np.full(360, 4.0, np.float32)
    z[::3] = 12.0
    z[1::3] = 25.0
    rid = ctx.prepare(m, sid, z, -math.pi, inc, 0.02, 40.0, n_theta=360, batch_k=10,
                      fine_metric=fine)
    rng = np.random.default_rng([7, fine])
    n = 200
    xy = np.stack([rng.integers(1, W - 1, n), rng.integers(1, H - 1, n)], 1).astype(np.int32)
    g = rng.integers(0, 360, n).astype(np.int32)
    _case("score %d random poses in an open hall, fine %d" % (n, fine))
    v, _ = ctx.score_poses(rid, xy, g)
    pr = oracle.prep(z, -math.pi, inc, 0.05, range_min=0.02, range_max=40.0, n_theta=360)
    ref = oracle.tam(k, 0.05, pr, xy, g)[:, oracle.FINE_COL[fine]]
    assert (np.abs(v.astype(np.float64) - ref) <= V_RTOL * np.abs(ref) + V_ATOL).all()
    ctx.release(rid)
    ctx.free_hypotheses(sid)
    ctx.unload_map(m)


def test_pose_arguments_checked(world):
    w, k, ctx, m = world
    H, W = w.occ.shape
    sid = ctx.set_hypotheses(m, np.array([[10, 10]], np.int32))
    rid = ctx.prepare(m, sid, **_scan(w), n_theta=360, batch_k=10)
    for xy, g in (([[W, 0]], [0]), ([[0, -1]], [0]), ([[3, 3]], [1440]), ([[3, 3]], [-1])):
        with pytest.raises(reloc.RelocError) as ei:
            ctx.score_poses(rid, np.array(xy, np.int32), np.array(g, np.int32))
        assert ei.value.code == reloc.E_INVALID
    v, ms = ctx.score_poses(rid, np.zeros((0, 2), np.int32), np.zeros(0, np.int32))
    assert len(v) == 0
    ctx.release(rid)
    ctx.free_hypotheses(sid)
