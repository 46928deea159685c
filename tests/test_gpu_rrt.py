"""Traversability-constrained RRT sampling (Algorithm 1) through the C ABI:
the library (k-d tree NearestNode) against the oracle (brute force), bit
for bit: every tree node, every parent, the hypothesis cells and the run's
counts. The sampler runs on the host copy of a resident map, so it needs a
context (a device); the full-size warehouse map is checked through
invariants (the oracle's brute-force NearestNode is too slow there).
"""
import math
import sys
import time

import numpy as np
import pytest

import oracle
import paper_2511_01219_amd as reloc
from synth import make_config, make_micro

pytestmark = pytest.mark.gpu


def _case(msg):
    print("[gpu case] " + msg, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def ctx():
    c = reloc.Context(0)
    yield c
    c.close()


def _run_both(ctx, occ, res, origin, p0, **kw):
    k = oracle.edt(occ)
    ref = oracle.rrt(occ, k, res, p0=p0, origin=origin, **kw)
    m = ctx.load_map(occ, res, origin)
    cap = len(ref["nodes"]) + 8
    sid, n, info, nodes, par = ctx.sample_rrt(m, p0, tree_cap=cap, **kw)
    cells = ctx.read_hypotheses(sid)
    ctx.free_hypotheses(sid)
    ctx.unload_map(m)
    return ref, (n, info, nodes, par, cells)


def _assert_equal(ref, got):
    n, info, nodes, par, cells = got
    assert info["rounds"] == ref["rounds"] and info["attempts"] == ref["attempts"]
    assert info["nodes"] == len(ref["nodes"]) and info["n_sampling"] == ref["n_sampling"]
    assert (nodes.view(np.uint64) == ref["nodes"].view(np.uint64)).all()
    assert (par == ref["parent"]).all()
    assert n == len(ref["cells"]) and (cells == ref["cells"]).all()


@pytest.mark.parametrize("seed", [1, 7])
def test_rrt_plain_small_bit_exact(ctx, seed):
    w = make_config(1)
    _case("rrt plain-small seed %d" % seed)
    ref, got = _run_both(ctx, w.occ, w.resolution, w.origin, w.pose[:2], rho=0.3, seed=seed)
    _assert_equal(ref, got)


def test_rrt_micro_doorway_bit_exact(ctx):
    occ = np.zeros((64, 126), np.int8)
    occ[:2, :] = occ[-2:, :] = occ[:, :2] = occ[:, -2:] = 100
    occ[:, 62:66] = 100
    occ[24:40, 62:66] = 0
    rng = np.random.default_rng(3)
    for _ in range(6):
        x, y = rng.integers(6, 118), rng.integers(6, 56)
        occ[y:y + 3, x:x + 3] = 100
    _case("rrt doorway map")
    ref, got = _run_both(ctx, occ, 0.05, (1.5, -2.0), (1.5 + 30 * 0.05, -2.0 + 32 * 0.05),
                         rho=0.25, eta_max=0.5, seed=11)
    _assert_equal(ref, got)


def test_rrt_warehouse_crop_bit_exact(ctx):
    w = make_config(2)
    occ = np.ascontiguousarray(w.occ[200:600, 100:500])
    k = oracle.edt(occ)
    ys, xs = np.nonzero((occ == 0) & (k >= 18))
    p0 = ((xs[len(xs) // 3] + 0.5) * 0.05, (ys[len(ys) // 3] + 0.5) * 0.05)
    _case("rrt warehouse crop 400x400")
    ref, got = _run_both(ctx, occ, 0.05, (0.0, 0.0), p0, rho=0.3, seed=2)
    _assert_equal(ref, got)


def test_rrt_warehouse_full_invariants(ctx):
    w = make_config(2)
    k = oracle.edt(w.occ)
    m = ctx.load_map(w.occ, w.resolution, w.origin)
    _case("rrt warehouse 2000x2000")
    t0 = time.perf_counter()
    sid, n, info = ctx.sample_rrt(m, w.pose[:2], rho=0.3, seed=2)
    dt = time.perf_counter() - t0
    print("[rrt] 2000x2000: %d hypotheses, %d nodes, %d rounds, %d attempts in %.2f s"
          % (n, info["nodes"], info["rounds"], info["attempts"], dt), flush=True)
    cells = ctx.read_hypotheses(sid)
    F = (w.occ >= 0) & (w.occ < 65) & (k >= 18)
    assert F[cells[:, 1], cells[:, 0]].all()
    assert len(np.unique(cells[:, 1] * 2000 + cells[:, 0])) == n
    # hypotheses at least about rho apart in voxel terms: one per 0.3 m voxel
    vox = np.floor((cells + 0.5) * 0.05 / 0.3).astype(np.int64)
    assert len(np.unique(vox[:, 1] * 10000 + vox[:, 0])) >= 0.9 * n
    assert n > 10000 and info["rounds"] >= 2
    ctx.free_hypotheses(sid)
    ctx.unload_map(m)


def test_rrt_set_relocalizes(ctx):
    w = make_config(1)
    k = oracle.edt(w.occ)
    m = ctx.load_map(w.occ, w.resolution, w.origin)
    sid, n, info = ctx.sample_rrt(m, w.pose[:2], rho=0.3, seed=1)
    hyp = ctx.read_hypotheses(sid)
    _case("relocalize on an RRT set of %d" % n)
    poses, st = ctx.relocalize(m, sid, w.ranges, w.angle_min, w.angle_increment, w.range_min,
                               w.range_max, n_theta=360, batch_k=10, tau=None, k_out=5)
    ref = oracle.relocalize(w.occ, w.resolution, w.origin, hyp, w.ranges, w.angle_min,
                            w.angle_increment, w.range_min, w.range_max, n_theta=360,
                            batch_k=10, tau=None, k_out=5, kmap=k, threads=16)
    b, rb = poses[0], ref["poses"][0]
    assert b["hyp"] == rb["hyp"] or abs(b["tam"] - rb["tam"]) <= 2e-4 * rb["tam"]
    d = math.hypot(b["x"] - w.pose[0], b["y"] - w.pose[1])
    assert d < 0.5
    ctx.free_hypotheses(sid)
    ctx.unload_map(m)


@pytest.mark.parametrize("bad", [
    dict(p0=(float("nan"), 0.0)),
    dict(p0=(0.0, float("inf"))),
    dict(rho=float("nan")),
    dict(rho=float("inf")),
    dict(eta_max=float("inf")),
    dict(rho=0.0),
    dict(rho=1e-4),             # finite but below the 0.05 m cell: ~1e12 attempts per round
    dict(rho=0.0499),
    dict(eta_max=0.1),          # below the robot radius
    dict(eps_gain=-1),
    dict(max_rounds=0),
])
def test_rrt_refuses_bad_parameters(ctx, bad):
    w = make_config(1)
    m = ctx.load_map(w.occ, w.resolution, w.origin)
    try:
        _case("RRT refuses %r" % (bad,))
        kw = dict(p0=w.pose[:2], rho=0.3, seed=1)
        kw.update(bad)
        before = ctx.bytes
        with pytest.raises(reloc.RelocError) as ei:
            ctx.sample_rrt(m, **kw)
        assert ei.value.code == reloc.E_INVALID, str(ei.value)
        assert ctx.bytes == before
    finally:
        ctx.unload_map(m)
