"""Ambiguity statistics through the C ABI against the oracle (Remark 1;
success criterion of Sec. IV-C).

Bars: with the same top-1 pose, best_margin within 2e-4 |T1| + 1e-6 of the
oracle's (a difference of two scores, each within the TAM tolerance) and -1
exactly when the oracle has no distinct pose; an exact tie (two
translation-symmetric rooms) gives margin 0 and bit 1 on both sides; bit 0
(a stage best within 1e-4 of tau) equal unless that best is within 1e-5 of
the band's edge; batched and plain statistics equal bit for bit.
"""
import math
import sys

import numpy as np
import pytest

import oracle
import paper_2511_01219_amd as reloc
from synth import make_config

pytestmark = pytest.mark.gpu
RES = 0.05


def _case(msg):
    print("[gpu case] " + msg, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def ctx():
    c = reloc.Context(0)
    yield c
    c.close()


def _twin_rooms(box):
    W, H = 162, 60
    occ = np.zeros((H, W), np.int8)
    occ[:2, :] = occ[-2:, :] = occ[:, :2] = occ[:, -2:] = 100
    occ[:, 80:82] = 100
    occ[10:14, 20:30] = 100
    occ[10:14, 100:110] = 100
    occ[40:44, 50:54] = 100
    occ[40:44, 130:134] = 100
    if box:
        occ[30:33, 60:63] = 100
    return occ


@pytest.mark.parametrize("box", [False, True])
def test_twin_rooms(ctx, box):
    occ = _twin_rooms(box)
    k = oracle.edt(occ)
    hyp = np.array([[40, 25], [120, 25], [60, 20], [140, 45]], np.int32)
    _, zhat = oracle.raycast(occ, hyp[:1], 360, 360, RES, 10.0)
    z = np.where(zhat[0] > 0, zhat[0], np.nan).astype(np.float32)
    _case("ambiguity twin rooms box=%s" % box)
    m = ctx.load_map(occ, RES)
    sid = ctx.set_hypotheses(m, hyp)
    poses, st = ctx.relocalize(m, sid, z, -math.pi, 2 * math.pi / 360, 0.02, 10.0, n_theta=90,
                               batch_k=4, tau=None, k_out=4)
    ref = oracle.relocalize(occ, RES, (0.0, 0.0), hyp, z, -math.pi, 2 * math.pi / 360, 0.02,
                            10.0, n_theta=90, batch_k=4, tau=None, k_out=4, kmap=k)
    if not box:
        assert st["best_margin"] == 0.0 and st["ambiguous"] & 2
        assert ref["best_margin"] == 0.0
    else:
        assert poses[0]["hyp"] == ref["poses"][0]["hyp"]
        t1 = ref["poses"][0]["tam"]
        assert abs(st["best_margin"] - ref["best_margin"]) <= 2e-4 * t1 + 1e-6
        assert not st["ambiguous"] & 2
    ctx.free_hypotheses(sid)
    ctx.unload_map(m)


@pytest.mark.parametrize("tau,K,refine", [(None, 10, 0), (0.95, 10, 0), (0.8, 16, 0),
                                          (None, 10, 3), (0.9, 7, 2)])
def test_margin_c1(ctx, tau, K, refine):
    w = make_config(1)
    k = oracle.edt(w.occ)
    hyp = oracle.sample(w.occ, k, w.resolution, n_target=300, seed=1, min_spacing=0.3,
                        robot_radius=0.21)
    _case("ambiguity c1 tau=%s K=%d refine=%d" % (tau, K, refine))
    m = ctx.load_map(w.occ, w.resolution)
    sid = ctx.set_hypotheses(m, hyp)
    kw = dict(n_theta=360, batch_k=K, tau=tau, k_out=5, refine_k=refine)
    poses, st = ctx.relocalize(m, sid, w.ranges, w.angle_min, w.angle_increment, w.range_min,
                               w.range_max, **kw)
    ref = oracle.relocalize(w.occ, w.resolution, (0.0, 0.0), hyp, w.ranges, w.angle_min,
                            w.angle_increment, w.range_min, w.range_max, kmap=k, threads=16,
                            **kw)
    if st["n_eval"] == ref["n_eval"] and poses[0]["rank"] == ref["poses"][0]["rank"]:
        t1 = ref["poses"][0]["tam"]
        if ref["best_margin"] < 0:
            assert st["best_margin"] == -1.0
        else:
            assert abs(st["best_margin"] - ref["best_margin"]) <= 2e-4 * t1 + 1e-6
    # a copy of the request without result rows still gets the statistics
    rid = ctx.prepare(m, sid, w.ranges, w.angle_min, w.angle_increment, w.range_min,
                      w.range_max, **kw)
    p0, s0 = ctx.run(rid, cap=0)
    assert p0 == [] and s0["best_margin"] == st["best_margin"]
    assert s0["ambiguous"] == st["ambiguous"]
    ctx.release(rid)
    ctx.free_hypotheses(sid)
    ctx.unload_map(m)


def test_margin_batched_equals_plain(ctx):
    w = make_config(1)
    k = oracle.edt(w.occ)
    hyp = oracle.sample(w.occ, k, w.resolution, n_target=300, seed=1, min_spacing=0.3,
                        robot_radius=0.21)
    _case("ambiguity batched vs plain")
    m = ctx.load_map(w.occ, w.resolution)
    sid = ctx.set_hypotheses(m, hyp)
    cfgs = [dict(batch_k=10, tau=0.95), dict(batch_k=10, tau=None, refine_k=2),
            dict(batch_k=7, tau=0.5, fine_metric=1)]
    scan = (w.ranges, w.angle_min, w.angle_increment, w.range_min, w.range_max)
    plain = [ctx.relocalize(m, sid, *scan, n_theta=360, k_out=5, **c) for c in cfgs]
    rids = [ctx.prepare(m, sid, *scan, n_theta=360, k_out=5, **c) for c in cfgs]
    batched = ctx.run_batch(rids, cap=5)
    for r in rids:
        ctx.release(r)
    for (pa, sa), (pb, sb) in zip(plain, batched):
        assert pa == pb
        assert sa["best_margin"] == sb["best_margin"] and sa["ambiguous"] == sb["ambiguous"]
    ctx.free_hypotheses(sid)
    ctx.unload_map(m)
