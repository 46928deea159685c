"""Oracle pins: the ambiguity statistics (Remark 1, eq. 5; success criterion
of Sec. IV-C).

* a map with two identical rooms side by side (a translation symmetry):
  the scan's true pose and its twin one room over score the same, so the
  best distinct pose ties the top-1 (margin 0, bit 1 set);
* breaking the symmetry (a box in the scanned room: its beams end in free
  space at the twin pose) gives a positive margin;
* the distinct set follows the criterion exactly: poses 0.45 m away with
  the same heading are not distinct, 0.5 m away are, and a 30 deg turn is;
* bit 0 marks a batch best within 1e-4 of tau.
"""
import math

import numpy as np

import oracle

RES = 0.05


def _twin_rooms(box=False):
    W, H = 162, 60
    occ = np.zeros((H, W), np.int8)
    occ[:2, :] = occ[-2:, :] = occ[:, :2] = occ[:, -2:] = 100
    occ[:, 80:82] = 100
    occ[10:14, 20:30] = 100
    occ[10:14, 100:110] = 100                      # the twin of the box above
    occ[40:44, 50:54] = 100
    occ[40:44, 130:134] = 100
    if box:
        occ[30:33, 60:63] = 100                    # in the scanned room only
    return occ


def _scan_from(occ, cell, Ns=360):
    _, zhat = oracle.raycast(occ, np.array([cell], np.int32), Ns, Ns, RES, 10.0)
    z = np.where(zhat[0] > 0, zhat[0], np.nan).astype(np.float32)
    return z, -math.pi, 2 * math.pi / Ns


def test_twin_rooms_tie_and_break():
    for box, tied in ((False, True), (True, False)):
        occ = _twin_rooms(box)
        k = oracle.edt(occ)
        hyp = np.array([[40, 25], [120, 25], [60, 20], [140, 45]], np.int32)
        z, amin, inc = _scan_from(occ, (40, 25))
        res = oracle.relocalize(occ, RES, (0.0, 0.0), hyp, z, amin, inc, 0.02, 10.0,
                                n_theta=90, batch_k=4, tau=None, k_out=4, kmap=k, keep=True)
        t = res["tstar"]
        if tied:
            assert res["best_margin"] == 0.0 and res["ambiguous"] & 2
        else:
            assert res["best_margin"] > 1e-3 and not res["ambiguous"] & 2
        assert res["poses"][0]["hyp"] in (0, 1)
        assert t.max() == res["poses"][0]["tam"]


def test_distinct_criterion_boundaries():
    hyp = np.array([[10, 10], [19, 10], [20, 10], [10, 10]], np.int32)
    order = np.arange(4)
    # rank 0 is the top-1; rank 1 is 9 cells (0.45 m) away, rank 2 10 cells
    # (0.5 m) away, rank 3 the same cell turned by exactly 30 deg
    Ng = 360
    tstar = np.array([0.9, 0.89, 0.5, 0.3])
    g = np.array([0, 0, 0, 30])
    dxy = np.zeros((4, 2), np.int64)
    a = oracle.ambiguity(order, tstar, dxy, g, hyp, Ng, RES, 4, None)
    assert a["top"] == 0 and abs(a["best_margin"] - 0.4) < 1e-15
    g2 = np.array([0, 0, 0, 29])
    t2 = np.array([0.9, 0.89, 0.5, 0.8])
    b = oracle.ambiguity(order, t2, dxy, g2, hyp, Ng, RES, 4, None)
    assert abs(b["best_margin"] - 0.4) < 1e-15           # 29 steps: not distinct
    g3 = np.array([0, 0, 0, 30])
    c = oracle.ambiguity(order, t2, dxy, g3, hyp, Ng, RES, 4, None)
    assert abs(c["best_margin"] - 0.1) < 1e-15           # 30 steps: distinct
    none = oracle.ambiguity(order[:2], tstar[:2], dxy[:2], g[:2], hyp, Ng, RES, 4, None)
    assert none["best_margin"] == -1.0 and none["ambiguous"] == 0


def test_stop_fragility_bit():
    hyp = np.array([[0, 0], [50, 0], [100, 0], [150, 0]], np.int32)
    tstar = np.array([0.2, 0.94995, 0.3, 0.1])
    dxy = np.zeros((4, 2), np.int64)
    g = np.zeros(4, np.int64)
    a = oracle.ambiguity(np.arange(4), tstar, dxy, g, hyp, 360, RES, 2, 0.95)
    assert a["ambiguous"] & 1
    b = oracle.ambiguity(np.arange(4), tstar, dxy, g, hyp, 360, RES, 2, 0.96)
    assert not b["ambiguous"] & 1
