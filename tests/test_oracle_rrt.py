"""Oracle pins: traversability-constrained RRT sampling (Algorithm 1,
Sec. III-A items 1-7, Remark 4).

* N_sampling = ceil(W H r^2 / rho^2) (Remark 4);
* every node lies in a feasible cell (known free, d_obs >= r_robot) of the
  8-connected feasible component of p0's cell (R(p0); consecutive points of
  a traversability check are at most r/2 apart), parents precede children;
* every edge is at most AdaptiveExpandDist(parent) long, recomputed from
  the EDT with the piecewise rule of item 5;
* the hypothesis cells are the cells of the first node of each rho-voxel,
  in node order, without repeats (VoxelDownsample, item 7);
* two rooms joined by a doorway narrower than 2 r_robot: no node in the
  second room; a wide doorway: the second room is covered;
* an empty room is covered: every feasible cell lies within rho * sqrt(2)
  of a hypothesis; eps_gain = huge stops after one round of N_sampling
  attempts; results are deterministic and depend on the seed.
"""
import math

import numpy as np
import pytest
from scipy import ndimage

import oracle
from synth import make_config, make_micro

RES = 0.05


def _room(W=120, H=90, wall=2):
    occ = np.zeros((H, W), np.int8)
    occ[:wall, :] = occ[-wall:, :] = occ[:, :wall] = occ[:, -wall:] = 100
    return occ


def _feasible(occ, kmap, rr=0.21):
    q = rr / RES
    Kr = math.ceil(q * q - 1e-9)
    return (occ >= 0) & (occ < 65) & (kmap >= Kr)


def _cells(xy, origin=(0.0, 0.0)):
    return np.floor((xy - np.asarray(origin)) / RES).astype(np.int64)


def _eta(kmap, xy, rr=0.21, eta_max=0.6):
    c = _cells(xy)
    k = kmap[c[:, 1], c[:, 0]].astype(np.float64)
    d = np.sqrt(k) * RES
    return np.where(d >= 2 * rr, eta_max,
                    np.where(d <= rr, rr, rr + (eta_max - rr) * (d - rr) / rr))


@pytest.mark.parametrize("shape,rho", [((200, 200), 0.3), ((90, 120), 0.25), ((77, 53), 1.0)])
def test_n_sampling_closed_form(shape, rho):
    H, W = shape
    occ = _room(W, H)
    k = oracle.edt(occ)
    r = oracle.rrt(occ, k, RES, p0=(W * RES / 2, H * RES / 2), rho=rho, max_rounds=1)
    assert r["n_sampling"] == math.ceil(W * H * RES * RES / (rho * rho) - 1e-9)
    assert r["rounds"] == 1 and r["attempts"] == r["n_sampling"]


@pytest.mark.parametrize("seed", [0, 1, 2])
def test_nodes_feasible_reachable_and_edges_bounded(seed):
    occ = make_micro(seed + 40, 110, 90, n_boxes=14)
    k = oracle.edt(occ)
    F = _feasible(occ, k)
    ys, xs = np.nonzero(F)
    i0 = len(xs) // 2
    p0 = ((xs[i0] + 0.5) * RES, (ys[i0] + 0.5) * RES)
    r = oracle.rrt(occ, k, RES, p0=p0, seed=seed)
    nodes, par = r["nodes"], r["parent"]
    c = _cells(nodes)
    assert F[c[:, 1], c[:, 0]].all()
    lab, _ = ndimage.label(F, structure=np.ones((3, 3)))
    assert (lab[c[:, 1], c[:, 0]] == lab[ys[i0], xs[i0]]).all()
    assert par[0] == -1 and (par[1:] < np.arange(1, len(par))).all() and (par[1:] >= 0).all()
    L = np.hypot(*(nodes[1:] - nodes[par[1:]]).T)
    eta = _eta(k, nodes[par[1:]])
    assert (L > 0).all() and (L <= eta * (1 + 1e-12)).all()
    # early expansions reach eta (random points far from a small tree); once
    # the tree is dense most random points are within eta and taken as is
    assert np.any(np.abs(L - eta) <= 1e-9 * eta) and np.any(L < eta * (1 - 1e-6))


@pytest.mark.parametrize("rho", [0.3, 0.55])
def test_voxel_representatives(rho):
    w = make_config(1)
    k = oracle.edt(w.occ)
    r = oracle.rrt(w.occ, k, w.resolution, p0=w.pose[:2], origin=w.origin, rho=rho, seed=3)
    nodes = r["nodes"]
    vox = np.floor((nodes - np.asarray(w.origin)) / rho).astype(np.int64)
    key = vox[:, 1] * 100000 + vox[:, 0]
    _, first = np.unique(key, return_index=True)
    first = np.sort(first)
    c = _cells(nodes[first], w.origin)
    ckey = c[:, 1] * 100000 + c[:, 0]
    _, cf = np.unique(ckey, return_index=True)
    want = c[np.sort(cf)]
    assert (r["cells"] == want).all()


@pytest.mark.parametrize("door,reach", [(6, False), (16, True)])
def test_doorway_reachability(door, reach):
    # two 60 x 60 rooms side by side; the 4-cell wall has a doorway of
    # `door` cells; r_robot = 0.21 m needs 2 * 4.2 + 1 >= 9.4 cells
    W, H = 126, 64
    occ = _room(W, H)
    occ[:, 62:66] = 100
    y0 = 32 - door // 2
    occ[y0:y0 + door, 62:66] = 0
    k = oracle.edt(occ)
    r = oracle.rrt(occ, k, RES, p0=(30 * RES, 32 * RES), rho=0.3, seed=5)
    right = r["cells"][:, 0] >= 66
    assert right.any() == reach
    if reach:
        assert right.sum() >= 0.8 * (~right).sum()


def test_empty_room_covered():
    occ = _room(100, 80)
    k = oracle.edt(occ)
    rho = 0.3
    r = oracle.rrt(occ, k, RES, p0=(2.5, 2.0), rho=rho, seed=9)
    F = _feasible(occ, k)
    ys, xs = np.nonzero(F)
    P = (r["cells"] + 0.5) * RES
    Q = np.stack([xs + 0.5, ys + 0.5], 1) * RES
    d = np.min(np.hypot(Q[:, None, 0] - P[None, :, 0], Q[:, None, 1] - P[None, :, 1]), axis=1)
    assert d.max() <= rho * math.sqrt(2) + RES


def test_gain_stop_determinism_seed():
    w = make_config(1)
    k = oracle.edt(w.occ)
    kw = dict(p0=w.pose[:2], origin=w.origin, rho=0.3)
    a = oracle.rrt(w.occ, k, w.resolution, seed=1, **kw)
    b = oracle.rrt(w.occ, k, w.resolution, seed=1, **kw)
    c = oracle.rrt(w.occ, k, w.resolution, seed=2, **kw)
    assert (a["nodes"] == b["nodes"]).all() and (a["cells"] == b["cells"]).all()
    assert len(a["nodes"]) != len(c["nodes"]) or (a["nodes"] != c["nodes"]).any()
    one = oracle.rrt(w.occ, k, w.resolution, seed=1, eps_gain=10 ** 9, **kw)
    assert one["rounds"] == 1 and one["attempts"] == one["n_sampling"]
    assert a["rounds"] > 1
    # a smaller node budget stops early with a prefix of the tree
    cap = oracle.rrt(w.occ, k, w.resolution, seed=1, max_nodes=500, **kw)
    assert len(cap["nodes"]) == 500 and (cap["nodes"] == a["nodes"][:500]).all()
