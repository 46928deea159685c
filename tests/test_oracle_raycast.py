"""Oracle pins: panoramic ray cast of the synthetic scan (eq. 13-14).

* the crossing-merge traversal equals a brute-force exact slab test against
  every occupied cell (micro-maps, grids with exact 45-degree rays that cross
  cell corners);
* closed form: in an empty rectangular room the range is the distance from
  the cell centre to the wall's inner face along the quantized direction,
  within 2 ulp, and the hit is the wall cell at the intersection point;
* a quarter-turn of the map maps hits and ranges onto the rotated directions;
* the Chebyshev cut-off never changes a result (range_max changes only which
  ranges are zeroed).
"""
import math

import numpy as np
import pytest

import oracle
from synth import make_micro


def _free_cells(occ, n, seed=0):
    ys, xs = np.nonzero((occ >= 0) & (occ < 65))
    rng = np.random.default_rng(seed)
    pick = rng.choice(len(xs), size=min(n, len(xs)), replace=False)
    return np.stack([xs[pick], ys[pick]], 1).astype(np.int32)


@pytest.mark.parametrize("seed,Ns,Ng", [(0, 480, 1440), (1, 360, 360), (2, 64, 64),
                                        (3, 96, 288), (4, 1440, 1440), (5, 8, 8)])
def test_traversal_equals_brute_force(seed, Ns, Ng):
    occ = make_micro(seed, 26, 21, n_boxes=6, p_unknown=0.05)
    hyp = _free_cells(occ, 25, seed)
    h1, r1 = oracle.raycast(occ, hyp, Ns, Ng, 0.05, 12.0)
    h2, r2 = oracle.raycast(occ, hyp, Ns, Ng, 0.05, 12.0, brute=True)
    assert (h1 == h2).all()
    assert (r1.view(np.uint32) == r2.view(np.uint32)).all()


def test_brute_force_with_holes_in_outer_wall():
    # rays that leave the map through gaps: exit rule and corner exits
    occ = make_micro(11, 20, 20, n_boxes=4)
    occ[0, 5:9] = 0
    occ[7:12, -1] = 0
    occ[-1, -1] = 0
    occ[0, 0] = 0
    hyp = _free_cells(occ, 40, 3)
    for Ns in (8, 64, 360):
        h1, r1 = oracle.raycast(occ, hyp, Ns, Ns, 0.05, 12.0)
        h2, r2 = oracle.raycast(occ, hyp, Ns, Ns, 0.05, 12.0, brute=True)
        assert (h1 == h2).all() and (r1.view(np.uint32) == r2.view(np.uint32)).all()
        assert (r1[h1 < 0] == 0).all() and (r1[h1 >= 0] > 0).all()


def test_analytic_rectangular_room():
    W, H, res = 61, 47, 0.05
    occ = np.zeros((H, W), dtype=np.int8)
    occ[0, :] = occ[-1, :] = 100
    occ[:, 0] = occ[:, -1] = 100
    Ns = Ng = 720
    U = oracle.dirs(Ng).astype(np.float64)
    hyp = np.array([[5, 7], [30, 23], [55, 40], [1, 1], [59, 45], [12, 33]],
                   dtype=np.int32)
    hit, rng = oracle.raycast(occ, hyp, Ns, Ng, res, 50.0)
    nrm = np.sqrt((U ** 2).sum(1))
    c, s = U[:, 0] / nrm, U[:, 1] / nrm
    checked = 0
    for h, (ix, iy) in enumerate(hyp):
        px, py = ix + 0.5, iy + 0.5
        for j in range(Ns):
            cand = []
            if c[j] > 0: cand.append(((W - 1 - px) / c[j], "x"))
            if c[j] < 0: cand.append(((px - 1) / -c[j], "x"))
            if s[j] > 0: cand.append(((H - 1 - py) / s[j], "y"))
            if s[j] < 0: cand.append(((py - 1) / -s[j], "y"))
            cand.sort()
            t = cand[0][0]
            ref = t * res
            assert abs(rng[h, j] - ref) <= 2.0 * np.spacing(np.float32(ref)), (h, j)
            if len(cand) > 1 and abs(cand[1][0] - t) < 1e-9:
                continue          # corner: tie rule decides the cell
            qx, qy = px + t * c[j], py + t * s[j]
            other = qy if cand[0][1] == "x" else qx
            if abs(other - round(other)) < 1e-9:
                continue          # the hit point is a grid corner: tie rule
            ex = W - 1 if (cand[0][1] == "x" and c[j] > 0) else (
                0 if cand[0][1] == "x" else int(math.floor(qx)))
            ey = H - 1 if (cand[0][1] == "y" and s[j] > 0) else (
                0 if cand[0][1] == "y" else int(math.floor(qy)))
            assert hit[h, j] == ey * W + ex, (h, j)
            checked += 1
    assert checked > 3000


def _rot90(occ):
    # world rotation by +90 degrees: cell (x, y) -> (H-1-y, x)
    return np.ascontiguousarray(occ.T[:, ::-1])


@pytest.mark.parametrize("seed", [0, 1, 2])
def test_quarter_turn(seed):
    occ = make_micro(20 + seed, 30, 22, n_boxes=6)
    H, W = occ.shape
    occ_r = _rot90(occ)
    hyp = _free_cells(occ, 20, seed)
    hyp_r = np.stack([H - 1 - hyp[:, 1], hyp[:, 0]], 1).astype(np.int32)
    Ns = 480
    h1, r1 = oracle.raycast(occ, hyp, Ns, Ns, 0.05, 12.0)
    h2, r2 = oracle.raycast(occ_r, hyp_r, Ns, Ns, 0.05, 12.0)
    q = Ns // 4
    r2s = np.roll(r2, -q, axis=1)
    h2s = np.roll(h2, -q, axis=1)
    # ranges: identical up to the FP32 rounding of the other axis' scale
    # factor at corner entries
    d = np.abs(r1.astype(np.float64) - r2s)
    assert (d <= np.spacing(np.maximum(r1, r2s)).astype(np.float64) * 1.01).all()
    # hits: map rotated hit cells back; disagreements only at equal-parameter
    # corner ties, where both cells must be occupied
    # rotated map has width H: index = y'*H + x' with x' = H-1-y, y' = x
    y_r, x_r = np.divmod(np.where(h2s >= 0, h2s, 0), H)
    back = np.where(h2s >= 0, (H - 1 - x_r) * W + y_r, -1)
    mism = back != h1
    assert ((h1 < 0) == (back < 0)).all()
    if mism.any():
        assert (occ.ravel()[back[mism]] >= 65).all()
        assert mism.mean() < 0.02


def test_cutoff_is_result_neutral():
    occ = make_micro(7, 60, 50, n_boxes=2)
    occ[1:-1, 1:-1][np.random.default_rng(0).random((48, 58)) < 0.01] = 100
    hyp = _free_cells(occ, 30, 1)
    for Ns in (360, 1440):
        hb, rb = oracle.raycast(occ, hyp, Ns, Ns, 0.05, 50.0)
        for rmax in (0.3, 0.77, 1.5):
            hs, rs = oracle.raycast(occ, hyp, Ns, Ns, 0.05, rmax)
            keep = rb <= np.float32(rmax)
            assert (rs == np.where(keep, rb, 0)).all()
            assert (hs == np.where(keep, hb, -1)).all()


def test_minimum_range_is_half_cell():
    # obstacle right next to the start cell: range = half a cell along the axis
    occ = np.zeros((5, 5), dtype=np.int8)
    occ[2, 3] = 100
    hit, rng = oracle.raycast(occ, np.array([[2, 2]], np.int32), 4, 4, 0.05, 10.0)
    assert hit[0, 0] == 2 * 5 + 3
    assert rng[0, 0] == np.float32(0.025)
