"""Oracle pins: local refinement of each batch's best poses (Sec. III
pipeline text: the top-k poses of a batch are refined by a local operator
and re-evaluated with TAM before the threshold test; Remark 2).

The operator is an exhaustive TAM search over the lattice of poses next to
the pose: cells within +-h, headings within +-s steps of the Ng direction
grid; off-map and occupied lattice cells other than the pose's own are not
visited; ties go to the pose itself, then to the smaller raster index.

* two-valued field: every lattice T in closed form from plain trigonometry
  (which beams end in the far region from the moved cell and the turned
  heading), and the chosen lattice point from the closed-form values with
  the tie rule; excluded cells are reported as NaN and never chosen, the
  pose's own cell is visited even when occupied;
* heading lattice across the wrap of the direction grid equals TAM on the
  grid N_theta = Ng (heading index = direction index);
* off-map lattice cells are not visited;
* stage loop: h = s = 0 is the identity; the refined ranks are each batch's
  refine_k best by (T* desc, rank asc); refined T >= unrefined T; the
  threshold is tested on the refined batch best.
"""
import math

import numpy as np
import pytest

import oracle
from synth import make_config, make_micro

RES = 0.05


def _pano_prep(ranges, Ntheta=360):
    N = len(ranges)
    return oracle.prep(np.asarray(ranges, np.float32), -math.pi, 2 * math.pi / N, RES,
                       range_max=30.0, n_theta=Ntheta)


def _sd(d, d_max, res=RES):
    dmin = res / 2
    dt = min(max(d, dmin), d_max)
    return 1.0 - (dt - dmin) / (d_max - dmin)


def _closed_form_T(nf, N, K0, K1):
    nn = N - nf
    d0, d1 = math.sqrt(K0) * RES, math.sqrt(K1) * RES
    l0 = math.log(math.exp(-d0 * d0 / 0.08) + 1e-6)
    l1 = math.log(math.exp(-d1 * d1 / 0.08) + 1e-6)
    kmid = (N * 700) // 1000
    top = min(kmid, nn) * l0 + max(0, kmid - nn) * l1
    p = nn / N
    dbar = p * d0 + (1 - p) * d1
    var = p * (1 - p) * (d1 - d0) ** 2
    return (math.exp(top / kmid) * _sd(dbar, 2.0) * math.exp(-var / 2)) ** (1 / 3)


@pytest.mark.parametrize("k0", [0, 30, 310, 359])
@pytest.mark.parametrize("hs", [(2, 1), (3, 2)])
def test_two_valued_field_lattice_closed_form(k0, hs):
    # beams at integer degrees; those in [0, 45) deg have range 2 m (40
    # cells), the rest 0.5 m (10 cells). Cells at least 21 columns right of
    # the pose's cell have k = K1, all others k = K0. From the lattice cell
    # dx columns over, a beam at world angle a ends in the far region iff its
    # range is 2 m and 40 cos(a) >= 20.5 - dx (the 10-cell beams never
    # reach it for |dx| <= 3).
    h, s = hs
    N, ix, iy = 360, 100, 100
    K0, K1 = 2, 85
    ang = -180 + np.arange(N)
    rng_m = np.where((ang >= 0) & (ang < 45), 2.0, 0.5)
    kmap = np.full((220, 220), K0, np.int64)
    kmap[:, ix + 21:] = K1
    # two occupied lattice cells (no endpoint can reach them: every endpoint
    # is 10 or 40 cells from its lattice cell) and an occupied pose cell
    kmap[iy + 2, ix + 1] = 0
    kmap[iy - 2, ix - 2] = 0
    kmap[iy, ix] = 0
    pr = _pano_prep(rng_m)
    assert pr["Ng"] == 360
    T, dxy, g, allv = oracle.refine(kmap, RES, pr, np.array([[ix, iy]]), np.array([k0]),
                                    refine_cells=h, refine_dirs=s, all_T=True)
    w = 2 * h + 1
    want = np.full((2 * s + 1, w, w), np.nan)
    for dg in range(-s, s + 1):
        world = np.radians(ang + ((k0 + dg) % 360))
        for dy in range(-h, h + 1):
            for dx in range(-h, h + 1):
                if (dx, dy) in ((1, 2), (-2, -2)):
                    continue
                thr = (20.5 - dx) / 40.0
                c = np.cos(world)
                near = (rng_m == 2.0) & (np.abs(c - thr) < 1e-4)
                assert not near.any()              # no beam within rounding of the edge
                nf = int(((rng_m == 2.0) & (c >= thr)).sum())
                want[dg + s, dy + h, dx + h] = _closed_form_T(nf, N, K0, K1)
    got = allv[0].reshape(2 * s + 1, w, w)
    assert (np.isnan(got) == np.isnan(want)).all()
    ok = ~np.isnan(want)
    assert np.abs(got[ok] - want[ok]).max() < 1e-12
    # the chosen point: largest T, ties to the pose itself, then raster order
    flat = want.reshape(-1)
    q_c = (s * w + h) * w + h
    keys = [(-flat[q], 0 if q == q_c else q + 1, q) for q in range(len(flat))
            if not np.isnan(flat[q])]
    q_best = min(keys)[2]
    dg_b, rem = divmod(q_best, w * w)
    dy_b, dx_b = divmod(rem, w)
    assert (dxy[0, 0], dxy[0, 1]) == (dx_b - h, dy_b - h)
    assert g[0] == (k0 + dg_b - s) % 360
    assert abs(T[0] - flat[q_best]) < 1e-12


def test_heading_lattice_equals_fine_grid_tam():
    occ = make_micro(7, 60, 48, n_boxes=6)
    kmap = oracle.edt(occ)
    hyp = oracle.sample(occ, kmap, RES, n_target=6, seed=7, min_spacing=0.3)
    N, inc = 120, math.radians(3.0)
    z = (np.random.default_rng(7).random(N) * 1.4 + 0.1).astype(np.float32)
    amin = -math.radians(180.0)
    pr = oracle.prep(z, amin, inc, RES, range_max=10.0, n_theta=40)
    Ng, o = pr["Ng"], pr["Ng"] // pr["Ntheta"]
    assert o == 3
    # TAM on the fine grid N_theta = Ng: heading index k' is direction index g
    fine = oracle.prep(z, amin, inc, RES, range_max=10.0, n_theta=Ng)
    assert fine["Ng"] == Ng and fine["Ntheta"] == Ng
    h, s = 1, o
    w = 2 * h + 1
    g0 = np.array([0, o * 39, o * 17, 5, 2, Ng - 1])[:len(hyp)]
    T, dxy, g, allv = oracle.refine(kmap, RES, pr, hyp, g0, refine_cells=h, refine_dirs=s,
                                    all_T=True)
    H, W = kmap.shape
    for i in range(len(hyp)):
        for dg in range(-s, s + 1):
            for dy in range(-h, h + 1):
                for dx in range(-h, h + 1):
                    q = ((dg + s) * w + dy + h) * w + dx + h
                    x, y = hyp[i, 0] + dx, hyp[i, 1] + dy
                    own = dx == 0 and dy == 0
                    if not own and not (0 <= x < W and 0 <= y < H and kmap[y, x] != 0):
                        assert np.isnan(allv[i, q])
                        continue
                    gg = (int(g0[i]) + dg) % Ng
                    ref = oracle.tam(kmap, RES, fine, np.array([[x, y]]), np.array([gg]))[0, 0]
                    assert allv[i, q] == ref
        assert T[i] == np.nanmax(allv[i])
        assert 0 <= g[i] < Ng


def test_off_map_lattice_cells_not_visited():
    kmap = np.full((12, 12), 5, np.int64)
    pr = _pano_prep(np.full(90, 0.2), Ntheta=90)
    T, dxy, g, allv = oracle.refine(kmap, RES, pr, np.array([[0, 11]]), np.array([0]),
                                    refine_cells=2, refine_dirs=0, all_T=True)
    a = allv[0].reshape(5, 5)
    for dy in range(-2, 3):
        for dx in range(-2, 3):
            off = not (0 <= dx < 12 and 0 <= 11 + dy < 12)
            assert np.isnan(a[dy + 2, dx + 2]) == off
    assert 0 <= dxy[0, 0] and dxy[0, 1] <= 0


def _world(seed, n_theta=60):
    occ = make_micro(seed, 64, 50, n_boxes=7)
    kmap = oracle.edt(occ)
    hyp = oracle.sample(occ, kmap, RES, n_target=48, seed=seed, min_spacing=0.2)
    N, inc = 90, math.radians(4.0)
    z = (np.random.default_rng(seed).random(N) * 1.5 + 0.1).astype(np.float32)
    pr = oracle.prep(z, -math.radians(180.0), inc, RES, range_max=10.0, n_theta=n_theta)
    _, zhat = oracle.raycast(occ, hyp, pr["Ns"], pr["Ng"], RES, 10.0)
    sm, _ = oracle.smad(zhat, pr)
    return kmap, hyp, pr, sm


@pytest.mark.parametrize("seed", [1, 2])
def test_stage_refinement_selection_and_values(seed):
    kmap, hyp, pr, sm = _world(seed)
    K, kr = 8, 3
    o = pr["Ng"] // pr["Ntheta"]
    base = oracle.stages(kmap, RES, pr, hyp, sm, K, None)
    ref = oracle.stages(kmap, RES, pr, hyp, sm, K, None, refine_k=kr, refine_cells=2)
    assert (ref["order"] == base["order"]).all() and ref["n_eval"] == base["n_eval"]
    assert (ref["kstar"] == base["kstar"]).all()
    for b0 in range(0, base["n_eval"], K):
        t = base["tstar"][b0:b0 + K]
        sel = b0 + np.lexsort((np.arange(len(t)), -t))[:kr]
        mask = np.zeros(len(t), bool)
        mask[sel - b0] = True
        assert (ref["refined"][b0:b0 + K] == mask).all()
        # unrefined ranks keep their values and heading o * k*
        un = np.arange(b0, b0 + len(t))[~mask]
        assert (ref["tstar"][un] == base["tstar"][un]).all()
        assert (ref["ref_g"][un] == o * base["kstar"][un]).all()
        assert (ref["ref_dxy"][un] == 0).all()
        # refined ranks: the lattice search around (cell, o * k*)
        cells = hyp[ref["order"][sel]]
        T, dxy, g = oracle.refine(kmap, RES, pr, cells, o * base["kstar"][sel],
                                  refine_cells=2)
        assert (ref["tstar"][sel] == T).all() and (T >= base["tstar"][sel]).all()
        assert (ref["ref_dxy"][sel] == dxy).all() and (ref["ref_g"][sel] == g).all()


def test_identity_lattice():
    kmap, hyp, pr, sm = _world(3)
    base = oracle.stages(kmap, RES, pr, hyp, sm, 8, None)
    ref = oracle.stages(kmap, RES, pr, hyp, sm, 8, None, refine_k=8, refine_cells=0,
                        refine_dirs=0)
    assert ref["refined"].all()
    assert (ref["tstar"] == base["tstar"]).all()
    assert (ref["ref_dxy"] == 0).all()
    assert (ref["ref_g"] == (pr["Ng"] // pr["Ntheta"]) * base["kstar"]).all()


def test_threshold_uses_refined_best():
    kmap, hyp, pr, sm = _world(4)
    K = 8
    base = oracle.stages(kmap, RES, pr, hyp, sm, K, None)
    ref = oracle.stages(kmap, RES, pr, hyp, sm, K, None, refine_k=2, refine_cells=3)
    b_un = [base["tstar"][b:b + K].max() for b in range(0, len(hyp), K)]
    b_rf = [ref["tstar"][b:b + K].max() for b in range(0, len(hyp), K)]
    assert all(r >= u for r, u in zip(b_rf, b_un))
    # a threshold between the first batch's unrefined and refined best
    j = next(i for i in range(len(b_un)) if b_rf[i] > b_un[i])
    tau = 0.5 * (b_un[j] + b_rf[j])
    st = oracle.stages(kmap, RES, pr, hyp, sm, K, tau, refine_k=2, refine_cells=3)
    first = next(i for i, b in enumerate(b_rf) if b > tau)
    assert st["early_stopped"] and st["stages"] == first + 1 and first <= j
    plain = oracle.stages(kmap, RES, pr, hyp, sm, K, tau)
    first_un = next((i for i, b in enumerate(b_un) if b > tau), None)
    assert plain["stages"] == (len(b_un) if first_un is None else first_un + 1)


def test_refinement_moves_plain_small_best_toward_truth():
    w = make_config(1)
    kmap = oracle.edt(w.occ)
    hyp = oracle.sample(w.occ, kmap, w.resolution, n_target=300, seed=1,
                        min_spacing=0.3, robot_radius=0.21)
    kw = dict(n_theta=360, batch_k=10, tau=None, k_out=1, kmap=kmap)
    args = (w.occ, w.resolution, w.origin, hyp, w.ranges, w.angle_min, w.angle_increment,
            w.range_min, w.range_max)
    a = oracle.relocalize(*args, **kw)["poses"][0]
    b = oracle.relocalize(*args, refine_k=2, refine_cells=3, **kw)["poses"][0]
    assert b["refined"] and b["tam"] >= a["tam"]
    da = math.hypot(a["x"] - w.pose[0], a["y"] - w.pose[1])
    db = math.hypot(b["x"] - w.pose[0], b["y"] - w.pose[1])
    assert db <= da
