"""Oracle pins: the ablation metrics of Sec. IV (Case 3).

Coarse metric CAER (eq. 21, Remark 5):
* noiseless scan cast at the hypothesis itself, shifted by m0: CAER(m0) = 0;
* constant measured and synthetic ranges with invalid FoV beams: the closed
  form ((N_FoV - n_inv) |d - c| + n_inv c) / N_FoV (placeholder 0 for the
  invalid measured beams, Sec. III-B);
* SMAD(p, m) <= CAER(p, m) for every shift (|mean| <= mean of |.|), tying
  CAER to the pinned SMAD;
* rolling the synthetic scan by t shifts every CAER value by t exactly.

Fine metrics LF (eq. 32), baseline (eq. 33), T_mean (eq. 34):
* constant distance field and two-valued field: closed forms from plain
  trigonometry (as for TAM);
* the stage loop with a fine metric picks theta* and the batch best by that
  metric (brute force over every pose).
"""
import math

import numpy as np
import pytest

import oracle
from synth import make_micro

RES = 0.05


def _tiny(seed, n=30):
    occ = make_micro(seed, 50, 40, n_boxes=6)
    kmap = oracle.edt(occ)
    hyp = oracle.sample(occ, kmap, RES, n_target=n, seed=seed, min_spacing=0.15)
    return occ, kmap, hyp


def test_caer_zero_at_true_shift():
    occ, kmap, hyp = _tiny(21)
    Ns, h0, m0 = 240, 5, 37
    _, zhat = oracle.raycast(occ, hyp[h0:h0 + 1], Ns, Ns, RES, 20.0)
    n_beams = 180                                   # 270 deg FoV
    inc = 2 * math.pi / Ns
    amin = -math.radians(135.0)
    j0 = int(round(amin / inc)) % Ns
    z = zhat[0][(j0 + np.arange(n_beams) + m0) % Ns]
    z = np.where(z > 0, z, np.nan).astype(np.float32)
    pr = oracle.prep(z, amin, inc, RES, range_max=20.0)
    c, a, allv = oracle.caer(zhat, pr, all_shifts=True)
    assert allv[0, m0] == 0.0 and c[0] == 0.0
    assert (allv[0] >= 0).all()
    zero = np.nonzero(allv[0] == 0.0)[0]
    assert a[0] == zero[0] and m0 in zero


@pytest.mark.parametrize("d,c", [(1.5, 0.75), (0.4, 2.0), (1.0, 1.0)])
def test_caer_constant_closed_form(d, c):
    Ns = 120
    inc = 2 * math.pi / Ns
    z = np.full(90, d, np.float32)
    z[[3, 17, 40, 41, 88]] = np.nan                # invalid FoV beams
    pr = oracle.prep(z, -math.pi, inc, RES, range_max=20.0)
    zhat = np.full((2, Ns), c, np.float32)
    zhat[1, :] = 0.0                                 # no return anywhere
    cv, _, allv = oracle.caer(zhat, pr, all_shifts=True)
    n_fov, n_inv = 90, 5
    dd, cc = float(np.float32(d)), float(np.float32(c))
    want0 = ((n_fov - n_inv) * abs(dd - cc) + n_inv * cc) / n_fov
    want1 = (n_fov - n_inv) * dd / n_fov
    assert np.allclose(allv[0], want0, rtol=1e-15) and np.allclose(allv[1], want1, rtol=1e-15)
    assert cv[0] == allv[0].min() and cv[1] == allv[1].min()


@pytest.mark.parametrize("seed", [0, 1])
def test_smad_bounded_by_caer_every_shift(seed):
    occ, kmap, hyp = _tiny(seed)
    rng = np.random.default_rng(seed)
    Ns = 180
    inc = 2 * math.pi / Ns
    z = (rng.random(120) * 2.0 + 0.1).astype(np.float32)
    z[rng.random(120) < 0.1] = np.nan
    pr = oracle.prep(z, -math.radians(120.0), inc, RES, range_max=10.0, n_skip_enum=1)
    assert not pr["panoramic"]
    _, zhat = oracle.raycast(occ, hyp, Ns, Ns, RES, 10.0)
    _, _, s_all = oracle.smad(zhat, pr, all_shifts=True)
    _, _, c_all = oracle.caer(zhat, pr, all_shifts=True)
    assert s_all.shape == c_all.shape
    assert (s_all <= c_all * (1 + 1e-12) + 1e-15).all()
    assert (c_all > s_all).any()


def test_caer_shift_invariance():
    occ, kmap, hyp = _tiny(3)
    Ns, t = 144, 29
    inc = 2 * math.pi / Ns
    z = (np.random.default_rng(3).random(100) * 1.5 + 0.2).astype(np.float32)
    pr = oracle.prep(z, -math.radians(100.0), inc, RES, range_max=10.0)
    _, zhat = oracle.raycast(occ, hyp, Ns, Ns, RES, 10.0)
    _, _, a = oracle.caer(zhat, pr, all_shifts=True)
    _, _, b = oracle.caer(np.roll(zhat, -t, axis=1), pr, all_shifts=True)
    assert (b == np.roll(a, -t, axis=1)).all()
    # panoramic scans score every shift too (CAER is not rotation invariant)
    zp = (np.random.default_rng(4).random(Ns) + 0.3).astype(np.float32)
    pp = oracle.prep(zp, -math.pi, inc, RES, range_max=10.0)
    assert pp["panoramic"]
    _, _, c = oracle.caer(zhat, pp, all_shifts=True)
    assert c.shape == (len(hyp), Ns)


def _pano_prep(ranges, Ntheta=360):
    N = len(ranges)
    return oracle.prep(np.asarray(ranges, np.float32), -math.pi, 2 * math.pi / N, RES,
                       range_max=30.0, n_theta=Ntheta)


def _sd(d, d_max=2.0):
    dmin = RES / 2
    dt = min(max(d, dmin), d_max)
    return 1.0 - (dt - dmin) / (d_max - dmin)


@pytest.mark.parametrize("K0", [0, 3, 40, 900])
def test_fine_metrics_constant_field(K0):
    kmap = np.full((100, 100), K0, np.int64)
    pr = _pano_prep(np.full(360, 1.0))
    out = oracle.tam(kmap, RES, pr, np.array([[50, 50]] * 3), np.array([0, 11, 200]))
    d = math.sqrt(K0) * RES
    l0 = math.log(math.exp(-d * d / 0.08) + 1e-6)
    N = 360
    LF, base, mean = out[:, 8], out[:, 9], out[:, 10]
    assert np.allclose(LF, N * l0, rtol=1e-13)
    assert np.allclose(base, math.sqrt(math.exp(l0) * _sd(d)), rtol=1e-13)
    assert np.allclose(mean, (math.exp(l0) + _sd(d) + 1.0) / 3.0, rtol=1e-13)


@pytest.mark.parametrize("heading", [0, 30, 100])
def test_fine_metrics_two_valued_field(heading):
    # as the TAM two-valued pin: beams in [0, 45) deg have range 2 m, the rest
    # 0.5 m; cells at least 21 columns right of the pose have k = K1
    N, ix, iy = 360, 100, 100
    K0, K1 = 2, 85
    ang = -180 + np.arange(N)
    rng_m = np.where((ang >= 0) & (ang < 45), 2.0, 0.5)
    kmap = np.full((220, 220), K0, np.int64)
    kmap[:, ix + 21:] = K1
    pr = _pano_prep(rng_m)
    out = oracle.tam(kmap, RES, pr, np.array([[ix, iy]]), np.array([heading]))[0]
    world = np.radians(ang + heading)
    nf = int(((rng_m == 2.0) & (np.cos(world) >= 0.5125)).sum())
    nn = N - nf
    d0, d1 = math.sqrt(K0) * RES, math.sqrt(K1) * RES
    l0 = math.log(math.exp(-d0 * d0 / 0.08) + 1e-6)
    l1 = math.log(math.exp(-d1 * d1 / 0.08) + 1e-6)
    LF = nn * l0 + nf * l1
    kmid = (N * 700) // 1000
    Lbar = (min(kmid, nn) * l0 + max(0, kmid - nn) * l1) / kmid
    p = nn / N
    dbar = p * d0 + (1 - p) * d1
    var = p * (1 - p) * (d1 - d0) ** 2
    assert abs(out[8] - LF) < 1e-10
    assert abs(out[9] - math.sqrt(math.exp(LF / N) * _sd(dbar))) < 1e-12
    assert abs(out[10] - (math.exp(Lbar) + _sd(dbar) + math.exp(-var / 2)) / 3) < 1e-12


@pytest.mark.parametrize("fine", [1, 2, 3])
def test_stage_loop_uses_fine_metric(fine):
    occ, kmap, hyp = _tiny(8, n=24)
    N, inc = 90, math.radians(4.0)
    z = (np.random.default_rng(8).random(N) * 1.4 + 0.1).astype(np.float32)
    pr = oracle.prep(z, -math.radians(180.0), inc, RES, range_max=10.0, n_theta=45)
    _, zhat = oracle.raycast(occ, hyp, pr["Ns"], pr["Ng"], RES, 10.0)
    sm, _ = oracle.smad(zhat, pr)
    st = oracle.stages(kmap, RES, pr, hyp, sm, 6, None, all_T=True, fine_metric=fine)
    q = np.repeat(hyp, 45, axis=0)
    k = np.tile(np.arange(45), len(hyp))
    V = oracle.tam(kmap, RES, pr, q, k)[:, oracle.FINE_COL[fine]].reshape(len(hyp), 45)
    assert (st["all_T"] == V[st["order"]]).all()
    for r in range(len(hyp)):
        row = V[st["order"][r]]
        assert st["tstar"][r] == row.max() and st["kstar"][r] == int(np.argmax(row))
    # refinement by the same metric
    o = pr["Ng"] // pr["Ntheta"]
    cells = hyp[st["order"][:4]]
    T, dxy, g, allv = oracle.refine(kmap, RES, pr, cells, o * st["kstar"][:4],
                                    refine_cells=1, refine_dirs=1, all_T=True,
                                    fine_metric=fine)
    assert (T == np.nanmax(allv, axis=1)).all()
