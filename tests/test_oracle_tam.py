"""Oracle pins: TAM (eq. 22-31).

* constant distance field: sigma^2 = 0 so c = 1, every l_i equal, and
  T = (exp(l(delta)) * s_d(delta))^(1/3) in closed form;
* every endpoint on an obstacle: T = (z_hit + z_rand + 1e-6)^(1/3);
* every endpoint off the map: d = d_max, s_d = 0, T = 0;
* two-valued field with beam counts fixed by plain trigonometry: the top-k_mid
  selection, the mean, the population variance, k_mid and the endpoint
  geometry all enter one closed form (a transposed or sign-flipped direction
  changes the counts);
* median identity of eq. 27 (top-k means are non-increasing in k), bounds of
  s_d, c and T;
* a quarter turn of the world maps T(p, theta_k) onto T(p', theta_{k+N/4}).
"""
import math

import numpy as np
import pytest

import oracle
from synth import make_config

RES = 0.05


def _pano_prep(ranges, Ntheta=360):
    N = len(ranges)
    return oracle.prep(np.asarray(ranges, np.float32), -math.pi, 2 * math.pi / N, RES,
                       range_max=30.0, n_theta=Ntheta)


def _sd(d, d_max, res=RES):
    dmin = res / 2
    dt = min(max(d, dmin), d_max)
    return 1.0 - (dt - dmin) / (d_max - dmin)


@pytest.mark.parametrize("K0", [0, 1, 2, 5, 50, 400, 1600, 10000])
@pytest.mark.parametrize("params", [(1.0, 0.2, 0.0, 2.0), (0.8, 0.35, 0.05, 3.0)])
def test_constant_field_closed_form(K0, params):
    z_hit, sig, z_rand, d_max = params
    kmap = np.full((120, 120), K0, np.int64)
    pr = _pano_prep(np.full(360, 1.0))
    out = oracle.tam(kmap, RES, pr, np.array([[60, 60]] * 4), np.array([0, 7, 90, 359]),
                     z_hit, sig, z_rand, d_max)
    d = math.sqrt(K0) * RES
    l = math.log(z_hit * math.exp(-(d * d) / (2 * sig * sig)) + z_rand + 1e-6)
    T = (math.exp(l) * _sd(d, d_max)) ** (1.0 / 3.0)
    assert np.allclose(out[:, 0], T, rtol=1e-13, atol=0)
    assert np.allclose(out[:, 3], 1.0, rtol=1e-15)
    assert np.allclose(out[:, 4], l, rtol=1e-13)


def test_all_endpoints_on_obstacles():
    kmap = np.zeros((100, 100), np.int64)
    pr = _pano_prep(np.linspace(0.3, 2.0, 720))
    out = oracle.tam(kmap, RES, pr, np.array([[50, 50]]), np.array([3]))
    assert abs(out[0, 0] - (1.0 + 1e-6) ** (1 / 3)) < 1e-15
    assert out[0, 2] == 1.0 and out[0, 3] == 1.0


def test_all_endpoints_off_map():
    kmap = np.zeros((7, 7), np.int64)
    pr = _pano_prep(np.full(360, 5.0))
    out = oracle.tam(kmap, RES, pr, np.array([[3, 3]]), np.array([0]), d_max=2.0)
    assert out[0, 0] == 0.0 and out[0, 2] == 0.0
    assert abs(out[0, 1] - (math.exp(-4.0 / 0.08) + 1e-6)) < 1e-18


@pytest.mark.parametrize("heading", [0, 30, 310, 100])
def test_two_valued_field_closed_form(heading):
    # beams at integer degrees; those in [0, 45) deg have range 2 m, the rest
    # 0.5 m. Cells at least 21 columns right of the hypothesis have k = K1,
    # all others k = K0. A beam ends in the far region iff its range is 2 m
    # and cos(angle) >= 20.5 / 40 = 0.5125.
    N, ix, iy = 360, 100, 100
    K0, K1 = 2, 85
    ang = -180 + np.arange(N)
    rng_m = np.where((ang >= 0) & (ang < 45), 2.0, 0.5)
    kmap = np.full((220, 220), K0, np.int64)
    kmap[:, ix + 21:] = K1
    pr = _pano_prep(rng_m)
    out = oracle.tam(kmap, RES, pr, np.array([[ix, iy]]), np.array([heading]))
    world = np.radians(ang + heading)
    far = (rng_m == 2.0) & (np.cos(world) >= 0.5125)
    nf = int(far.sum())
    nn = N - nf
    d0, d1 = math.sqrt(K0) * RES, math.sqrt(K1) * RES
    l0 = math.log(math.exp(-d0 * d0 / 0.08) + 1e-6)
    l1 = math.log(math.exp(-d1 * d1 / 0.08) + 1e-6)
    kmid = (N * 700) // 1000                       # lambda = 1 -> alpha_mid = 0.7
    top = min(kmid, nn) * l0 + max(0, kmid - nn) * l1
    Lbar = top / kmid
    p = nn / N
    dbar = p * d0 + (1 - p) * d1
    var = p * (1 - p) * (d1 - d0) ** 2
    T = (math.exp(Lbar) * _sd(dbar, 2.0) * math.exp(-var / 2)) ** (1 / 3)
    assert pr["k_mid"] == kmid
    assert abs(out[0, 4] - Lbar) < 1e-12
    assert abs(out[0, 3] - math.exp(-var / 2)) < 1e-12
    assert abs(out[0, 0] - T) < 1e-12
    assert nf == {0: 45, 30: 30, 310: 45, 100: 0}[heading]


def test_median_identity_and_bounds():
    w = make_config(1)
    kmap = oracle.edt(w.occ)
    pr = oracle.prep(w.ranges, w.angle_min, w.angle_increment, w.resolution,
                     range_min=w.range_min, range_max=w.range_max, n_theta=360)
    rng = np.random.default_rng(0)
    ys, xs = np.nonzero((w.occ == 0) & (kmap >= 18))
    pick = rng.choice(len(xs), 200)
    q = np.stack([xs[pick], ys[pick]], 1)
    k = rng.integers(0, 360, 200)
    out = oracle.tam(kmap, RES, pr, q, k)
    T, P, sd, c, Lbar, mf, mm, ml = out.T[:8]
    assert (ml >= mm).all() and (mm >= mf).all()
    assert (Lbar == mm).all()
    assert ((sd >= 0) & (sd <= 1)).all() and ((c > 0) & (c <= 1)).all()
    assert ((T >= 0) & (T <= (1 + 1e-6) ** (1 / 3))).all()
    assert np.allclose(T ** 3, P * sd * c, rtol=1e-12)


def test_quarter_turn_invariance():
    w = make_config(1)
    occ = w.occ
    H, W = occ.shape
    occ_r = np.ascontiguousarray(occ.T[:, ::-1])
    k1 = oracle.edt(occ)
    k2 = oracle.edt(occ_r)
    pr = oracle.prep(w.ranges, w.angle_min, w.angle_increment, w.resolution,
                     range_min=w.range_min, range_max=w.range_max, n_theta=360)
    rng = np.random.default_rng(1)
    ys, xs = np.nonzero((occ == 0) & (k1 >= 18))
    pick = rng.choice(len(xs), 100)
    q = np.stack([xs[pick], ys[pick]], 1)
    qr = np.stack([H - 1 - q[:, 1], q[:, 0]], 1)
    k = rng.integers(0, 360, 100)
    a = oracle.tam(k1, RES, pr, q, k)[:, 0]
    b = oracle.tam(k2, RES, pr, qr, (k + 90) % 360)[:, 0]
    same = np.abs(a - b) <= 1e-12 * np.maximum(a, 1e-300)
    assert same.mean() >= 0.97
    assert np.abs(a - b).max() < 0.05
