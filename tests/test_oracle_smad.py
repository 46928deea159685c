"""Oracle pins: scan preprocessing (eq. 11-16, 25-26) and SMAD (eq. 16-20).

* SMAD = 0 exactly at the true pose of a noiseless scan synthesised by the
  oracle's own ray cast from an on-grid pose;
* rotation shift: a scan taken r beam steps further round shifts the whole
  SMAD curve by r, bit for bit, and leaves SMAD(p) unchanged;
* panoramic scans: SMAD(p, theta_m) is constant in m, and eq. 20 keeps m = 0;
* the prefix-sum form of eq. 17-18 equals the direct sum bit for bit (all
  partial sums are exact in FP64 for ranges in [2^-6, 2^6) m);
* constant synthetic scan: closed form |zbar - c|; ties give the smallest m;
* preprocessing closed forms (N_s, N_FoV, lambda, k_mid, k_low) and error
  codes.
"""
import math

import numpy as np
import pytest

import oracle
from synth import make_config, make_micro

RES = 0.05


def _scan_from_synthetic(zhat_row, Ns, n_beams, j0, m0):
    """Measured ranges of a noiseless scan at heading index m0: beam i looks
    along panoramic direction (j0 + i + m0) mod Ns; no return -> NaN."""
    idx = (j0 + np.arange(n_beams) + m0) % Ns
    z = zhat_row[idx].astype(np.float32)
    return np.where(z > 0, z, np.float32(np.nan)).astype(np.float32)


def _room_setup(seed=0):
    occ = make_micro(seed, 60, 48, n_boxes=7)
    ys, xs = np.nonzero(occ == 0)
    rng = np.random.default_rng(seed)
    pick = rng.choice(len(xs), size=12, replace=False)
    hyp = np.stack([xs[pick], ys[pick]], 1).astype(np.int32)
    return occ, hyp


@pytest.mark.parametrize("fov_deg,n_beams,m0", [(270.0, 360, 37), (180.0, 240, 400),
                                                (240.0, 320, 5), (90.0, 120, 250)])
def test_smad_zero_at_true_pose(fov_deg, n_beams, m0):
    occ, hyp = _room_setup(1)
    inc = math.radians(fov_deg) / n_beams
    Ns = int(round(2 * math.pi / inc))
    amin = -math.radians(fov_deg) / 2
    _, zhat = oracle.raycast(occ, hyp, Ns, Ns, RES, 30.0)
    pr0 = oracle.prep(np.ones(n_beams, np.float32), amin, inc, RES, range_max=30.0)
    z = _scan_from_synthetic(zhat[3], Ns, n_beams, pr0["j0"], m0)
    pr = oracle.prep(z, amin, inc, RES, range_max=30.0)
    assert pr["status"] == 0 and not pr["panoramic"]
    s, a, allv = oracle.smad(zhat, pr, all_shifts=True)
    assert s[3] == 0.0
    assert allv[3, m0] == 0.0
    assert a[3] <= m0
    # every other hypothesis is (almost surely) worse
    assert (np.delete(s, 3) > 0).all()


def test_rotation_shift_of_smad_curve():
    # turning the world about p by r beam steps rotates the panoramic
    # synthetic scan by r; the SMAD curve of eq. 19 must turn with it
    occ, hyp = _room_setup(2)
    n_beams, inc = 360, math.radians(0.75)
    Ns, amin = 480, -math.radians(135.0)
    _, zhat = oracle.raycast(occ, hyp, Ns, Ns, RES, 30.0)
    j0 = oracle.prep(np.ones(n_beams, np.float32), amin, inc, RES)["j0"]
    z = _scan_from_synthetic(zhat[5], Ns, n_beams, j0, 100)
    pr = oracle.prep(z, amin, inc, RES, range_max=30.0)
    s0, a0, all0 = oracle.smad(zhat, pr, all_shifts=True)
    for r in (1, 17, 250, 479):
        s, a, allv = oracle.smad(np.roll(zhat, r, axis=1), pr, all_shifts=True)
        assert (s == s0).all()
        assert (allv == np.roll(all0, r, axis=1)).all()
        assert a[5] == (a0[5] + r) % Ns


def test_panoramic_constant_over_shifts():
    occ, hyp = _room_setup(3)
    Ns = 720
    inc = 2 * math.pi / Ns
    _, zhat = oracle.raycast(occ, hyp, Ns, Ns, RES, 30.0)
    rng = np.random.default_rng(0)
    z = (rng.random(Ns) * 3 + 0.1).astype(np.float32)
    pr = oracle.prep(z, -math.pi, inc, RES, range_max=30.0)
    assert pr["panoramic"] and pr["n_shifts"] == 1 and pr["lam"] == 1.0
    s, a = oracle.smad(zhat, pr)
    assert (a == 0).all()
    pr2 = dict(pr, panoramic=False, n_shifts=Ns)
    s2, a2, allv = oracle.smad(zhat, pr2, all_shifts=True)
    assert (allv == allv[:, :1]).all()
    assert (s2 == s).all()


def test_prefix_sum_form_equals_direct_sum():
    occ, hyp = _room_setup(4)
    n_beams, inc, Ns = 360, math.radians(0.75), 480
    amin = -math.radians(135.0)
    fov = [(-math.radians(135.0), math.radians(-20.0)),
           (math.radians(10.0), math.radians(134.0))]
    _, zhat = oracle.raycast(occ, hyp, Ns, Ns, RES, 30.0)
    rng = np.random.default_rng(1)
    z = (rng.random(n_beams) * 5 + 0.2).astype(np.float32)
    pr = oracle.prep(z, amin, inc, RES, fov=fov, range_max=30.0)
    assert pr["n_runs"] == 2
    s, a, allv = oracle.smad(zhat, pr, all_shifts=True)
    # eq. 17-18: cyclic prefix sums over the duplicated scan
    st = pr["beam_state"]
    runs = []
    i = 0
    while i < len(st):
        if st[i] >= 1:
            k = i
            while k + 1 < len(st) and st[k + 1] >= 1:
                k += 1
            runs.append((int(pr["beam_j"][i]), k - i + 1))
            i = k + 1
        else:
            i += 1
    for h in range(len(hyp)):
        S = np.concatenate([[0.0], np.cumsum(np.tile(zhat[h].astype(np.float64), 3))])
        for m in range(Ns):
            tot = 0.0
            for u, L in runs:
                tot += S[u + m + L] - S[u + m]
            v = abs(pr["zbar"] - tot / pr["N_fov"])
            assert v == allv[h, m]


def test_constant_synthetic_scan_closed_form_and_ties():
    n_beams, inc = 360, math.radians(0.75)
    rng = np.random.default_rng(2)
    z = (rng.random(n_beams) * 4 + 0.5).astype(np.float32)
    pr = oracle.prep(z, -math.radians(135.0), inc, RES, range_max=30.0)
    zhat = np.full((3, 480), 1.5, np.float32)
    zhat[1] = 0.75
    zhat[2] = 0.0
    s, a, allv = oracle.smad(zhat, pr, all_shifts=True)
    for h, c in enumerate((1.5, 0.75, 0.0)):
        assert (allv[h] == abs(pr["zbar"] - c)).all()
        assert a[h] == 0


def test_prep_closed_forms_c1_like():
    n_beams, inc = 360, math.radians(0.75)
    z = np.full(n_beams, 2.0, np.float32)
    drop = np.random.default_rng(3).choice(n_beams, 18, replace=False)
    z[drop] = np.nan
    pr = oracle.prep(z, -math.radians(135.0), inc, RES, range_max=12.0, n_theta=360)
    assert pr["status"] == 0
    assert (pr["Ns"], pr["Ntheta"], pr["Ng"]) == (480, 360, 1440)
    assert pr["N_fov"] == 360 and pr["N_valid"] == 342 and pr["lam"] == 0.75
    assert pr["k_mid"] == 256 and pr["k_low"] == 188 and pr["k_full"] == 342
    assert pr["j0"] == 480 - 180
    assert pr["zbar"] == (342 * 2.0) / 360
    assert pr["n_shifts"] == 480
    assert (pr["valid_zq"] == 10240).all()


def test_prep_downsample_and_errors():
    inc = math.radians(0.25)
    z = np.full(1080, 3.0, np.float32)
    pr = oracle.prep(z, -math.radians(135.0), inc, RES, n_skip_beam=4, range_max=30.0)
    assert pr["status"] == 0 and pr["Ns"] == 360 and pr["n_down"] == 270
    # increment that does not divide the circle
    bad = oracle.prep(z, -math.radians(135.0), math.radians(0.7), RES)
    assert bad["status"] == oracle.E_BEAMGRID
    # first beam off the angular grid
    bad = oracle.prep(z, -math.radians(135.1), inc, RES)
    assert bad["status"] == oracle.E_BEAMGRID
    # no valid beam
    bad = oracle.prep(np.full(100, np.nan, np.float32), 0.0, math.radians(1.0), RES)
    assert bad["status"] == oracle.E_EMPTY
    # everything outside range
    bad = oracle.prep(np.full(100, 50.0, np.float32), 0.0, math.radians(1.0), RES,
                      range_max=20.0)
    assert bad["status"] == oracle.E_EMPTY


def test_zbar_is_exact_sum():
    w = make_config(1)
    pr = oracle.prep(w.ranges, w.angle_min, w.angle_increment, w.resolution,
                     range_min=w.range_min, range_max=w.range_max, n_theta=360)
    zp = pr["beam_z"][pr["beam_state"] >= 1]
    assert pr["zbar"] == math.fsum(zp) / pr["N_fov"]
