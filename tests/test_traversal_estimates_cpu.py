"""The two float estimates of the jump traversal (scan synthesis by ray
casting, Sec. III-B, eq. 13) against exact integer arithmetic, over the real
direction tables.

The fused ray cast jumps through free space and lands on the exact crossing
sequence by two FP32 estimates that are biased low, so that each is either
exact or one short:

* landing: the minor crossing count just after the na-th major crossing is
  nb = floor((na - 1/2) b / a + 1/2); the kernel truncates
  fma(na, r, c) with r = fl(b / a) and c = fl(fl(1/2 - r/2) - 2^-7) and then
  takes at most one exact step up, so the estimate must be nb or nb - 1;
* run jump: ceil(-Dm / (256 b)) major crossings come before the next minor
  one; the kernel takes ceil(min(fma(fl(Dm), -fl(1 / (256 b)), -2^-12), 256))
  with no check after it, so the estimate must never exceed the true count
  (and, to lose little, be at most one short of it below the cap).

The kernel's FP32 fma is emulated exactly: the product of two floats plus a
float is exact in the 64-bit mantissa of long double for the ranges used
here, and the cast to float32 rounds once, to nearest even. The constants are
formed as the library's host code and skip_start form them.
"""
import numpy as np
import pytest

import oracle

pytestmark = pytest.mark.skipif(np.finfo(np.longdouble).nmant < 63,
                                reason="needs an 80-bit long double to emulate fma exactly")


def _fma32(x, y, z):
    ld = np.longdouble
    return (x.astype(ld) * y.astype(ld) + z.astype(ld)).astype(np.float32)


def _ab(Ng):
    U = oracle.dirs(Ng).astype(np.int64)
    ax, ay = np.abs(U[:, 0]), np.abs(U[:, 1])
    return np.maximum(ax, ay), np.minimum(ax, ay)


@pytest.mark.parametrize("Ng", [360, 1440, 5760])
def test_landing_estimate_is_exact_or_one_low(Ng):
    a, b = _ab(Ng)
    r = (b.astype(np.float64) / a.astype(np.float64)).astype(np.float32)
    c = (np.float32(0.5) - np.float32(0.5) * r) - np.float32(2.0 ** -7)
    assert r.dtype == np.float32 and c.dtype == np.float32
    assert (r <= 1).all()
    na = np.arange(1, 2 ** 13, dtype=np.int64)
    for j0 in range(0, len(a), 256):
        aj, bj = a[j0:j0 + 256, None], b[j0:j0 + 256, None]
        rj, cj = r[j0:j0 + 256, None], c[j0:j0 + 256, None]
        x = _fma32(np.broadcast_to(na.astype(np.float32), (len(aj), len(na))), rj, cj)
        assert (x > 0).all()
        est = np.trunc(x).astype(np.int64)
        nb = ((2 * na - 1) * bj + aj) // (2 * aj)
        ok = (est == nb) | (est == nb - 1)
        assert ok.all(), "direction %d, na %d" % tuple(np.argwhere(~ok)[0])


@pytest.mark.parametrize("Ng", [360, 1440, 5760])
def test_run_estimate_never_overshoots(Ng):
    a, b = _ab(Ng)
    keep = b > 0                                  # b = 0: every crossing is major
    a, b = a[keep], b[keep]
    ninv = -(1.0 / (256.0 * b.astype(np.float64))).astype(np.float32)
    step = 256 * b[:, None]
    # -Dm at, just below and just above every exact multiple of 256 b up to
    # 300 crossings, plus seeded values in between; |Dm| < 2^28
    k = np.arange(0, 301, dtype=np.int64)[None, :, None]
    d = np.array([-2, -1, 0, 1, 2], dtype=np.int64)[None, None, :]
    tn = (k * step[:, :, None] + d).reshape(len(b), -1)
    rng = np.random.default_rng(20251101)
    tn = np.concatenate([tn, rng.integers(1, 300 * step + 1, size=(len(b), 512))], axis=1)
    bb = np.broadcast_to(b[:, None], tn.shape)
    valid = (tn > 0) & (tn < 2 ** 28)
    dm = np.where(valid, -tn, -1)
    est = np.minimum(_fma32(dm.astype(np.float32), np.broadcast_to(ninv[:, None], tn.shape),
                            np.full(tn.shape, -2.0 ** -12, dtype=np.float32)), np.float32(256))
    kr = np.ceil(est).astype(np.int64)
    kmax = (-dm + 256 * bb - 1) // (256 * bb)     # ceil(-Dm / (256 b))
    over = valid & (kr > kmax)
    assert not over.any(), "direction %d, sample %d" % tuple(np.argwhere(over)[0])
    short = valid & (kmax <= 256) & (kr < kmax - 1)
    assert not short.any(), "direction %d, sample %d" % tuple(np.argwhere(short)[0])
    # the cap: beyond 256 crossings the estimate is 256 (the run byte is at most 255)
    assert (kr[valid & (kmax > 257)] == 256).all()
