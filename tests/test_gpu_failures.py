"""Failure handling through the C ABI: every refused call leaves the context
usable and holding the same device bytes, and the next relocalization
returns exactly what it returned before the failures.

* a context with a 40 MB HBM budget: the 200^2 map and its request fit; the
  2000^2 map (EDT 16 MB + walk words 32 MB + tiles) does not (E_NOMEM);
* a malformed scan (E_BEAMGRID), an unknown request (E_NOTFOUND), a second
  release (E_NOTFOUND), unloading a map whose set is alive (E_BUSY), bad
  search parameters (E_INVALID), a scan with no valid beam (E_EMPTY), rank
  ranges of the debug TAM call outside the request, including one whose end
  wraps in 32 bits (E_INVALID, refused before any launch).
"""
import math
import sys

import numpy as np
import pytest

import oracle
import paper_2511_01219_amd as reloc
from synth import make_config

pytestmark = pytest.mark.gpu


def _case(msg):
    print("[gpu case] " + msg, flush=True)
    sys.stdout.flush()


def _scan(w):
    return dict(ranges=w.ranges, angle_min=w.angle_min, angle_increment=w.angle_increment,
                range_min=w.range_min, range_max=w.range_max)


def test_failures_leave_context_usable():
    w1 = make_config(1)
    k1 = oracle.edt(w1.occ)
    hyp = oracle.sample(w1.occ, k1, w1.resolution, n_target=300, seed=1, min_spacing=0.3,
                        robot_radius=0.21)
    w2 = make_config(2)
    ctx = reloc.Context(0, hbm_budget=40 << 20)
    try:
        _case("failures: small map and request in a 40 MB context")
        m = ctx.load_map(w1.occ, w1.resolution)
        sid = ctx.set_hypotheses(m, hyp)
        kw = dict(n_theta=360, batch_k=10, tau=0.95, k_out=10)
        first, st0 = ctx.relocalize(m, sid, **_scan(w1), **kw)
        held = ctx.bytes

        def refused(code, fn, *a, **k):
            with pytest.raises(reloc.RelocError) as ei:
                fn(*a, **k)
            assert ei.value.code == code, (ei.value.code, str(ei.value))
            assert ctx.bytes == held

        _case("failures: map beyond the budget")
        refused(reloc.E_NOMEM, ctx.load_map, w2.occ, w2.resolution)
        _case("failures: malformed and empty scans, bad parameters")
        bad = dict(_scan(w1), angle_increment=math.radians(0.7))
        refused(reloc.E_BEAMGRID, ctx.prepare, m, sid, **bad, **kw)
        nan = dict(_scan(w1), ranges=np.full(len(w1.ranges), np.nan, np.float32))
        refused(reloc.E_EMPTY, ctx.prepare, m, sid, **nan, **kw)
        refused(reloc.E_INVALID, ctx.prepare, m, sid, **_scan(w1), n_theta=360, batch_k=0)
        refused(reloc.E_INVALID, ctx.prepare, m, sid, **_scan(w1), n_theta=360, refine_k=65)
        _case("failures: unknown and released requests, busy map")
        refused(reloc.E_NOTFOUND, ctx.run, 12345)
        rid = ctx.prepare(m, sid, **_scan(w1), **kw)
        _case("failures: debug TAM rank ranges outside the request (C ABI, no outputs)")
        nh = len(hyp)
        with_req = ctx.bytes
        for r0, n in ((1, 2**31 - 1), (2**31 - 1, 1), (-1, 5), (0, 0), (nh, 1), (0, nh + 1)):
            rc = ctx._lib.reloc_debug_tam(ctx._h, rid, r0, n, None, None, None)
            assert rc == reloc.E_INVALID, (r0, n, rc)
            assert ctx.bytes == with_req
        ctx.release(rid)
        assert ctx.bytes == held
        refused(reloc.E_NOTFOUND, ctx.release, rid)
        refused(reloc.E_BUSY, ctx.unload_map, m)
        _case("failures: the context still relocalizes identically")
        again, st1 = ctx.relocalize(m, sid, **_scan(w1), **kw)
        assert again == first
        for f in ("stages", "n_eval", "early_stopped", "smad_evals", "tam_evals"):
            assert st0[f] == st1[f]
        ctx.free_hypotheses(sid)
        ctx.unload_map(m)
        assert ctx.bytes < held
    finally:
        ctx.close()
