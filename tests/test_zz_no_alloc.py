"""The no-allocation entry point (reloc_relocalize_noalloc) against
reloc_relocalize, through the C ABI: two calls in a row, the second with a
smaller request, each giving bit-identical poses and statistics; a search
that ranks more than 2048 evaluated poses (the library radix sort with its
scratch carved from the region); a request that does not fit the region is
refused before any device work, and the context keeps working."""
import sys

import numpy as np
import pytest

import paper_2511_01219_amd as reloc
from synth import make_config

pytestmark = pytest.mark.gpu

_KEYS = ("hyp", "k", "rank", "stage", "cx", "cy", "g", "refined")
_STATS = ("n_hyp", "stages", "early_stopped", "n_eval", "smad_evals", "tam_evals", "rays",
          "tam_lookups", "ambiguous")


def _case(msg):
    print("[gpu case] " + msg, flush=True)
    sys.stdout.flush()


def _same(a, b):
    pa, sa = a
    pb, sb = b
    assert len(pa) == len(pb) > 0
    for x, y in zip(pa, pb):
        for k in _KEYS:
            assert x[k] == y[k], (k, x, y)
        assert np.float32(x["tam"]).view(np.uint32) == np.float32(y["tam"]).view(np.uint32)
        assert np.float32(x["smad"]).view(np.uint32) == np.float32(y["smad"]).view(np.uint32)
        assert x["x"] == y["x"] and x["y"] == y["y"] and x["theta"] == y["theta"]
    for k in _STATS:
        assert sa[k] == sb[k], (k, sa[k], sb[k])
    assert np.float32(sa["best_margin"]) == np.float32(sb["best_margin"])


def _setup(ctx, cid):
    w = make_config(cid)
    m = ctx.load_map(w.occ, w.resolution, w.origin)
    s = w.sample
    sid, _ = ctx.sample_hypotheses(m, s["n_target"], s["min_spacing"], s["robot_radius"],
                                   seed=s["seed"])
    scan = (w.ranges, w.angle_min, w.angle_increment, w.range_min, w.range_max)
    return w, m, sid, scan


def test_noalloc_matches_relocalize():
    ctx = reloc.Context(0)
    try:
        w2, m2, s2, scan2 = _setup(ctx, 2)
        w1, m1, s1, scan1 = _setup(ctx, 1)
        # 1: plain-large (20 000 hypotheses), then 2: plain-small (300)
        for tag, m, sid, scan, kw in (("plain-large", m2, s2, scan2, w2.search),
                                      ("plain-small", m1, s1, scan1, w1.search)):
            _case("no-alloc vs relocalize: %s" % tag)
            ref = ctx.relocalize(m, sid, *scan, k_out=10, **kw)
            got = ctx.relocalize_noalloc(m, sid, *scan, k_out=10, **kw)
            _same(got, ref)
        # a search without early termination ranks every evaluated pose (6000,
        # beyond the 2048 of the one-workgroup ranking)
        _case("no-alloc vs relocalize: plain-large, tau none, 6000 hypotheses")
        kw = dict(w2.search, tau=None, n_hyp=6000)
        ref = ctx.relocalize(m2, s2, *scan2, k_out=20, **kw)
        got = ctx.relocalize_noalloc(m2, s2, *scan2, k_out=20, **kw)
        assert got[1]["n_eval"] == 6000
        _same(got, ref)
        # the split ray cast of CAER needs 4 Ns bytes per hypothesis: 77 MB
        # at plain-large, beyond the 64 MiB region
        _case("no-alloc refuses a request beyond its scratch")
        before = ctx.bytes
        with pytest.raises(reloc.RelocError) as ei:
            ctx.relocalize_noalloc(m2, s2, *scan2, k_out=10, coarse_metric=2, **w2.search)
        assert ei.value.code == reloc.E_NOMEM
        assert "scratch" in str(ei.value)
        assert ctx.bytes == before
        _case("no-alloc after a refusal: plain-small again")
        _same(ctx.relocalize_noalloc(m1, s1, *scan1, k_out=10, **w1.search),
              ctx.relocalize(m1, s1, *scan1, k_out=10, **w1.search))
        for sid, m in ((s1, m1), (s2, m2)):
            ctx.free_hypotheses(sid)
            ctx.unload_map(m)
    finally:
        ctx.close()
