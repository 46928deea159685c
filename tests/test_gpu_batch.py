"""GPU tests of the batched form (reloc_run_batch) and of serving
(reloc_submit / reloc_poll), through the C ABI.

Bars:
  * every request's result in a batch or in the served mix is bit-identical
    to the plain one-request path (poses, T bits, ranks, stages, n_eval);
  * each served result is the same alone and in a mix;
  * against the FP64 oracle, the batched results meet the plain path's bars
    (ray-cast hit cells bit-exact, SMAD order identical, TAM within 1e-4).
"""
import math
import sys

import numpy as np
import pytest

import oracle
import paper_2511_01219_amd as reloc
from synth import make_batched, make_serving

pytestmark = pytest.mark.gpu

T_RTOL, T_ATOL = 1e-4, 1e-7


def _case(msg):
    print("[gpu case] " + msg, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def ctx():
    c = reloc.Context(0)
    yield c
    c.close()


@pytest.fixture(scope="module")
def multi():
    # two map sizes, rooms and warehouse each; hypothesis counts span 40 to
    # 3000 so that stage counts and TAM kernel classes differ between queries
    return make_batched(12, sizes=(160, 260), n_range=(40, 3000))


@pytest.fixture(scope="module")
def loaded(ctx, multi):
    mids, sids = [], []
    for m, occ in enumerate(multi.maps):
        mid = ctx.load_map(occ, multi.resolution)
        sid, _ = ctx.sample_hypotheses(mid, multi.sample["n_target"][m], 0.3, 0.21,
                                       seed=multi.sample["seeds"][m])
        mids.append(mid)
        sids.append(sid)
    yield mids, sids
    for mid, sid in zip(mids, sids):
        ctx.free_hypotheses(sid)
        ctx.unload_map(mid)


def _args(q):
    return dict(ranges=q.ranges, angle_min=q.angle_min, angle_increment=q.angle_increment,
                range_min=q.range_min, range_max=q.range_max)


def _search(q, **over):
    s = dict(q.search)
    s["n_hyp"] = q.n_hyp
    s.update(over)
    return s


def _prepare(ctx, loaded, q, **over):
    mids, sids = loaded
    return ctx.prepare(mids[q.map_index], sids[q.map_index], **_args(q), **_search(q, **over))


def _same(a, b):
    pa, sa = a
    pb, sb = b
    assert len(pa) == len(pb)
    for x, y in zip(pa, pb):
        for f in ("hyp", "k", "rank", "stage", "x", "y", "theta"):
            assert x[f] == y[f], (f, x, y)
        assert np.float32(x["tam"]).view(np.uint32) == np.float32(y["tam"]).view(np.uint32)
        assert np.float32(x["smad"]).view(np.uint32) == np.float32(y["smad"]).view(np.uint32)
    for f in ("n_hyp", "stages", "early_stopped", "n_eval", "smad_evals", "tam_evals", "rays"):
        assert sa[f] == sb[f], (f, sa[f], sb[f])


@pytest.mark.parametrize("tau", [0.95, None, 0.3])
def test_batch_equals_plain(ctx, multi, loaded, tau):
    _case("batch == plain, %d queries, tau=%s" % (len(multi.queries), tau))
    rids = [_prepare(ctx, loaded, q, tau=tau, k_out=12) for q in multi.queries]
    plain = [ctx.run(r, cap=16) for r in rids]
    batch = ctx.run_batch(rids, cap=16)
    for a, b in zip(plain, batch):
        _same(a, b)
        assert b[1]["status"] == reloc.OK
    # twice in a row: identical again
    again = ctx.run_batch(rids[::-1], cap=16)
    for a, b in zip(plain[::-1], again):
        _same(a, b)
    for r in rids:
        ctx.release(r)


def test_batch_one_and_errors(ctx, multi, loaded):
    q = multi.queries[0]
    _case("batch of one")
    r = _prepare(ctx, loaded, q)
    _same(ctx.run(r), ctx.run_batch([r])[0])
    assert ctx.run_batch([]) == []
    with pytest.raises(reloc.RelocError) as ei:
        ctx.run_batch([r, r])
    assert ei.value.code == reloc.E_INVALID
    with pytest.raises(reloc.RelocError) as ei:
        ctx.run_batch([r, 987654])
    assert ei.value.code == reloc.E_NOTFOUND
    ctx.release(r)


def test_batch_matches_oracle(ctx, multi, loaded):
    """Ray-cast hit cells and SMAD order bit-exact, stage counts and best pose
    as the oracle's, for three queries of different maps run as one batch."""
    mids, sids = loaded
    qs = [q for q in multi.queries if q.n_hyp <= 1500][:3]
    assert len(qs) >= 2
    rids = [_prepare(ctx, loaded, q, tau=None, k_out=5) for q in qs]
    _case("batch vs oracle: %s" % [(q.map_index, q.n_hyp, q.fov_deg, q.n_beams) for q in qs])
    res = ctx.run_batch(rids, cap=5)
    for q, rid, (poses, st) in zip(qs, rids, res):
        occ = multi.maps[q.map_index]
        hyp = ctx.read_hypotheses(sids[q.map_index])[:st["n_hyp"]]
        k = oracle.edt(occ)
        pr = oracle.prep(q.ranges, q.angle_min, q.angle_increment, multi.resolution,
                         range_min=q.range_min, range_max=q.range_max, n_theta=360)
        hit, _ = oracle.raycast(occ, hyp, pr["Ns"], pr["Ng"], multi.resolution, q.range_max,
                                threads=16)
        ghit, _ = ctx.debug_raycast(rid, len(hyp), pr["Ns"])
        assert (ghit == hit).all()
        _, zhat = oracle.raycast(occ, hyp, pr["Ns"], pr["Ng"], multi.resolution, q.range_max,
                                 threads=16)
        sm, _ = oracle.smad(zhat, pr, threads=16)
        ref = oracle.stages(k, multi.resolution, pr, hyp, sm, 64, None, all_T=True, threads=16)
        assert st["n_eval"] == ref["n_eval"] == len(hyp)
        ro = np.lexsort((np.arange(ref["n_eval"]), -ref["tstar"]))
        best = ro[0]
        tied = [r for r in ro[:5] if ref["tstar"][r] >= ref["tstar"][best] * (1 - 2e-4)]
        assert poses[0]["rank"] in tied
        assert int(ref["order"][poses[0]["rank"]]) == poses[0]["hyp"]
        r0 = poses[0]["rank"]
        assert abs(poses[0]["tam"] - ref["tstar"][r0]) <= T_RTOL * ref["tstar"][r0] + T_ATOL
        ctx.release(rid)


def test_serve_alone_and_in_mix(ctx, multi, loaded):
    mids, sids = loaded
    qs = multi.queries
    _case("serve: plain references")
    ref = []
    for q in qs:
        r = _prepare(ctx, loaded, q)
        ref.append(ctx.run(r))
        ctx.release(r)
    _case("serve: query 3 alone")
    t = ctx.submit(mids[qs[3].map_index], sids[qs[3].map_index], **_args(qs[3]),
                   **_search(qs[3]))
    alone = ctx.poll(t, wait_ms=60000)
    assert alone is not None
    _same(alone, ref[3])
    _case("serve: all queries submitted together")
    tickets = [ctx.submit(mids[q.map_index], sids[q.map_index], **_args(q), **_search(q))
               for q in qs]
    got = [ctx.poll(t, wait_ms=60000) for t in tickets]
    for g, r in zip(got, ref):
        assert g is not None
        _same(g, r)
    _same(got[3], alone)
    st = ctx.serve_stats()
    assert st["completed"] >= len(qs) + 1 and st["queued"] == 0 and st["inflight"] == 0
    with pytest.raises(reloc.RelocError) as ei:
        ctx.poll(tickets[0], wait_ms=0)
    assert ei.value.code == reloc.E_NOTFOUND


def test_serve_admission_limits(ctx, multi, loaded):
    mids, sids = loaded
    qs = multi.queries[:6]
    ref = []
    for q in qs:
        r = _prepare(ctx, loaded, q)
        ref.append(ctx.run(r))
        ctx.release(r)
    _case("serve: max_inflight 2, max_admit 1")
    ctx.serve_configure(max_inflight=2, max_admit=1)
    try:
        t0 = ctx.serve_stats()["ticks"]
        tickets = [ctx.submit(mids[q.map_index], sids[q.map_index], **_args(q), **_search(q))
                   for q in qs]
        got = [ctx.poll(t, wait_ms=60000) for t in tickets]
        for g, r in zip(got, ref):
            _same(g, r)
        assert ctx.serve_stats()["ticks"] - t0 >= len(qs)
        _case("serve: request larger than the budget fails with E_NOMEM")
        ctx.serve_configure(max_inflight=4, hbm_reserve=1 << 62, max_admit=4)
        t = ctx.submit(mids[qs[0].map_index], sids[qs[0].map_index], **_args(qs[0]),
                       **_search(qs[0]))
        with pytest.raises(reloc.RelocError) as ei:
            ctx.poll(t, wait_ms=60000)
        assert ei.value.code == reloc.E_NOMEM
    finally:
        ctx.serve_configure()


def _check_oracle(poses, st, occ, k, hyp, q, res, K=64, tau=0.95):
    """A result against the full oracle path (ray cast, direct-sum SMAD,
    order, stage loop): stop stage and evaluated count identical unless the
    deciding batch best lies within 1e-4 of tau; best pose identical up to
    the tie rule, T within 1e-4; every pose the oracle's hypothesis at its
    rank with bit-identical FP32 SMAD."""
    pr = oracle.prep(q.ranges, q.angle_min, q.angle_increment, res, range_min=q.range_min,
                     range_max=q.range_max, n_theta=360)
    _, zhat = oracle.raycast(occ, hyp, pr["Ns"], pr["Ng"], res, q.range_max, threads=16)
    sm, _ = oracle.smad(zhat, pr, threads=16)
    ref = oracle.stages(k, res, pr, hyp, sm, K, tau, all_T=True, threads=16)
    for p in poses:
        assert int(ref["order"][p["rank"]]) == p["hyp"]
        assert np.float32(p["smad"]) == np.float32(sm[p["hyp"]])
    if ref["early_stopped"] != bool(st["early_stopped"]) or ref["stages"] != st["stages"]:
        s = min(ref["stages"], st["stages"]) - 1
        tb = ref["tstar"][s * K:(s + 1) * K].max()
        assert tau is not None and abs(tb - tau) <= 1e-4, (ref["stages"], st["stages"])
        return
    assert st["n_eval"] == ref["n_eval"]
    ro = np.lexsort((np.arange(ref["n_eval"]), -ref["tstar"]))
    best = ro[0]
    tied = [r for r in ro[:5] if ref["tstar"][r] >= ref["tstar"][best] * (1 - 2e-4)]
    b = poses[0]
    assert b["rank"] in tied
    assert abs(b["tam"] - ref["tstar"][b["rank"]]) <= T_RTOL * ref["tstar"][b["rank"]] + T_ATOL
    if b["rank"] == best:
        assert b["k"] == ref["kstar"][best] or \
            abs(ref["all_T"][best][b["k"]] - ref["tstar"][best]) <= 2e-4 * ref["tstar"][best]


def test_serve_poisson_trace_small(ctx):
    """A short Poisson trace on its own maps: every served result equals the
    plain path's and meets the oracle's bars (the full oracle path run for
    each request)."""
    w = make_serving(200.0, 10, sizes=(200,), per_size=2, n_range=(100, 2000))
    mids, sids = [], []
    for m, occ in enumerate(w.maps):
        mid = ctx.load_map(occ, w.resolution)
        sid, _ = ctx.sample_hypotheses(mid, w.sample["n_target"][m], 0.3, 0.21,
                                       seed=w.sample["seeds"][m])
        mids.append(mid)
        sids.append(sid)
    _case("serve poisson: %d requests" % len(w.queries))
    tickets = [ctx.submit(mids[q.map_index], sids[q.map_index], **_args(q), **_search(q))
               for q in w.queries]
    got = [ctx.poll(t, wait_ms=60000) for t in tickets]
    kmaps = [oracle.edt(occ) for occ in w.maps]
    for i, (q, g) in enumerate(zip(w.queries, got)):
        r = ctx.prepare(mids[q.map_index], sids[q.map_index], **_args(q), **_search(q))
        _same(g, ctx.run(r))
        ctx.release(r)
        _case("serve poisson: request %d against the oracle" % i)
        hyp = ctx.read_hypotheses(sids[q.map_index])[:q.n_hyp]
        _check_oracle(g[0], g[1], w.maps[q.map_index], kmaps[q.map_index], hyp, q,
                      w.resolution)
    for mid, sid in zip(mids, sids):
        ctx.free_hypotheses(sid)
        ctx.unload_map(mid)


def test_batch_tam_mixed_beam_tables(ctx):
    """Regression: one TAM class launch serving two requests whose beam
    tables differ in length (about 1045 and 1950 valid beams, both in the
    32-keys-per-lane class). Every gather batch reads only the request's own
    padded table; results equal the plain path's."""
    from synth import ScanSpec, lidar_scan, make_config
    w = make_config(1)
    mid = ctx.load_map(w.occ, w.resolution)
    sid, _ = ctx.sample_hypotheses(mid, 200, 0.3, 0.21, seed=11)
    rids = []
    for n_beams in (1100, 2048, 1100):
        spec = ScanSpec(360.0, n_beams, 12.0, 0.02, 0.02, 0.05, 0.0)
        ranges, amin, ainc, _ = lidar_scan(w.occ, w.resolution, w.origin, w.pose, spec,
                                           np.random.default_rng([11, n_beams]))
        rids.append(ctx.prepare(mid, sid, ranges, amin, ainc, 0.02, 12.0, n_theta=360,
                                batch_k=16, tau=None, k_out=8))
    _case("batch TAM with mixed beam tables: 1100, 2048, 1100 beams")
    plain = [ctx.run(r, cap=8) for r in rids]
    batch = ctx.run_batch(rids, cap=8)
    for a, b in zip(plain, batch):
        _same(a, b)
    for r in rids:
        ctx.release(r)
    ctx.free_hypotheses(sid)
    ctx.unload_map(mid)


def test_batch_and_serve_deadline(ctx, multi, loaded):
    """deadline_s in the batched form and in serving: the request ends with
    E_TIMEOUT after the stages it ran and returns their ranking."""
    mids, sids = loaded
    q = max(multi.queries, key=lambda x: x.n_hyp)
    _case("deadline batch / serve: %d hypotheses" % q.n_hyp)
    r = _prepare(ctx, loaded, q, tau=None, batch_k=4, deadline_s=1e-9)
    (poses, st), = ctx.run_batch([r])
    assert st["status"] == reloc.E_TIMEOUT
    assert 0 < st["n_eval"] < st["n_hyp"] and len(poses) > 0
    ctx.release(r)
    t = ctx.submit(mids[q.map_index], sids[q.map_index], **_args(q),
                   **_search(q, tau=None, batch_k=4, deadline_s=1e-9))
    poses, st = ctx.poll(t, wait_ms=60000)
    assert st["status"] == reloc.E_TIMEOUT
    assert 0 < st["n_eval"] < st["n_hyp"] and len(poses) > 0


def test_batch_and_serve_far_cells(ctx):
    """An open hall where most endpoints lie 128 or more cells from any
    obstacle, so the TAM kernels take the escape path through the 32-bit
    plane: batched and served results equal the plain path's (which the
    parity tests hold to the oracle on such maps), with 2 kcap below and
    above 2^15 and a full search."""
    W, H = 700, 600
    occ = np.zeros((H, W), np.int8)
    occ[0, :] = occ[H - 1, :] = 100
    occ[:, 0] = occ[:, W - 1] = 100
    occ[280:300, 150:200] = 100
    k = oracle.edt(occ)
    assert (k >= (1 << 14)).mean() > 0.2
    rng = np.random.default_rng(5)
    xs = np.concatenate([rng.integers(250, 450, 150), rng.integers(3, 40, 30)])
    ys = np.concatenate([rng.integers(200, 400, 150), rng.integers(3, 40, 30)])
    keep = occ[ys, xs] == 0
    hyp = np.unique(np.stack([xs[keep], ys[keep]], 1).astype(np.int32), axis=0)
    m = ctx.load_map(occ, 0.05)
    sid = ctx.set_hypotheses(m, hyp)
    inc = 2 * math.pi / 360
    cases = []
    for i, params in enumerate([dict(), dict(sigma_hit=1.0), dict(tau=None)]):
        z = np.full(360, 3.0 + i, np.float32)
        z[::3] = 12.0
        z[1::3] = 25.0
        scan = dict(ranges=z, angle_min=-math.pi, angle_increment=inc, range_min=0.02,
                    range_max=40.0)
        search = dict(n_theta=90, batch_k=16, tau=0.95, k_out=8)
        search.update(params)
        cases.append((scan, search))
    _case("far cells: %d hypotheses, plain and batched" % len(hyp))
    rids = [ctx.prepare(m, sid, **sc, **se) for sc, se in cases]
    plain = [ctx.run(r) for r in rids]
    for a, b in zip(plain, ctx.run_batch(rids)):
        _same(a, b)
    _case("far cells: served")
    tickets = [ctx.submit(m, sid, **sc, **se) for sc, se in cases]
    for t, a in zip(tickets, plain):
        got = ctx.poll(t, wait_ms=60000)
        assert got is not None
        _same(got, a)
    for r in rids:
        ctx.release(r)
    ctx.free_hypotheses(sid)
    ctx.unload_map(m)
