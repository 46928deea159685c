"""Boundary checks that need no GPU: the C-ABI library loads, exports every
function declared in include/reloc.h, its host-side scan preprocessing agrees
with the oracle's, and device entry points fail cleanly without a device."""
import math
import os
import re

import numpy as np
import pytest

import oracle
import paper_2511_01219_amd as reloc
from paper_2511_01219_amd import _abi
from synth import make_config

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _declared_functions():
    src = open(os.path.join(ROOT, "include", "reloc.h")).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"\b(reloc_[a-z_]+)\s*\(", src)))


def test_header_declares_the_three_calls():
    names = _declared_functions()
    for n in ("reloc_load_map", "reloc_sample_hypotheses", "reloc_relocalize"):
        assert n in names


def test_library_exports_every_declared_function():
    lib = reloc.lib()
    for n in _declared_functions():
        assert hasattr(lib, n), n
    assert set(_declared_functions()) == set(_abi.PROTOS), "binding and header differ"


def test_struct_layouts_match_c(tmp_path):
    # sizes and field offsets as the C compiler lays out include/reloc.h
    import ctypes
    import subprocess
    structs = ["reloc_allocator", "reloc_map_desc", "reloc_sample_params",
               "reloc_interval", "reloc_scan", "reloc_search_params", "reloc_scan_info",
               "reloc_pose", "reloc_stats", "reloc_serve_config", "reloc_serve_stats",
               "reloc_rrt_params", "reloc_rrt_info", "reloc_peaks"]
    lines = ['#include <stdio.h>', '#include <stddef.h>', '#include "reloc.h"',
             'int main(void) {']
    for st in structs:
        lines.append('printf("%s %%zu\\n", sizeof(%s));' % (st, st))
        for f, _ in getattr(_abi, st)._fields_:
            cf = "lambda" if f == "lambda_" else f
            lines.append('printf("%s.%s %%zu\\n", offsetof(%s, %s));' % (st, f, st, cf))
    lines.append("return 0; }")
    src = tmp_path / "layout.c"
    src.write_text("\n".join(lines))
    exe = tmp_path / "layout"
    subprocess.check_call(["gcc", "-I", os.path.join(ROOT, "include"), str(src), "-o", str(exe)])
    out = subprocess.check_output([str(exe)]).decode().split()
    got = dict(zip(out[::2], map(int, out[1::2])))
    for st in structs:
        cls = getattr(_abi, st)
        assert ctypes.sizeof(cls) == got[st], st
        for f, _ in cls._fields_:
            assert getattr(cls, f).offset == got["%s.%s" % (st, f)], (st, f)


def test_version_and_error_text():
    assert reloc.version() == 1
    assert isinstance(reloc.lib().reloc_last_error(), bytes)


def test_ctx_create_without_device_is_an_error():
    with pytest.raises(reloc.RelocError) as ei:
        reloc.Context(use_torch=False)
    assert ei.value.code == reloc.E_DEVICE


def _both(ranges, amin, inc, res=0.05, fov=None, rmin=0.02, rmax=20.0, **kw):
    a = reloc.scan_info(ranges, amin, inc, res, rmin, rmax, fov=fov, **kw)
    b = oracle.prep(ranges, amin, inc, res, fov=fov, range_min=rmin, range_max=rmax,
                    n_skip_beam=kw.get("n_skip_beam", 1), n_skip_enum=kw.get("n_skip_enum", 1),
                    n_theta=kw.get("n_theta", 0),
                    alpha_mid_pm=kw.get("alpha_mid_pm", (900, 700)),
                    alpha_low_pm=kw.get("alpha_low_pm", (700, 500)))
    return a, b


@pytest.mark.parametrize("cid", [1, 2, 5])
def test_scan_info_matches_oracle_on_workloads(cid):
    w = make_config(cid, n_target=10)
    nt = {1: 360, 2: 720, 5: 1440}[cid]
    a, b = _both(w.ranges, w.angle_min, w.angle_increment, w.resolution,
                 rmin=w.range_min, rmax=w.range_max, n_theta=nt)
    assert b["status"] == 0
    for ka, kb in (("Ns", "Ns"), ("Ntheta", "Ntheta"), ("Ng", "Ng"), ("n_fov", "N_fov"),
                   ("n_valid", "N_valid"), ("k_mid", "k_mid"), ("k_low", "k_low"),
                   ("k_full", "k_full"), ("n_shifts", "n_shifts"), ("j0", "j0"),
                   ("n_runs", "n_runs"), ("n_down", "n_down")):
        assert a[ka] == b[kb], ka
    assert a["zbar"] == b["zbar"]
    assert bool(a["panoramic"]) == b["panoramic"]


@pytest.mark.parametrize("seed", range(6))
def test_scan_info_matches_oracle_random(seed):
    rng = np.random.default_rng(seed)
    fov_deg = [90.0, 180.0, 240.0, 270.0, 360.0, 220.0][seed]
    n = [120, 360, 320, 720, 1440, 440][seed]
    inc = math.radians(fov_deg) / n
    amin = -math.pi if fov_deg == 360 else -math.radians(fov_deg) / 2
    z = (rng.random(n) * 15).astype(np.float32)
    z[rng.random(n) < 0.1] = np.nan
    z[rng.random(n) < 0.05] = 50.0
    fov = None
    if seed % 2:
        fov = [(amin, amin + 0.3 * math.radians(fov_deg)),
               (amin + 0.45 * math.radians(fov_deg), amin + math.radians(fov_deg))]
    kw = dict(n_theta=[0, 360, 720, 360, 1440, 0][seed], n_skip_beam=1 + seed % 3,
              n_skip_enum=1 + (seed % 2), alpha_mid_pm=(900, 650), alpha_low_pm=(720, 480))
    try:
        a, b = _both(z, amin, inc, fov=fov, **kw)
    except reloc.RelocError as e:
        b = oracle.prep(z, amin, inc, 0.05, fov=fov, range_max=20.0,
                        n_skip_beam=kw["n_skip_beam"], n_skip_enum=kw["n_skip_enum"],
                        n_theta=kw["n_theta"], alpha_mid_pm=kw["alpha_mid_pm"],
                        alpha_low_pm=kw["alpha_low_pm"])
        assert e.code == b["status"]
        return
    assert (a["Ns"], a["n_valid"], a["k_mid"], a["k_low"], a["n_fov"], a["n_runs"]) == \
        (b["Ns"], b["N_valid"], b["k_mid"], b["k_low"], b["N_fov"], b["n_runs"])
    assert a["zbar"] == b["zbar"]


def test_scan_info_errors_match_oracle_codes():
    z = np.full(100, 2.0, np.float32)
    with pytest.raises(reloc.RelocError) as ei:
        reloc.scan_info(z, 0.0, math.radians(0.7), 0.05)
    assert ei.value.code == reloc.E_BEAMGRID == oracle.E_BEAMGRID
    with pytest.raises(reloc.RelocError) as ei:
        reloc.scan_info(np.full(100, np.nan, np.float32), 0.0, math.radians(1.0), 0.05)
    assert ei.value.code == reloc.E_EMPTY == oracle.E_EMPTY
    with pytest.raises(reloc.RelocError) as ei:
        reloc.scan_info(z, 0.0, math.radians(1.0), 0.05, range_max=80.0)
    assert ei.value.code == reloc.E_INVALID
    with pytest.raises(reloc.RelocError) as ei:
        reloc.scan_info(z, 0.0, 2 * math.pi / 8192, 0.05)
    assert ei.value.code == reloc.E_INVALID        # Ns above the 4096 limit


def test_alpha_order_refused_on_both_sides():
    """Eq. 25 orders alpha_low < alpha_mid. The library's top-k_mid mean is
    the median of eq. 27 only when k_low <= k_mid, so misordered alphas are
    refused before any work, by the library and by the oracle; equal alphas
    (k_low == k_mid) and the defaults are accepted."""
    z = np.full(360, 2.0, np.float32)
    inc = 2 * math.pi / 360
    for mid, low in (((900, 700), (700, 500)), ((800, 600), (800, 600)), ((900, 700), (100, 100))):
        a, b = _both(z, -math.pi, inc, alpha_mid_pm=mid, alpha_low_pm=low)
        assert b["status"] == 0 and a["k_low"] == b["k_low"] <= a["k_mid"] == b["k_mid"]
    for mid, low in (((900, 700), (901, 500)), ((900, 700), (700, 701)),
                     ((500, 500), (900, 100))):
        with pytest.raises(reloc.RelocError) as ei:
            reloc.scan_info(z, -math.pi, inc, 0.05, alpha_mid_pm=mid, alpha_low_pm=low)
        assert ei.value.code == reloc.E_INVALID, (mid, low)
        b = oracle.prep(z, -math.pi, inc, 0.05, alpha_mid_pm=mid, alpha_low_pm=low)
        assert b["status"] == oracle.E_INVALID, (mid, low)


def test_search_param_defaults():
    p = reloc.search_params()
    assert (p.batch_k, p.k_out, p.tau, p.z_hit, p.sigma_hit, p.z_rand, p.d_max) == \
        (64, 10, 0.95, 1.0, 0.2, 0.0, 2.0)
    assert tuple(p.alpha_mid_pm) == (900, 700) and tuple(p.alpha_low_pm) == (700, 500)
    q = reloc.search_params(tau=None)
    assert math.isnan(q.tau)
    assert (p.refine_k, p.refine_cells, p.refine_dirs) == (0, 3, -1)
    assert (p.coarse_metric, p.fine_metric) == (0, 0)
    assert p.use_graph == 0   # the head graph is opt-in


def test_metric_choices_checked_on_host():
    z = np.full(360, 2.0, np.float32)
    inc = 2 * math.pi / 360
    for cm in range(4):
        for fm in range(4):
            reloc.scan_info(z, -math.pi, inc, 0.05, coarse_metric=cm, fine_metric=fm)
    for kw in (dict(coarse_metric=4), dict(coarse_metric=-1), dict(fine_metric=4),
               dict(fine_metric=-1)):
        with pytest.raises(reloc.RelocError) as ei:
            reloc.scan_info(z, -math.pi, inc, 0.05, **kw)
        assert ei.value.code == reloc.E_INVALID, kw


def test_refinement_limits():
    """Refinement parameters are checked on the host: refine_k in 0..64,
    refine_cells in 0..15, refine_dirs >= -1 and below Ng, and the lattice
    (2s + 1)(2h + 1)^2 at most 65536 points."""
    z = np.full(360, 2.0, np.float32)
    inc = 2 * math.pi / 360

    def info(**kw):
        return reloc.scan_info(z, -math.pi, inc, 0.05, n_theta=90, **kw)

    assert info(refine_k=64, refine_cells=15, refine_dirs=-1)["Ng"] == 360
    assert info(refine_k=1, refine_cells=15, refine_dirs=33)["Ng"] == 360   # 67 * 961 points
    for kw in (dict(refine_k=65), dict(refine_k=-1), dict(refine_k=1, refine_cells=16),
               dict(refine_k=1, refine_cells=-1), dict(refine_k=1, refine_dirs=-2),
               dict(refine_k=1, refine_dirs=360), dict(refine_k=1, refine_cells=15,
                                                      refine_dirs=34)):
        with pytest.raises(reloc.RelocError) as ei:
            info(**kw)
        assert ei.value.code == reloc.E_INVALID, kw


def test_null_context_calls_are_invalid():
    """Every entry point rejects a null context with RELOC_E_INVALID and
    writes zero counts; no device is needed."""
    import ctypes as C
    lib = reloc.lib()
    n = C.c_int32(7)
    st = np.zeros(4, np.int32)
    assert lib.reloc_run(None, 1, None, 0, C.byref(n), None) == reloc.E_INVALID
    assert n.value == 0
    ids = np.array([1, 2], np.int32)
    n_out = np.full(2, 9, np.int32)
    assert lib.reloc_run_batch(None, 2, ids.ctypes.data, None, 0, n_out.ctypes.data,
                               st.ctypes.data, None) == reloc.E_INVALID
    t = C.c_uint64(5)
    assert lib.reloc_submit(None, 1, 1, None, None, C.byref(t)) == reloc.E_INVALID
    assert t.value == 0
    n.value = 3
    assert lib.reloc_poll(None, 1, 0, None, 0, C.byref(n), None) == reloc.E_INVALID
    assert lib.reloc_serve_configure(None, None) == reloc.E_INVALID
    assert lib.reloc_serve_stats_get(None, None) == reloc.E_INVALID
    assert lib.reloc_prepare(None, 1, 1, None, None, C.byref(n)) == reloc.E_INVALID
    assert lib.reloc_release(None, 1) == reloc.E_INVALID
    sid = C.c_int32(4)
    n.value = 6
    p = _abi.reloc_rrt_params()
    lib.reloc_rrt_defaults(C.byref(p))
    assert (p.rho, p.robot_radius, p.eta_max, p.eps_gain) == (0.3, 0.21, 0.6, 2)
    assert lib.reloc_sample_rrt(None, 1, C.byref(p), C.byref(sid), C.byref(n), None, None,
                                None, 0) == reloc.E_INVALID
    assert n.value == 0
    assert lib.reloc_coarse_scores(None, 1, 0, None, None, None, None) == reloc.E_INVALID
    ms = C.c_float(3.0)
    assert lib.reloc_score_poses(None, 1, None, None, 0, None, C.byref(ms)) == reloc.E_INVALID
    assert ms.value == 0.0


def test_multi_map_generators_are_seeded():
    """The batched and serving workloads are functions of their seeds: two
    calls give identical maps, queries and arrival times."""
    from synth import make_batched, make_serving
    a = make_batched(6, sizes=(120, 160), n_range=(50, 500))
    b = make_batched(6, sizes=(120, 160), n_range=(50, 500))
    assert all((x == y).all() for x, y in zip(a.maps, b.maps))
    for p, q in zip(a.queries, b.queries):
        assert p.map_index == q.map_index and p.n_hyp == q.n_hyp and p.pose == q.pose
        assert np.array_equal(p.ranges, q.ranges, equal_nan=True)
        assert (360.0 * p.n_beams / p.fov_deg) == int(360.0 * p.n_beams / p.fov_deg)
    s1 = make_serving(100.0, 8, sizes=(120,), per_size=2, n_range=(50, 500))
    s2 = make_serving(100.0, 8, sizes=(120,), per_size=2, n_range=(50, 500))
    arr = [q.arrival for q in s1.queries]
    assert arr == [q.arrival for q in s2.queries]
    assert arr[0] == 0.0 and all(x < y for x, y in zip(arr, arr[1:]))
