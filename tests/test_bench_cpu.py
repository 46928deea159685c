"""Host-side checks of the benchmark script (no GPU): it refuses more than
one GPU, its accuracy report applies the success criterion of Sec. IV-C
(position error below 0.5 m and heading error below 30 deg, headings
compared on the circle), and the committed HBM-traffic summary belongs to
the committed ray-cast sources (else the benchmark would report null)."""
import math
import os
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)
import bench  # noqa: E402


def test_more_than_one_gpu_is_refused():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"],
                       capture_output=True, text=True, timeout=120)
    assert r.returncode == 2
    assert "one GPU" in r.stderr
    assert r.stdout == ""


@pytest.mark.parametrize("dx,dth,ok", [
    (0.49, math.radians(29.0), True),
    (0.5001, 0.0, False),
    (0.0, math.radians(30.001), False),
    (0.3, math.radians(-29.5), True),
])
def test_accuracy_criterion(dx, dth, ok):
    truth = (3.0, -2.0, 0.4)
    pose = {"x": truth[0] + dx * 0.6, "y": truth[1] - dx * 0.8, "theta": truth[2] + dth}
    a = bench.accuracy(pose, truth, {"best_margin": 0.01, "ambiguous": 0})
    assert a["d_err_m"] == pytest.approx(dx, abs=1e-12)
    assert a["phi_err_deg"] == pytest.approx(abs(math.degrees(dth)), abs=1e-9)
    assert a["success"] is ok


def test_accuracy_heading_wraps():
    # 179 deg and -179 deg are 2 deg apart
    a = bench.accuracy({"x": 0.0, "y": 0.0, "theta": math.radians(179.0)},
                       (0.0, 0.0, math.radians(-179.0)), {"best_margin": -1.0, "ambiguous": 1})
    assert a["phi_err_deg"] == pytest.approx(2.0, abs=1e-9)
    assert a["success"] is True
    assert a["best_margin"] == -1.0 and a["ambiguous"] == 1


def test_traffic_summary_is_current():
    path = os.path.join(ROOT, bench.TRAFFIC_FILE)
    kv = {}
    for line in open(path):
        if ":" in line and not line.startswith("#"):
            k, v = line.split(":", 1)
            kv[k.strip()] = v.strip()
    got = bench.measured_traffic()
    assert got is not None, "ray-cast sources changed since the traffic counters were taken"
    assert got == float(kv["bytes_per_launch"])
    # scaled fetch + write add up to the reported total
    assert abs(float(kv["fetch_bytes_per_launch"]) + float(kv["write_bytes_per_launch"])
               - got) <= 2.0


def test_counter_summary_is_current():
    """The executed-instruction summary the roofline divides by its live
    launch time belongs to the committed ray-cast sources, its per-launch
    figures are the medians of its per-dispatch rows, and the executed VALU
    fraction it records is at most 1."""
    import statistics
    cnt = bench.measured_counters()
    assert cnt is not None, "ray-cast sources changed since the counters were taken"
    kv = {}
    for line in open(os.path.join(ROOT, bench.COUNTERS_FILE)):
        if ":" in line and not line.startswith("#"):
            k, v = line.split(":", 1)
            kv[k.strip()] = v.strip()
    per = [float(x) for x in kv["valu_insts_per_dispatch"].split(",")]
    assert cnt["valu_insts_per_launch"] == statistics.median(per)
    assert 0.0 < float(kv["executed_valu_frac_of_measured_peak"]) <= 1.0
