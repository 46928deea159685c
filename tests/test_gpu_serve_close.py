"""Closing a serving context while another thread waits in reloc_poll.

The waiting poll has to end before the serving state is freed: it returns
the finished result, or RELOC_E_PENDING (None from the binding) for a
request that was still in flight, and the process stays up. Sixteen
plain-large requests without early termination (every stage, tens of
milliseconds each on the device) keep the polled request in flight well
past the moment the context is closed.
"""
import sys
import threading
import time

import pytest

import paper_2511_01219_amd as reloc
from synth import make_config

pytestmark = pytest.mark.gpu


def _case(msg):
    print("[gpu case] " + msg, flush=True)
    sys.stdout.flush()


def test_close_ends_a_blocked_poll():
    w = make_config(2)
    ctx = reloc.Context(0)
    closed = False
    try:
        m = ctx.load_map(w.occ, w.resolution, w.origin)
        s = w.sample
        sid, _ = ctx.sample_hypotheses(m, s["n_target"], s["min_spacing"], s["robot_radius"],
                                       seed=s["seed"])
        scan = dict(ranges=w.ranges, angle_min=w.angle_min, angle_increment=w.angle_increment,
                    range_min=w.range_min, range_max=w.range_max)
        kw = dict(w.search, tau=None)
        _case("serve close: 16 plain-large requests without early termination")
        tickets = [ctx.submit(m, sid, **scan, **kw) for _ in range(16)]
        got = {}

        def waiter():
            try:
                got["r"] = ctx.poll(tickets[-1], wait_ms=-1)
            except Exception as e:   # reported below
                got["e"] = e

        th = threading.Thread(target=waiter)
        th.start()
        # the waiter is counted inside reloc_poll (under the serving lock)
        # before it waits; close only once it is there
        t_end = time.monotonic() + 30.0
        while ctx.serve_stats()["pollers"] < 1:
            assert time.monotonic() < t_end, "the poll never entered the library"
            assert th.is_alive() or "r" in got or "e" in got
            if not th.is_alive():
                break
            time.sleep(0.001)
        _case("serve close: closing the context while a poll waits")
        ctx.close()
        closed = True
        th.join(timeout=60)
        assert not th.is_alive(), "the waiting poll did not return"
        assert "e" not in got, repr(got.get("e"))
        r = got["r"]
        assert r is None or r[1]["status"] == reloc.OK
    finally:
        if not closed:
            ctx.close()
