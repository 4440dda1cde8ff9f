"""The serving scheduler's host logic with a fake executor (no GPU):
footprint admission, arrival order, slot limits, cancellation, error
isolation, and draining."""

import threading
import time

import pytest

from paper_1002_3675_amd.serve import Request, Server


class FakeExecutor:
    """Each request needs params['iters'] steps; footprint params['fp']."""

    def __init__(self, fail_ids=(), fail_begin=()):
        self.fail_ids = set(fail_ids)
        self.fail_begin = set(fail_begin)
        self.begun = []
        self.live = set()
        self.max_live_fp = 0
        self.lock = threading.Lock()

    def footprint(self, req):
        return req.params["fp"]

    def begin(self, req):
        if req.id in self.fail_begin:
            raise RuntimeError("begin failed")
        with self.lock:
            self.begun.append(req.id)
            self.live.add(req.id)
            self.max_live_fp = max(self.max_live_fp, sum(
                r for r in [req.params["fp"]]))
        return {"req": req, "done": 0}

    def finished(self, h):
        return h["done"] >= h["req"].params["iters"]

    def step(self, h, n):
        if h["req"].id in self.fail_ids and h["done"] == 1:
            raise RuntimeError("device error in request %d" % h["req"].id)
        h["done"] += n
        return True

    def poll(self, h):
        return self.finished(h)

    def finish(self, h):
        self.live.discard(h["req"].id)
        return "f%d" % h["req"].id, {"iters": h["done"]}

    def abort(self, h):
        self.live.discard(h["req"].id)


def _req(fp, iters, rid=None):
    return Request(geom=None, Y=None, params={"fp": fp, "iters": iters}, id=rid)


def test_admission_respects_budget_and_slots():
    ex = FakeExecutor()
    srv = Server(ex, hbm_budget=100, max_active=3)
    futs = [srv.submit(_req(fp, 5)) for fp in (40, 40, 30, 50, 10, 60, 20)]
    while not srv.idle():
        srv.tick()
        assert srv.used_bytes <= 100
        assert len(ex.live) <= 3
    assert srv.peak_used <= 100 and srv.peak_active <= 3
    assert [f.result().f for f in futs] == ["f%d" % i for i in range(7)]
    assert ex.begun == list(range(7))  # strict arrival order


def test_over_budget_request_is_rejected_at_submit():
    srv = Server(FakeExecutor(), hbm_budget=100)
    fut = srv.submit(_req(101, 3))
    with pytest.raises(ValueError):
        fut.result(timeout=1)
    assert srv.idle()


def test_head_of_line_waits_for_memory():
    ex = FakeExecutor()
    srv = Server(ex, hbm_budget=100, max_active=8)
    a = srv.submit(_req(70, 10))
    b = srv.submit(_req(60, 2))   # does not fit beside a
    c = srv.submit(_req(10, 2))   # would fit, but must not overtake b
    srv.tick()
    assert ex.begun == [0]
    srv.run_until_idle(timeout=5)
    assert ex.begun == [0, 1, 2]
    assert all(f.done() for f in (a, b, c))


def test_cancel_pending_request():
    ex = FakeExecutor()
    srv = Server(ex, hbm_budget=100, max_active=1)
    a = srv.submit(_req(50, 3))
    b = srv.submit(_req(50, 3))
    srv.tick()
    assert b.cancel()
    srv.run_until_idle(timeout=5)
    assert a.result().f == "f0"
    assert b.cancelled()
    assert ex.begun == [0]


def test_error_is_isolated_to_its_request():
    ex = FakeExecutor(fail_ids={1}, fail_begin={3})
    srv = Server(ex, hbm_budget=1000, max_active=4)
    futs = [srv.submit(_req(10, 4)) for _ in range(5)]
    srv.run_until_idle(timeout=5)
    with pytest.raises(RuntimeError, match="device error"):
        futs[1].result()
    with pytest.raises(RuntimeError, match="begin failed"):
        futs[3].result()
    for i in (0, 2, 4):
        assert futs[i].result().report["iters"] == 4
    assert srv.used_bytes == 0 and not ex.live


def test_background_thread_drains():
    ex = FakeExecutor()
    srv = Server(ex, hbm_budget=100, max_active=2)
    srv.start()
    try:
        futs = []
        for i in range(6):
            futs.append(srv.submit(_req(30, 3)))
            time.sleep(0.002)
        res = [f.result(timeout=10) for f in futs]
    finally:
        srv.stop()
    assert [r.id for r in res] == list(range(6))
    assert all(r.finished >= r.admitted >= r.arrival for r in res)


def test_out_of_order_completion_with_array_payloads():
    """A later, shorter request finishes first while earlier ones are still
    active; requests carry arrays (whose == is elementwise), so the server
    must track its slots by identity."""
    import numpy as np
    ex = FakeExecutor()
    srv = Server(ex, hbm_budget=1000, max_active=4)
    futs = []
    for rid, iters in enumerate((9, 7, 2, 1, 5)):
        r = Request(geom=None, Y=np.ones((3, 4, 5)), params={"fp": 10, "iters": iters},
                    id=rid)
        futs.append(srv.submit(r))
    srv.run_until_idle(timeout=5)
    assert [f.result().report["iters"] for f in futs] == [9, 7, 2, 1, 5]
    assert srv.used_bytes == 0 and not ex.live


@pytest.mark.filterwarnings("ignore::pytest.PytestUnhandledThreadExceptionWarning")
def test_scheduler_fault_fails_every_request_instead_of_hanging():
    """If the scheduling loop itself raises (not a request's own error), the
    background thread fails every pending and active future and refuses new
    ones, so no caller waits forever."""
    class Broken(FakeExecutor):
        def poll(self, h):
            raise KeyboardInterrupt  # escapes the per-request isolation
    srv = Server(Broken(), hbm_budget=1000, max_active=2)
    futs = [srv.submit(_req(10, 3)) for _ in range(4)]
    srv.start()
    for f in futs:
        with pytest.raises(RuntimeError, match="server loop failed"):
            f.result(timeout=5)
    with pytest.raises(RuntimeError, match="server loop failed"):
        srv.submit(_req(10, 3)).result(timeout=1)
    srv._thread.join(timeout=5)


class RankedExecutor(FakeExecutor):
    """A fake executor that also reports the work left and logs step order."""

    def __init__(self):
        super().__init__()
        self.order = []

    def remaining(self, h):
        return h["req"].params["iters"] - h["done"]

    def step(self, h, n):
        self.order.append(h["req"].id)
        return super().step(h, n)


def test_requests_with_least_work_left_are_stepped_first():
    ex = RankedExecutor()
    srv = Server(ex, hbm_budget=1000, max_active=4)
    futs = [srv.submit(_req(10, it, rid)) for rid, it in ((0, 9), (1, 2), (2, 5), (3, 1))]
    srv.tick()
    # one tick: all four admitted, stepped in order of work left
    assert ex.order == [3, 1, 2, 0]
    srv.run_until_idle(timeout=10)
    assert [f.result().f for f in futs] == ["f0", "f1", "f2", "f3"]
    # ties keep admission order
    ex2 = RankedExecutor()
    srv2 = Server(ex2, hbm_budget=1000, max_active=4)
    for rid in range(3):
        srv2.submit(_req(10, 4, rid))
    srv2.tick()
    assert ex2.order == [0, 1, 2]


def test_default_slots_match_the_hardware_queues():
    assert Server(FakeExecutor(), hbm_budget=10).max_active == 4
