"""Continuous-batching reconstruction server on one GPU.

Requests (geometry, projections Y, solver settings) arrive at any time.
The scheduler admits them in arrival order while their device footprint
(cbct_fbs_footprint: Y, f and all solver scratch) fits the HBM budget and
an execution slot is free, keeps every admitted request's iterate resident
on the device, and advances all admitted requests a few outer iterations
per tick, each on its own HIP stream, so the kernels of different requests
overlap on the GPU.  A request leaves when its last iteration has run on
the device; its slot and memory are then reused by the next arrival.

The scheduler (this module's Server) is host logic only; the device work
sits behind an executor with five calls (footprint, begin, step, poll,
finish).  GpuExecutor drives libcbct through the step API
(cbct_fbs_init / cbct_fbs_step / cbct_fbs_free); tests substitute a fake
executor to check admission, ordering, cancellation and error isolation
without a GPU.
"""

from __future__ import annotations

import collections
import dataclasses
import itertools
import threading
import time
from concurrent.futures import Future
from typing import Any, Callable, Dict, List, Optional

__all__ = ["Request", "Result", "Server", "GpuExecutor"]


@dataclasses.dataclass(eq=False)
class Request:
    """One reconstruction: geometry (any object with the Geometry fields),
    projections Y ([n_views][nv][nu], numpy or torch), solver settings."""
    geom: Any
    Y: Any
    params: Any
    id: Optional[int] = None
    arrival: Optional[float] = None


@dataclasses.dataclass
class Result:
    id: int
    f: Any                  # reconstructed volume (device tensor)
    report: Any             # FbsReport
    arrival: float
    admitted: float
    finished: float

    @property
    def latency(self) -> float:
        return self.finished - self.arrival


@dataclasses.dataclass(eq=False)  # slots compare by identity (fields hold arrays)
class _Slot:
    req: Request
    fut: Future
    handle: Any
    footprint: int
    admitted: float


class Server:
    """Admission by footprint, stepping by least remaining work, completion
    polling.

    hbm_budget: device bytes the admitted requests may hold together.
    max_active: execution slots (requests advanced concurrently); the
    default 4 matches the hardware queues a process gets, so each active
    request's stream has a queue of its own.
    iters_per_tick: outer iterations enqueued per request per tick.
    Each tick offers work to the active requests in order of the work they
    have left (executor.remaining, ties by admission), so a small request
    admitted behind large ones has its kernels queued first.
    Call start() for a background scheduler thread, or tick() yourself.
    """

    def __init__(self, executor, hbm_budget: int, max_active: int = 4,
                 iters_per_tick: int = 1, clock: Callable[[], float] = time.perf_counter):
        if hbm_budget <= 0 or max_active <= 0 or iters_per_tick <= 0:
            raise ValueError("budget, slots and iterations per tick must be positive")
        self.ex = executor
        self.budget = int(hbm_budget)
        self.max_active = int(max_active)
        self.iters_per_tick = int(iters_per_tick)
        self.clock = clock
        self._pending: collections.deque = collections.deque()
        self._active: List[_Slot] = []
        self._used = 0
        self._ids = itertools.count()
        self._lock = threading.Lock()
        self._wake = threading.Event()
        self._stop = False
        self._thread: Optional[threading.Thread] = None
        self.peak_used = 0
        self.peak_active = 0
        self._broken: Optional[BaseException] = None

    # ---------------------------------------------------------------- API --
    def submit(self, req: Request) -> Future:
        fut: Future = Future()
        if self._broken is not None:
            fut.set_exception(RuntimeError("server loop failed: %r" % (self._broken,)))
            return fut
        fp = int(self.ex.footprint(req))
        if fp <= 0 or fp > self.budget:
            fut.set_exception(ValueError(
                "request footprint %d bytes exceeds the HBM budget %d" % (fp, self.budget)))
            return fut
        with self._lock:
            req.id = next(self._ids) if req.id is None else req.id
            req.arrival = self.clock() if req.arrival is None else req.arrival
            self._pending.append((req, fut, fp))
        self._wake.set()
        return fut

    @property
    def used_bytes(self) -> int:
        return self._used

    def idle(self) -> bool:
        with self._lock:
            return not self._pending and not self._active

    def tick(self) -> bool:
        """One scheduling round; returns True if it did any work."""
        worked = self._admit()
        rem = getattr(self.ex, "remaining", None)
        order = list(self._active)
        if rem is not None:
            order.sort(key=lambda s: rem(s.handle))  # stable: ties keep admission order
        for s in order:
            try:
                if not self.ex.finished(s.handle):
                    worked |= bool(self.ex.step(s.handle, self.iters_per_tick))
                if self.ex.poll(s.handle):
                    f, rep = self.ex.finish(s.handle)
                    self._retire(s)
                    s.fut.set_result(Result(s.req.id, f, rep, s.req.arrival, s.admitted,
                                            self.clock()))
                    worked = True
            except Exception as e:  # isolate the failure to its request
                self._retire(s)
                try:
                    self.ex.abort(s.handle)
                finally:
                    s.fut.set_exception(e)
                worked = True
        return worked

    def run_until_idle(self, timeout: float = 3600.0, poll: float = 5e-4):
        end = self.clock() + timeout
        while not self.idle():
            if self.clock() > end:
                raise TimeoutError("server did not drain")
            if not self.tick():
                time.sleep(poll)

    def start(self, poll: float = 5e-4):
        def loop():
            try:
                while not self._stop:
                    if not self.tick():
                        self._wake.wait(poll)
                        self._wake.clear()
            except BaseException as e:  # a scheduler fault: no caller waits forever
                self._fail_all(e)
                raise
        self._stop = False
        self._thread = threading.Thread(target=loop, name="cbct-serve", daemon=True)
        self._thread.start()

    def stop(self):
        self._stop = True
        self._wake.set()
        if self._thread is not None:
            self._thread.join()
            self._thread = None

    # ----------------------------------------------------------- internals --
    def _fail_all(self, e: BaseException):
        """Fail every pending and active request with e; stop accepting."""
        with self._lock:
            self._broken = e
            pending, self._pending = list(self._pending), type(self._pending)()
            active, self._active = list(self._active), []
        for _, fut, _ in pending:
            if not fut.done():
                fut.set_exception(RuntimeError("server loop failed: %r" % (e,)))
        for s in active:
            try:
                self.ex.abort(s.handle)
            except Exception:
                pass
            if not s.fut.done():
                s.fut.set_exception(RuntimeError("server loop failed: %r" % (e,)))
        self._used = 0

    def _admit(self) -> bool:
        worked = False
        while True:
            with self._lock:
                while self._pending and self._pending[0][1].cancelled():
                    self._pending.popleft()
                if not self._pending or len(self._active) >= self.max_active:
                    return worked
                req, fut, fp = self._pending[0]
                if self._used + fp > self.budget:
                    return worked  # strict arrival order: wait for memory
                self._pending.popleft()
            if not fut.set_running_or_notify_cancel():
                continue
            try:
                handle = self.ex.begin(req)
            except Exception as e:
                fut.set_exception(e)
                worked = True
                continue
            self._active.append(_Slot(req, fut, handle, fp, self.clock()))
            self._used += fp
            self.peak_used = max(self.peak_used, self._used)
            self.peak_active = max(self.peak_active, len(self._active))
            worked = True

    def _retire(self, s: _Slot):
        for i, a in enumerate(self._active):
            if a is s:
                del self._active[i]
                self._used -= s.footprint
                break


class GpuExecutor:
    """Runs requests with libcbct's step API, one HIP stream per request.

    Plans are cached per geometry (their lambda estimates too).  At most
    `lookahead` steps of a request are in flight on its stream, so the host
    does not run arbitrarily far ahead of the device.
    """

    def __init__(self, device=0, lookahead: int = 2):
        import torch
        import paper_1002_3675_amd as cb
        self.torch = torch
        self.cb = cb
        self.device = torch.device("cuda", device)
        self.lookahead = lookahead
        self._plans: Dict[Any, Any] = {}

    def plan_for(self, geom):
        g = self.cb.Geometry.of(geom)
        p = self._plans.get(g)
        if p is None:
            with self.torch.cuda.device(self.device):
                p = self.cb.Plan(g, device=self.device)
            self._plans[g] = p
        return p

    def footprint(self, req) -> int:
        return self.cb.footprint(self.cb.Geometry.of(req.geom), req.params)

    def begin(self, req):
        torch = self.torch
        plan = self.plan_for(req.geom)
        stream = torch.cuda.Stream(device=self.device)
        # inputs produced on the submitter's stream are ready before use
        stream.wait_stream(torch.cuda.current_stream(self.device))
        with torch.cuda.device(self.device), torch.cuda.stream(stream):
            Y = torch.as_tensor(req.Y, dtype=torch.float32).to(self.device, non_blocking=True)
            Y = Y.contiguous()
            f = torch.zeros(plan.geom.vol_shape, dtype=torch.float32, device=self.device)
        st = self.cb.FbsState(plan, Y, f, req.params, stream=stream)
        g = plan.geom
        nvox = float(g.nx * g.ny * g.nz)
        iters = list(req.params.iters)
        # level l (coarse first) has about 8^-(levels - 1 - l) of the voxels
        per_iter = [nvox / 8.0 ** (len(iters) - 1 - l) for l in range(len(iters))]
        return {"st": st, "stream": stream, "Y": Y, "f": f, "events": collections.deque(),
                "done_event": None, "sched": [it for it in iters], "per_iter": per_iter,
                "work_left": sum(n * w for n, w in zip(iters, per_iter))}

    def finished(self, h) -> bool:
        return h["st"].finished

    def remaining(self, h) -> float:
        """Work left, in fine-level iteration equivalents: iterations not yet
        enqueued, a level's weighted by its voxel count over the finest's,
        times the finest level's voxel count (so requests compare)."""
        return h["work_left"]

    def step(self, h, n) -> bool:
        ev = h["events"]
        while ev and ev[0].query():
            ev.popleft()
        if len(ev) >= self.lookahead:
            return False
        with self.torch.cuda.device(self.device):
            h["st"].step(n)
            e = self.torch.cuda.Event()
            e.record(h["stream"])
        ev.append(e)
        # the schedule as enqueued so far (a tolerance stop may end a level
        # earlier; the figure only orders the requests)
        left = n
        for l, it in enumerate(h["sched"]):
            take = min(it, left)
            h["sched"][l] -= take
            left -= take
        h["work_left"] = sum(i * w for i, w in zip(h["sched"], h["per_iter"]))
        if h["st"].finished:
            h["done_event"] = e
        return True

    def poll(self, h) -> bool:
        return h["done_event"] is not None and h["done_event"].query()

    def finish(self, h):
        rep = h["st"].report()
        h["st"].close()
        f = h["f"]
        h.clear()
        return f, rep

    def abort(self, h):
        st = h.get("st")
        if st is not None:
            h["stream"].synchronize()
            st.close()
        h.clear()
