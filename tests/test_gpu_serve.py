"""Continuous batching on the GPU: requests of mixed sizes and view counts
run concurrently on separate streams and each result equals the same
request solved alone (bitwise: every kernel is deterministic and the
streams share no buffers)."""

import numpy as np
import pytest

from workloads import Geometry, analytic_projections, noisy_log_projections, \
    random_ellipsoid_object

from gpu_util import require_gpu

pytestmark = pytest.mark.gpu

CLASSES = [
    Geometry(32, 32, 24, 4.0, 4.0, 5.0, 64, 48, 3.2, 3.2, 1000.0, 1500.0, 10),
    Geometry(48, 48, 32, 3.0, 3.0, 4.0, 80, 60, 3.0, 3.0, 1000.0, 1500.0, 10),
    Geometry(64, 64, 40, 2.4, 2.4, 3.5, 96, 72, 2.6, 2.6, 1000.0, 1500.0, 10),
]


def _requests(n, seed=50):
    import paper_1002_3675_amd as cb
    from paper_1002_3675_amd.serve import Request
    rng = np.random.default_rng(seed)
    out = []
    for k in range(n):
        g = CLASSES[k % 3].with_views(int(rng.choice([8, 12, 16])))
        ph = random_ellipsoid_object(g, 100 + k, n_inner=(3, 6))
        Y = noisy_log_projections(analytic_projections(g, ph), 5e4, 200 + k).astype(np.float32)
        out.append(Request(g, Y, cb.FbsParams(mu=1e-3, iters=(3, 3))))
    return out


def test_mixed_stream_equals_alone():
    torch = require_gpu()
    import paper_1002_3675_amd as cb
    from paper_1002_3675_amd.serve import GpuExecutor, Server
    reqs = _requests(9)
    ex = GpuExecutor(0)
    alone = []
    for r in reqs:
        f, _ = cb.fbs_solve(ex.plan_for(r.geom), torch.as_tensor(r.Y, device="cuda"), r.params)
        alone.append(f)
    torch.cuda.synchronize()
    srv = Server(ex, hbm_budget=8 << 30, max_active=4, iters_per_tick=1)
    futs = [srv.submit(r) for r in reqs]
    srv.run_until_idle(timeout=300)
    assert srv.peak_active >= 2  # requests really overlapped
    for fut, want in zip(futs, alone):
        res = fut.result()
        torch.cuda.synchronize()
        assert torch.equal(res.f, want), res.id
        assert res.report.iters_done == 6


def test_budget_forces_queueing():
    torch = require_gpu()
    import paper_1002_3675_amd as cb
    from paper_1002_3675_amd.serve import GpuExecutor, Server
    reqs = _requests(4, seed=51)
    ex = GpuExecutor(0)
    fps = [ex.footprint(r) for r in reqs]
    srv = Server(ex, hbm_budget=max(fps) + min(fps) - 1, max_active=4)
    futs = [srv.submit(r) for r in reqs]
    srv.run_until_idle(timeout=300)
    assert srv.peak_used <= srv.budget
    assert srv.peak_active <= 2
    assert all(f.result().report.iters_done == 6 for f in futs)


def test_mixed_schedules_equal_alone():
    """Requests with three levels, a tolerance stop or the Eq. (2) gradient
    share the GPU with plain ones; each result and its per-level iteration
    counts equal the same request solved alone."""
    torch = require_gpu()
    import dataclasses
    import paper_1002_3675_amd as cb
    from paper_1002_3675_amd.serve import GpuExecutor, Server
    reqs = _requests(8, seed=52)
    variants = [dict(iters=(2, 2, 3)), dict(iters=(10, 10), tol=2e-2),
                dict(gradient="eq2"), dict()]
    for k, r in enumerate(reqs):
        r.params = dataclasses.replace(r.params, **variants[k % 4])
    ex = GpuExecutor(0)
    alone = []
    for r in reqs:
        alone.append(cb.fbs_solve(ex.plan_for(r.geom), torch.as_tensor(r.Y, device="cuda"),
                                  r.params))
    torch.cuda.synchronize()
    srv = Server(ex, hbm_budget=8 << 30, max_active=4, iters_per_tick=1)
    futs = [srv.submit(r) for r in reqs]
    srv.run_until_idle(timeout=300)
    assert srv.peak_active >= 2
    for fut, (want_f, want_rep) in zip(futs, alone):
        res = fut.result()
        torch.cuda.synchronize()
        assert torch.equal(res.f, want_f), res.id
        assert res.report.level_iters == want_rep.level_iters, res.id
