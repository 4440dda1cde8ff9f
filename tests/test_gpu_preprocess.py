"""GPU parity of the device log transform of detector counts, and a
short-scan (200 degree) solve, against the oracle."""

import math

import numpy as np
import pytest

import oracle
from workloads import Geometry, tiny_geometry, analytic_projections, shepp_logan_standin, \
    noisy_log_projections

from gpu_util import require_gpu, rel_l2, to_dev, to_np

pytestmark = pytest.mark.gpu


def test_log_counts_matches_oracle():
    torch = require_gpu()
    import paper_1002_3675_amd as cb
    rng = np.random.default_rng(40)
    p = rng.uniform(0.0, 6.0, (5, 33, 47))
    counts = rng.poisson(5e4 * np.exp(-p)).astype(np.float64)
    counts.flat[:20] = [0.0, -2.0, 0.3] * 6 + [1.0, 5e4]   # floor and open beam
    flat = rng.uniform(4e4, 6e4, counts.shape)
    c32 = counts.astype(np.float32).astype(np.float64)
    f32 = flat.astype(np.float32).astype(np.float64)
    for kw, want in (({"i0": 5e4}, oracle.log_counts(c32, i0=5e4)),
                     ({"flat": to_dev(flat)}, oracle.log_counts(c32, flat=f32))):
        got = to_np(cb.log_counts(to_dev(counts), **kw))
        assert np.max(np.abs(got - want)) <= 1e-6, np.max(np.abs(got - want))
    # in place
    t = to_dev(counts)
    cb.log_counts(t, i0=5e4, out=t)
    assert np.max(np.abs(to_np(t) - oracle.log_counts(c32, i0=5e4))) <= 1e-6
    with pytest.raises(cb.CbctError):
        cb.log_counts(to_dev(counts), i0=-1.0)


def test_short_scan_solve_matches_oracle():
    """24 views over 200 degrees (a short scan), 64^3 stand-in, 5 iterations
    with beta and the inner count from the oracle's rule."""
    torch = require_gpu()
    import paper_1002_3675_amd as cb
    ang = tuple(math.radians(200.0) * k / 23 for k in range(24))
    g = Geometry(64, 64, 64, 2.0, 2.0, 2.0, 128, 96, 1.6, 1.6, 500.0, 750.0, 24, angles=ang)
    Y = noisy_log_projections(analytic_projections(g, shepp_logan_standin(1000)), 1e5, 2100)
    beta = oracle.beta_rule(g, 1e-3, oracle.power_lambda(g, 30))
    k = oracle.default_inner(np.array([g.hx, g.hy, g.hz]), beta, 1e-3)
    want = oracle.fbs_solve(g, Y, 1e-3, (5,), beta=(beta,), n_inner=(k,))
    f, rep = cb.fbs_solve(cb.Plan(g), to_dev(Y),
                          cb.FbsParams(mu=1e-3, iters=(5,), beta=(beta,), n_inner=(k,),
                                       trace_energy=True))
    assert rel_l2(to_np(f), want["f"]) <= 1e-3
    assert abs(rep.E - want["report"][0]) <= 1e-4 * abs(want["report"][0])
