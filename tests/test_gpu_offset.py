"""GPU parity on a shifted detector (half-fan: the detector moved sideways
so that it sees a little more than half of the field in each view, over a
full turn) and on a shifted volume (a region of interest off the axis)
against the FP64 oracle: P, P^T, the Eq. (2) gradient and a short solve."""

import math
import sys

import numpy as np
import pytest

import oracle
from workloads import Geometry, analytic_projections, shepp_logan_standin, \
    noisy_log_projections

from gpu_util import require_gpu, rel_l2, to_dev, to_np

pytestmark = pytest.mark.gpu

HALF_FAN = Geometry(64, 64, 48, 2.0, 2.0, 2.0, 80, 72, 1.6, 1.6, 500.0, 750.0, 30,
                    u_off=0.4 * 80 * 1.6, v_off=-1.3,
                    angles=tuple(2.0 * math.pi * k / 30 for k in range(30)))


def _log(msg):
    print(msg, flush=True)
    sys.stdout.flush()


def test_half_fan_operators_match_oracle():
    require_gpu()
    import paper_1002_3675_amd as cb
    g = HALF_FAN
    _log("half-fan operators")
    rng = np.random.default_rng(60)
    f = rng.uniform(0.0, 0.02, g.vol_shape).astype(np.float32).astype(np.float64)
    y = rng.uniform(-1.0, 4.0, g.proj_shape).astype(np.float32).astype(np.float64)
    p = cb.Plan(g)
    got_p = to_np(p.project(to_dev(f)))
    assert rel_l2(got_p, oracle.project(g, f)) <= 1e-5
    got_t = to_np(p.backproject(to_dev(y)))
    assert rel_l2(got_t, oracle.backproject(g, y)) <= 1e-5
    got_e = to_np(p.backproject_eq2(to_dev(y)))
    assert rel_l2(got_e, oracle.eq2_backproject(g, y)) <= 1e-5
    # the shift is seen: without it the projections differ at order one
    g0 = Geometry(64, 64, 48, 2.0, 2.0, 2.0, 80, 72, 1.6, 1.6, 500.0, 750.0, 30,
                  angles=g.angles)
    assert rel_l2(to_np(cb.Plan(g0).project(to_dev(f))), got_p) > 0.1


def test_half_fan_solve_matches_oracle():
    require_gpu()
    import paper_1002_3675_amd as cb
    g = HALF_FAN
    _log("half-fan solve")
    Y = noisy_log_projections(analytic_projections(g, shepp_logan_standin(1000)), 1e5, 2600)
    beta = oracle.beta_rule(g, 1e-3, oracle.power_lambda(g, 30))
    k = oracle.default_inner(np.array([g.hx, g.hy, g.hz]), beta, 1e-3)
    want = oracle.fbs_solve(g, Y, 1e-3, (5,), beta=(beta,), n_inner=(k,))
    f, rep = cb.fbs_solve(cb.Plan(g), to_dev(Y),
                          cb.FbsParams(mu=1e-3, iters=(5,), beta=(beta,), n_inner=(k,),
                                       trace_energy=True))
    assert rel_l2(to_np(f), want["f"]) <= 1e-3
    assert abs(rep.E - want["report"][0]) <= 1e-4 * abs(want["report"][0])


def test_shifted_volume_operators_match_oracle():
    require_gpu()
    import paper_1002_3675_amd as cb
    g = Geometry(48, 40, 36, 1.5, 1.5, 1.75, 96, 80, 1.6, 1.6, 500.0, 750.0, 9,
                 x_off=31.0, y_off=-17.5, z_off=12.3)
    _log("shifted volume operators")
    rng = np.random.default_rng(61)
    f = rng.uniform(0.0, 0.02, g.vol_shape).astype(np.float32).astype(np.float64)
    y = rng.uniform(-1.0, 4.0, g.proj_shape).astype(np.float32).astype(np.float64)
    p = cb.Plan(g)
    assert abs(p.samples - oracle.count_samples(g)) <= 1e-6 * p.samples
    assert rel_l2(to_np(p.project(to_dev(f))), oracle.project(g, f)) <= 1e-5
    assert rel_l2(to_np(p.backproject(to_dev(y))), oracle.backproject(g, y)) <= 1e-5
    assert rel_l2(to_np(p.backproject_eq2(to_dev(y))), oracle.eq2_backproject(g, y)) <= 1e-5


def test_float64_kernels_on_shifted_geometry():
    """The float64 kernels follow the oracle to 1e-12 with both the detector
    and the grid shifted (every shift enters the double ray arithmetic)."""
    require_gpu()
    import torch
    import paper_1002_3675_amd as cb
    g = Geometry(30, 26, 20, 2.0, 2.0, 2.5, 48, 40, 2.0, 2.0, 400.0, 650.0, 5,
                 u_off=17.0, v_off=-3.1, x_off=-11.0, y_off=6.5, z_off=4.25)
    _log("float64 shifted geometry")
    rng = np.random.default_rng(62)
    f = rng.uniform(0.0, 0.02, g.vol_shape)
    y = rng.uniform(-1.0, 4.0, g.proj_shape)
    p = cb.Plan(g)
    assert rel_l2(to_np(p.project(to_dev(f, torch.float64))), oracle.project(g, f)) <= 1e-12
    assert rel_l2(to_np(p.backproject(to_dev(y, torch.float64))),
                  oracle.backproject(g, y)) <= 1e-12
