"""GPU parity of the paper's Eq. (2) gradient (voxel-driven, bilinear
residual lookup, on the transpose's scale) and of the solver's Eq. (2)
mode against the FP64 oracle."""

import sys

import numpy as np
import pytest

import oracle
from workloads import Geometry, tiny_case, tiny_geometry, diff_geometry

from gpu_util import require_gpu, rel_l2, to_dev, to_np

pytestmark = pytest.mark.gpu

RAGGED = Geometry(70, 45, 33, 2.1, 2.3, 2.7, 97, 61, 2.4, 2.2, 700.0, 1100.0, 7,
                  angles=(0.05, 0.9, 1.7, 2.6, 3.3, 4.4, 5.9))


def _log(msg):
    print(msg, flush=True)
    sys.stdout.flush()


@pytest.mark.parametrize("name,g", [("tiny", tiny_geometry()), ("ragged", RAGGED),
                                    ("diff", diff_geometry())])
def test_eq2_operator_matches_oracle(name, g):
    require_gpu()
    import paper_1002_3675_amd as cb
    _log("eq2 parity %s" % name)
    rng = np.random.default_rng(30)
    y = rng.uniform(-1.0, 4.0, g.proj_shape)
    p = cb.Plan(g)
    got = to_np(p.backproject_eq2(to_dev(y)))
    want = oracle.eq2_backproject(g, y.astype(np.float32).astype(np.float64))
    assert rel_l2(got, want) <= 1e-5, rel_l2(got, want)
    # bitwise repeatable
    again = to_np(p.backproject_eq2(to_dev(y)))
    assert np.array_equal(got, again)


def test_eq2_approximates_the_transpose():
    """For a smooth residual Eq. (2) is P^T to first order in the pitch."""
    require_gpu()
    import paper_1002_3675_amd as cb
    g = tiny_geometry()
    u = (np.arange(g.nu) - 0.5 * (g.nu - 1)) * g.au
    v = (np.arange(g.nv) - 0.5 * (g.nv - 1)) * g.av
    U, V = np.meshgrid(u, v)
    y = np.stack([np.exp(-(U ** 2 + (V - 0.1 * k) ** 2) / (2 * 40.0 ** 2))
                  for k in range(g.n_views)])
    p = cb.Plan(g)
    a = to_np(p.backproject(to_dev(y)))
    b = to_np(p.backproject_eq2(to_dev(y)))
    sl = (slice(8, 56),) * 3
    assert rel_l2(b[sl], a[sl]) < 0.03, rel_l2(b[sl], a[sl])


def test_fbs_eq2_mode_matches_oracle():
    """64^3 stand-in phantom, 16 views, 10 iterations with the Eq. (2)
    gradient; beta and the inner count from the oracle's rule."""
    require_gpu()
    import paper_1002_3675_amd as cb
    import torch
    case = tiny_case()
    g = case.geom
    lam = oracle.power_lambda(g, 30)
    beta = oracle.beta_rule(g, case.mu, lam)
    k = oracle.default_inner(np.array([g.hx, g.hy, g.hz]), beta, case.eps)
    want = oracle.fbs_solve(g, case.Y, case.mu, (10,), beta=(beta,), n_inner=(k,),
                            eps=case.eps, gradient="eq2")
    f, rep = cb.fbs_solve(cb.Plan(g), torch.as_tensor(case.Y, dtype=torch.float32,
                                                      device="cuda"),
                          cb.FbsParams(mu=case.mu, iters=(10,), beta=(beta,), n_inner=(k,),
                                       eps=case.eps, trace_energy=True, gradient="eq2"))
    err = rel_l2(to_np(f), want["f"])
    assert err <= 1e-3, err
    E = want["report"][0]
    assert abs(rep.E - E) <= 1e-4 * abs(E), (rep.E, E)
    assert float(f.min()) >= 0.0


def test_eq2_head_size_two_views():
    """Full 512x512x70 Eq. (2) operator on the 40-view head geometry with
    data on two views (the others zero), against the oracle on those two."""
    require_gpu()
    import dataclasses
    import math
    import paper_1002_3675_amd as cb
    from workloads import head_geometry
    _log("eq2 head size")
    g = head_geometry(40)
    rng = np.random.default_rng(33)
    y = np.zeros(g.proj_shape, dtype=np.float32)
    ks = (3, 22)
    for k in ks:
        y[k] = rng.uniform(-1.0, 4.0, (g.nv, g.nu))
    got = to_np(cb.Plan(g).backproject_eq2(to_dev(y)))
    gk = dataclasses.replace(g, n_views=2, angles=tuple(2 * math.pi * k / 40 for k in ks))
    want = oracle.eq2_backproject(gk, y[list(ks)].astype(np.float64))
    assert rel_l2(got, want) <= 1e-5, rel_l2(got, want)
