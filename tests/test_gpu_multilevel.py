"""GPU parity of the deeper multigrid (three levels on odd sizes, so the
coarser grids sit half a finer spacing off the axis) and of the
relative-change stopping rule against the FP64 oracle."""

import sys

import numpy as np
import pytest

import oracle
from workloads import Geometry, analytic_projections, noisy_log_projections, \
    shepp_logan_standin

from gpu_util import require_gpu, rel_l2, to_dev, to_np

pytestmark = pytest.mark.gpu

ODD = Geometry(45, 41, 29, 2.0, 2.0, 2.25, 92, 69, 1.6, 1.6, 1000.0, 1500.0, 16)


def _log(msg):
    print(msg, flush=True)
    sys.stdout.flush()


def _data(g, seed):
    return noisy_log_projections(analytic_projections(g, shepp_logan_standin(1000)), 1e5, seed)


def test_three_levels_match_oracle():
    require_gpu()
    import paper_1002_3675_amd as cb
    _log("three-level solve, odd sizes")
    g, mu, iters = ODD, 1e-3, (3, 3, 3)
    Y = _data(g, 80).astype(np.float32).astype(np.float64)
    setup = oracle.fbs_solve(g, Y, mu, (0, 0, 0))
    beta, inner = tuple(setup["used_beta"]), tuple(int(k) for k in setup["used_inner"])
    want = oracle.fbs_solve(g, Y, mu, iters, beta=beta, n_inner=inner, trace=True)
    f, rep = cb.fbs_solve(cb.Plan(g), to_dev(Y),
                          cb.FbsParams(mu=mu, iters=iters, beta=beta, n_inner=inner,
                                       trace_energy=True))
    assert rel_l2(to_np(f), want["f"]) <= 1e-3, rel_l2(to_np(f), want["f"])
    assert rep.level_iters == (3, 3, 3) and rep.iters_done == 9
    tr = np.array(rep.trace)
    assert tr.shape == want["trace"].shape
    assert np.max(np.abs(tr[:, 0] - want["trace"][:, 0]) / want["trace"][:, 0]) <= 1e-4
    # the GPU's own beta estimate agrees with the oracle's on every level
    _, rep2 = cb.fbs_solve(cb.Plan(g), to_dev(Y), cb.FbsParams(mu=mu, iters=(0, 0, 0)))
    assert np.allclose(rep2.beta_used, beta, rtol=1e-4)


def _changes(g, Y, mu, beta, n):
    runs = [np.zeros(g.vol_shape)] + [oracle.fbs_solve(g, Y, mu, (k,), beta=beta)["f"]
                                      for k in range(1, n + 1)]
    return [np.linalg.norm(runs[k] - runs[k - 1]) / np.linalg.norm(runs[k])
            for k in range(1, n + 1)]


def test_tolerance_stop_matches_oracle():
    require_gpu()
    import paper_1002_3675_amd as cb
    _log("tolerance stop")
    g = Geometry(40, 40, 24, 2.5, 2.5, 2.5, 80, 48, 2.0, 2.0, 1000.0, 1500.0, 12)
    mu = 1e-3
    Y = _data(g, 81).astype(np.float32).astype(np.float64)
    beta = tuple(oracle.fbs_solve(g, Y, mu, (0,))["used_beta"])
    ch = _changes(g, Y, mu, beta, 7)
    stop = 4
    # a threshold well between the changes of iterations stop - 1 and stop,
    # so float32 rounding cannot move the decision
    assert ch[stop - 2] > 1.1 * ch[stop - 1], ch
    tol = float(np.sqrt(ch[stop - 2] * ch[stop - 1]))
    want = oracle.fbs_solve(g, Y, mu, (7,), beta=beta, tol=tol)
    assert want["used_iters"][0] == stop
    plan = cb.Plan(g)
    params = cb.FbsParams(mu=mu, iters=(7,), beta=beta, tol=tol)
    f, rep = cb.fbs_solve(plan, to_dev(Y), params)
    assert rep.level_iters == (stop,) and rep.iters_done == stop
    assert abs(rep.change[0] - ch[stop - 1]) <= 1e-3 * ch[stop - 1]
    assert rel_l2(to_np(f), want["f"]) <= 1e-3
    # the step API, one iteration at a time, stops at the same place
    fs = to_dev(np.zeros(g.vol_shape))
    st = cb.FbsState(plan, to_dev(Y), fs, params)
    n = 0
    while not st.finished:
        st.step(1)
        n += 1
    assert st.report().level_iters == (stop,)
    assert n == stop        # the call that meets the tolerance closes the level
    assert np.array_equal(to_np(fs), to_np(f))
    st.close()
    # two levels, a tolerance no iteration meets: the counts are maxima
    _, rep = cb.fbs_solve(plan, to_dev(Y), cb.FbsParams(mu=mu, iters=(2, 3), tol=1e-9))
    assert rep.level_iters == (2, 3)


def test_single_plane_coarse_level_matches_oracle():
    """Three planes coarsen to one (and 21 columns to 10, half a spacing off
    the axis): the coarse level is a single slab of cells."""
    require_gpu()
    import paper_1002_3675_amd as cb
    _log("single-plane coarse level")
    g = Geometry(21, 18, 3, 4.0, 4.0, 5.0, 40, 12, 3.2, 3.2, 1000.0, 1500.0, 8)
    mu = 1e-3
    Y = _data(g, 90).astype(np.float32).astype(np.float64)
    setup = oracle.fbs_solve(g, Y, mu, (0, 0))
    beta, inner = tuple(setup["used_beta"]), tuple(int(k) for k in setup["used_inner"])
    want = oracle.fbs_solve(g, Y, mu, (3, 3), beta=beta, n_inner=inner, trace=True)
    f, rep = cb.fbs_solve(cb.Plan(g), to_dev(Y),
                          cb.FbsParams(mu=mu, iters=(3, 3), beta=beta, n_inner=inner,
                                       trace_energy=True))
    assert rel_l2(to_np(f), want["f"]) <= 1e-3, rel_l2(to_np(f), want["f"])
    assert abs(rep.E - want["report"][0]) <= 1e-4 * abs(want["report"][0])
