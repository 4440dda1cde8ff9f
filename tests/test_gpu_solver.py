"""GPU parity of the TV sweep, the energies and the full FBS solve against
the FP64 oracle: volume within 1e-3 relative L2 and energy within 1e-4
relative after the fixed iteration counts, one and two levels."""

import dataclasses
import sys

import numpy as np
import pytest

import oracle
from workloads import Geometry, tiny_case, tiny_geometry, analytic_projections, \
    noisy_log_projections, random_ellipsoid_object

from gpu_util import require_gpu, rel_l2, to_dev, to_np

pytestmark = pytest.mark.gpu


def _log(msg):
    print(msg, flush=True)
    sys.stdout.flush()


@pytest.mark.parametrize("shape,h", [((64, 64, 64), (2.0, 2.0, 2.0)),
                                     ((23, 29, 37), (1.3, 0.7, 2.1)),
                                     ((23, 29, 36), (1.3, 0.7, 2.1))])
def test_tv_prox_matches_oracle(shape, h):
    torch = require_gpu()
    import paper_1002_3675_amd as cb
    rng = np.random.default_rng(20)
    g = rng.uniform(-0.002, 0.02, shape).astype(np.float32).astype(np.float64)
    z0 = rng.uniform(0.0, 0.02, shape).astype(np.float32).astype(np.float64)
    hh = np.array(h)
    for beta, k in [(40.0, 7), (600.0, 3)]:
        z = to_np(cb.tv_prox(to_dev(g), to_dev(z0), hh, beta, 1e-3, k))
        want = oracle.tv_prox(g, z0, hh, beta, 1e-3, k)
        assert rel_l2(z, want) <= 1e-5, rel_l2(z, want)
        assert float(z.min()) >= 0.0


@pytest.mark.parametrize("shape", [(21, 37, 45), (33, 17, 70), (1, 9, 40), (19, 13, 44)])
def test_tv_steps_compose(shape):
    """k inner steps in one call equal k calls of one step, and the oracle;
    the shapes cut tiles, z chunks (16 planes) and the borders."""
    torch = require_gpu()
    import paper_1002_3675_amd as cb
    rng = np.random.default_rng(22)
    g = to_dev(rng.uniform(-0.002, 0.02, shape))
    z0 = to_dev(rng.uniform(0.0, 0.02, shape))
    h = np.array([0.9, 1.1, 2.3])
    for beta, k in [(40.0, 2), (600.0, 5)]:
        many = cb.tv_prox(g, z0, h, beta, 1e-3, k)
        z = z0
        for _ in range(k):
            z = cb.tv_prox(g, z, h, beta, 1e-3, 1)
        assert torch.equal(many, z)
        want = oracle.tv_prox(g.double().cpu().numpy(), z0.double().cpu().numpy(), h, beta,
                              1e-3, k)
        assert rel_l2(to_np(many), want) <= 1e-5


@pytest.mark.parametrize("shape", [(19, 13, 44), (70, 40, 64)])
def test_tv_sweep_aligned_equals_unaligned(shape):
    """Rows of a multiple of 4 voxels in 16-byte aligned arrays take the
    float4 sweep; the same data one float off alignment takes the scalar
    sweep.  Both compute each voxel with the same operations, so the
    results agree bit for bit."""
    torch = require_gpu()
    import paper_1002_3675_amd as cb
    rng = np.random.default_rng(23)
    n = int(np.prod(shape))
    g = to_dev(rng.uniform(-0.002, 0.02, shape))
    z0 = to_dev(rng.uniform(0.0, 0.02, shape))
    h = np.array([0.9, 1.1, 2.3])
    bufs = [torch.empty(n + 1, device="cuda") for _ in range(3)]
    gu, zu, ou = (b[1:].view(shape) for b in bufs)
    assert gu.data_ptr() % 16 == 4
    gu.copy_(g)
    zu.copy_(z0)
    for beta, k in [(40.0, 2), (600.0, 5)]:
        aligned = cb.tv_prox(g, z0, h, beta, 1e-3, k)
        unaligned = cb.tv_prox(gu, zu, h, beta, 1e-3, k, out=ou)
        assert torch.equal(aligned, unaligned)


def test_tv_energy_matches_oracle():
    require_gpu()
    import paper_1002_3675_amd as cb
    rng = np.random.default_rng(21)
    f = rng.uniform(0.0, 0.02, (23, 29, 37)).astype(np.float32).astype(np.float64)
    h = np.array([1.3, 0.7, 2.1])
    e0, e1 = cb.tv_energy(to_dev(f), h, eps=1e-3)
    assert abs(e0 - oracle.tv(f, h)) <= 1e-6 * oracle.tv(f, h)
    assert abs(e1 - oracle.tv(f, h, 1e-3)) <= 1e-6 * oracle.tv(f, h, 1e-3)


def _oracle_settings(g, mu, eps, levels):
    geoms = [g] if levels == 1 else [oracle.coarse_geometry(g), g]
    beta, inner = [], []
    for gl in geoms:
        lam = oracle.power_lambda(gl, 30)
        b = oracle.beta_rule(gl, mu, lam)
        beta.append(b)
        inner.append(oracle.default_inner(np.array([gl.hx, gl.hy, gl.hz]), b, eps))
    return beta, inner


def test_fbs_tiny_matches_oracle():
    """64^3 stand-in phantom, 16 views, I0 = 1e5, mu = 1e-3, 10 iterations."""
    require_gpu()
    import paper_1002_3675_amd as cb
    case = tiny_case()
    g = case.geom
    _log("oracle settings")
    beta, inner = _oracle_settings(g, case.mu, case.eps, 1)
    Y32 = case.Y.astype(np.float32).astype(np.float64)
    _log("oracle solve beta=%s inner=%s" % (beta, inner))
    want = oracle.fbs_solve(g, Y32, case.mu, [10], beta=beta, eps=case.eps, n_inner=inner)
    _log("gpu solve")
    plan = cb.Plan(g)
    f, rep = cb.fbs_solve(plan, to_dev(Y32), cb.FbsParams(mu=case.mu, iters=(10,), beta=beta,
                                                         eps=case.eps, n_inner=inner,
                                                         trace_energy=True))
    err = rel_l2(to_np(f), want["f"])
    e_or = want["report"][0]
    assert err <= 1e-3, err
    assert abs(rep.E - e_or) <= 1e-4 * abs(e_or), (rep.E, e_or)
    assert float(f.min()) >= 0.0
    assert rep.n_inner_used[0] == inner[0]


def test_fbs_two_level_matches_oracle():
    """Coarse-to-fine schedule on a 48^3 grid (coarse 24^3, binned detector)."""
    require_gpu()
    import paper_1002_3675_amd as cb
    g = Geometry(48, 48, 40, 2.6, 2.6, 3.0, 96, 72, 2.0, 2.0, 1000.0, 1500.0, 12)
    ph = random_ellipsoid_object(g, 77, n_inner=(6, 8))
    Y = noisy_log_projections(analytic_projections(g, ph), 5e4, 78)
    Y32 = Y.astype(np.float32).astype(np.float64)
    mu, eps = 1e-3, 1e-3
    beta, inner = _oracle_settings(g, mu, eps, 2)
    _log("oracle two-level solve")
    want = oracle.fbs_solve(g, Y32, mu, [4, 4], beta=beta, eps=eps, n_inner=inner, trace=True)
    plan = cb.Plan(g)
    f, rep = cb.fbs_solve(plan, to_dev(Y32), cb.FbsParams(mu=mu, iters=(4, 4), beta=beta,
                                                         eps=eps, n_inner=inner,
                                                         trace_energy=True))
    err = rel_l2(to_np(f), want["f"])
    assert err <= 1e-3, err
    tr = np.array(rep.trace)
    assert tr.shape == want["trace"].shape
    assert np.max(np.abs(tr[:, 0] - want["trace"][:, 0]) / np.abs(want["trace"][:, 0])) <= 1e-4


def test_fbs_energy_monotone_on_gpu():
    require_gpu()
    import paper_1002_3675_amd as cb
    case = tiny_case()
    plan = cb.Plan(case.geom)
    f, rep = cb.fbs_solve(plan, to_dev(case.Y), cb.FbsParams(mu=case.mu, iters=(8,),
                                                            trace_energy=True))
    e = np.array(rep.trace)[:, 1]
    assert np.all(np.diff(e) <= 1e-6 * np.abs(e[:-1])), e
    assert float(f.min()) >= 0.0


def test_final_energy_mode_matches_traced_solve():
    """trace_energy="final" computes only the returned volume's energy: the
    volume and that energy equal, bit for bit, those of the solve traced at
    every iteration, and a solve without energies returns the same volume."""
    torch = require_gpu()
    import paper_1002_3675_amd as cb
    case = tiny_case()
    plan = cb.Plan(case.geom)
    Y = to_dev(case.Y)
    runs = {}
    for mode in (True, "final", False):
        runs[mode] = cb.fbs_solve(plan, Y, cb.FbsParams(mu=case.mu, iters=(3, 4), beta=(40.0, 40.0),
                                                        trace_energy=mode))
    (ft, rt), (ff, rf), (fn, rn) = runs[True], runs["final"], runs[False]
    assert torch.equal(ft, ff) and torch.equal(ft, fn)
    assert (rf.E, rf.E_eps, rf.E1, rf.E2) == (rt.E, rt.E_eps, rt.E1, rt.E2)
    assert rf.E > 0 and rn.E == 0.0
    assert rf.trace is None and len(rt.trace) == (3 + 1) + (4 + 1)
    assert rt.trace[-1][0] == rt.E


def test_step_api_equals_solve_bitwise():
    torch = require_gpu()
    import paper_1002_3675_amd as cb
    g = Geometry(32, 32, 24, 4.0, 4.0, 5.0, 64, 48, 3.2, 3.2, 1000.0, 1500.0, 10)
    ph = random_ellipsoid_object(g, 5, n_inner=(4, 6))
    Y = to_dev(noisy_log_projections(analytic_projections(g, ph), 5e4, 6))
    plan = cb.Plan(g)
    params = cb.FbsParams(mu=1e-3, iters=(3, 3))
    f1, _ = cb.fbs_solve(plan, Y, params)
    f2 = torch.zeros(g.vol_shape, device="cuda")
    st = cb.FbsState(plan, Y, f2, params)
    n = 0
    while not st.finished:
        st.step(1)
        n += 1
    rep = st.report()
    st.close()
    torch.cuda.synchronize()
    assert n == 6 and rep.iters_done == 6
    assert torch.equal(f1, f2)
