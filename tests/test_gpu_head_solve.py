"""Full-size gates: the head workload (512x512x70, 40 views, 512x384) with
the full two-level 20 + 20 schedule against the FP64 oracle's solve stored
by tests/golden/make_head_fbs.py (energy within 1e-4; volume within 1e-3
relative L2 on five whole axial planes, the first and last included, and
on 4096 seeded non-air voxels of the field of view; every plane's norm and
sum, and the whole volume's norm, within 1e-3), and the power iteration
that sets beta against the oracle's."""

import json
import os
import sys

import numpy as np
import pytest

import oracle
from workloads import head_case, tiny_geometry

from gpu_util import require_gpu

pytestmark = pytest.mark.gpu

HERE = os.path.dirname(os.path.abspath(__file__))
GOLDEN = os.path.join(HERE, "golden", "head40_fbs.json")


def test_head_full_schedule_matches_oracle():
    torch = require_gpu()
    if not os.path.exists(GOLDEN):
        pytest.skip("golden oracle solve not generated (tests/golden/make_head_fbs.py)")
    import paper_1002_3675_amd as cb
    sys.path.insert(0, os.path.join(HERE, "golden"))
    import make_head_fbs as mk
    want = json.load(open(GOLDEN))
    case = head_case(40, iters=(20, 20))
    g = case.geom
    plan = cb.Plan(g)
    print("head solve: 512x512x70, 40 views, 20 + 20 iterations", flush=True)
    Y = torch.as_tensor(case.Y.astype(np.float32), device="cuda")
    f, rep = cb.fbs_solve(plan, Y, cb.FbsParams(mu=case.mu, iters=(20, 20), beta=want["beta"],
                                               eps=case.eps, n_inner=want["n_inner"],
                                               trace_energy=True))
    vol = f.cpu().double().numpy().reshape(g.vol_shape)
    assert float(vol.min()) >= 0.0
    assert abs(rep.E - want["E"]) <= 1e-4 * abs(want["E"]), (rep.E, want["E"])
    # whole volume: its norm
    assert abs(np.linalg.norm(vol) - want["f_norm"]) <= 1e-3 * want["f_norm"]
    # seeded voxels of the field of view where the phantom is not air
    got = vol.ravel()[mk.sample_indices(case)]
    ref = np.array(want["samples"])
    err = np.linalg.norm(got - ref) / np.linalg.norm(ref)
    print("head solve: E rel %.2e, samples rel L2 %.2e"
          % (abs(rep.E - want["E"]) / want["E"], err), flush=True)
    assert err <= 1e-3, err
    # every z plane: L2 norm and sum
    tot = np.linalg.norm(vol)
    for k in range(g.nz):
        pn, ps = np.linalg.norm(vol[k]), vol[k].sum()
        assert abs(pn - want["plane_norm"][k]) <= 1e-3 * max(want["plane_norm"][k], 1e-3 * tot), k
        assert abs(ps - want["plane_sum"][k]) <= 1e-3 * max(abs(want["plane_sum"][k]),
                                                          1e-3 * abs(sum(want["plane_sum"]))), k
    # whole axial planes, the first and the last included; a plane the
    # oracle leaves exactly zero (no object there, clipped by f >= 0) must
    # stay zero to 1e-3 of the RMS plane norm
    slices = np.load(os.path.join(HERE, "golden", mk.SLICE_NAME))
    rms_plane = want["f_norm"] / np.sqrt(g.nz)
    for k in want["slices"]:
        ref = slices["z%d" % k].astype(np.float64)
        rn = np.linalg.norm(ref)
        if rn > 0.0:
            err = np.linalg.norm(vol[k] - ref) / rn
            print("head solve: plane %d rel L2 %.2e" % (k, err), flush=True)
            assert err <= 1e-3, (k, err)
        else:
            assert np.linalg.norm(vol[k]) <= 1e-3 * rms_plane, (k, np.linalg.norm(vol[k]))


def test_power_iteration_matches_oracle():
    require_gpu()
    import paper_1002_3675_amd as cb
    g = tiny_geometry()
    lam_gpu = cb.Plan(g).power_lambda(30)
    lam_or = oracle.power_lambda(g, 30)
    assert abs(lam_gpu - lam_or) <= 1e-5 * lam_or, (lam_gpu, lam_or)


def test_automatic_beta_matches_oracle_rule():
    torch = require_gpu()
    import paper_1002_3675_amd as cb
    from workloads import tiny_case
    case = tiny_case()
    g = case.geom
    plan = cb.Plan(g)
    _, rep = cb.fbs_solve(plan, torch.as_tensor(case.Y, dtype=torch.float32, device="cuda"),
                          cb.FbsParams(mu=case.mu, iters=(1,), eps=case.eps))
    want = oracle.beta_rule(g, case.mu, oracle.power_lambda(g, 30))
    assert abs(rep.beta_used[0] - want) <= 1e-5 * want
    assert rep.n_inner_used[0] == oracle.default_inner(np.array([g.hx, g.hy, g.hz]),
                                                       rep.beta_used[0], case.eps)
