"""The no-allocation TV prox entry point (cbct_tv_prox_noalloc) gives the
same result as cbct_tv_prox, bit for bit, on two calls in a row (the second
on a smaller grid, so the fixed scratch array holds the first call's
contents), with an odd and an even number of sweeps; grids beyond its
fixed scratch are refused with EINVAL.  Also checked against the FP64
oracle's projected gradient steps."""

import numpy as np
import pytest

import oracle

from gpu_util import require_gpu, rel_l2, to_dev, to_np

pytestmark = pytest.mark.gpu


def _case(shape, seed):
    rng = np.random.default_rng(seed)
    g = rng.uniform(0.0, 0.02, shape)
    z0 = np.clip(g + rng.normal(0.0, 0.004, shape), 0.0, None)
    return g, z0


def test_noalloc_prox_equals_allocating_prox():
    torch = require_gpu()
    import paper_1002_3675_amd as cb
    h = (1.5, 1.25, 2.0)
    beta, eps = 600.0, 1e-3
    for shape, n_inner, seed in (((40, 72, 96), 7, 1), ((17, 33, 50), 4, 2)):
        print("noalloc prox %s, %d sweeps" % (shape, n_inner), flush=True)
        g, z0 = _case(shape, seed)
        gd, zd = to_dev(g), to_dev(z0)
        want = cb.tv_prox(gd, zd, h, beta, eps, n_inner)
        got = cb.tv_prox(gd, zd, h, beta, eps, n_inner, noalloc=True)
        torch.cuda.synchronize()
        assert torch.equal(got, want), shape
        # in place (f is z0 on entry) gives the same
        zi = zd.clone()
        cb.tv_prox(gd, zi, h, beta, eps, n_inner, noalloc=True, out=zi)
        assert torch.equal(zi, want), shape
        ref = oracle.tv_prox(g.astype(np.float32).astype(np.float64),
                             z0.astype(np.float32).astype(np.float64), np.array(h), beta, eps,
                             n_inner)
        assert rel_l2(to_np(got), ref) <= 1e-5


def test_noalloc_prox_refuses_grids_beyond_its_scratch():
    torch = require_gpu()
    import paper_1002_3675_amd as cb
    shape = (65, 512, 512)  # 2^24 + 2^18 voxels
    g = torch.zeros(shape, device="cuda")
    with pytest.raises(cb.CbctError) as e:
        cb.tv_prox(g, g, (1.0, 1.0, 1.0), 10.0, 1e-3, 1, noalloc=True)
    assert e.value.code == -1 and "exceeds" in str(e.value)
