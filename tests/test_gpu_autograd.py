"""The differentiable projector: torch.autograd.Function whose backward is
the library's hand-written transpose.  Checked with gradcheck (float64,
32^3 at 6 mm, 60 views, 64x48 detector), central finite differences of
0.5||P f - y||^2 along random directions, and against the FP64 oracle's
P^T (P f - y) on the 128^3 / 60-view / 256x192 workload in float32."""

import numpy as np
import pytest

import oracle
from workloads import diff_inputs

from gpu_util import require_gpu, rel_l2, to_dev, to_np

pytestmark = pytest.mark.gpu


def test_gradcheck_float64_32cubed():
    torch = require_gpu()
    import paper_1002_3675_amd as cb
    g, f, y = diff_inputs(fd=True)
    plan = cb.Plan(g)
    x = torch.tensor(f, dtype=torch.float64, device="cuda", requires_grad=True)
    assert torch.autograd.gradcheck(lambda t: cb.Project.apply(t, plan), (x,),
                                    eps=1e-6, atol=1e-8, rtol=1e-6, fast_mode=True)


def test_loss_gradient_central_differences():
    torch = require_gpu()
    import paper_1002_3675_amd as cb
    g, f, y = diff_inputs(fd=True)
    plan = cb.Plan(g)
    yt = torch.tensor(y, dtype=torch.float64, device="cuda")
    x = torch.tensor(f, dtype=torch.float64, device="cuda", requires_grad=True)

    def loss(t):
        return 0.5 * ((cb.Project.apply(t, plan) - yt) ** 2).sum()

    L = loss(x)
    L.backward()
    grad = x.grad.detach()
    rng = np.random.default_rng(31)
    h = 1e-4
    for _ in range(3):
        d = torch.tensor(rng.standard_normal(g.vol_shape), dtype=torch.float64, device="cuda")
        with torch.no_grad():
            fd = (loss(x + h * d) - loss(x - h * d)) / (2 * h)
        an = (grad * d).sum()
        assert abs(float(fd - an)) <= 1e-7 * abs(float(an)), (float(fd), float(an))


def test_backward_matches_oracle_128cubed():
    """float32 backward of 0.5||P f - y||^2 is P^T (P f - y): within 1e-5 of
    the FP64 oracle applied to the same float32 inputs."""
    torch = require_gpu()
    import paper_1002_3675_amd as cb
    g, f, y = diff_inputs(fd=False)
    f32 = f.astype(np.float32)
    y32 = y.astype(np.float32)
    plan = cb.Plan(g)
    x = torch.tensor(f32, device="cuda", requires_grad=True)
    yt = to_dev(y32)
    loss = 0.5 * ((cb.Project.apply(x, plan) - yt) ** 2).sum()
    loss.backward()
    r = oracle.project(g, f32.astype(np.float64)) - y32.astype(np.float64)
    want = oracle.backproject(g, r)
    assert rel_l2(to_np(x.grad), want) <= 1e-5, rel_l2(to_np(x.grad), want)


def test_autograd_composes_with_torch_ops():
    """P inside a larger graph: a weighted loss and a non-negativity
    reparametrisation f = softplus(w)."""
    torch = require_gpu()
    import paper_1002_3675_amd as cb
    g, f, y = diff_inputs(fd=True)
    plan = cb.Plan(g)
    w = torch.zeros(g.vol_shape, dtype=torch.float64, device="cuda", requires_grad=True)
    yt = torch.tensor(y, dtype=torch.float64, device="cuda")
    wt = torch.linspace(0.5, 1.5, g.n_views, dtype=torch.float64, device="cuda")[:, None, None]
    fv = torch.nn.functional.softplus(w)
    loss = (wt * (cb.Project.apply(fv, plan) - yt) ** 2).sum()
    loss.backward()
    # manual chain rule through the library's operators
    with torch.no_grad():
        r = 2 * wt * (plan.project(fv.detach().contiguous()) - yt)
        want = plan.backproject(r.contiguous()) * torch.sigmoid(w)
    assert torch.allclose(w.grad, want, rtol=1e-12, atol=0)
