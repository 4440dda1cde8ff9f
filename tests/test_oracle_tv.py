"""Pins of the oracle's TV pieces (E1 of Eq. (1), Step 2 of Algorithm A1):
adjointness, closed forms of E1, finite differences, monotone inner
descent, and the 1-D case against an exact TV-denoising solution computed
by a library bound-constrained least-squares solver on the dual problem."""

import math

import numpy as np
import pytest
from scipy.optimize import lsq_linear

import oracle

H = np.array([1.3, 0.7, 2.1])


def test_grad_adjoint_identity():
    rng = np.random.default_rng(0)
    z = rng.standard_normal((7, 9, 11))
    p = [rng.standard_normal((7, 9, 11)) for _ in range(3)]
    dz = oracle.grad(z, H)
    lhs = math.fsum(np.concatenate([(a * b).ravel() for a, b in zip(dz, p)]))
    rhs = math.fsum((z * oracle.grad_adjoint(p, H)).ravel())
    assert abs(lhs - rhs) <= 1e-14 * max(abs(lhs), 1.0) * 10


def test_e1_closed_forms():
    nz, ny, nx = 5, 6, 8
    x = (np.arange(nx) - (nx - 1) / 2) * H[0]
    alpha = 0.37
    ramp = np.broadcast_to(alpha * x[None, None, :], (nz, ny, nx)).copy()
    assert abs(oracle.tv(ramp, H) - alpha * (nx - 1) / nx) <= 1e-14
    for m in (1, 3, 7):
        step = np.zeros((nz, ny, nx))
        step[:, :, m:] = 1.0
        assert abs(oracle.tv(step, H) - 1.0 / (nx * H[0])) <= 1e-14
    assert oracle.tv(np.full((nz, ny, nx), 4.2), H) == 0.0
    # smoothed E1 of a constant is eps itself
    assert abs(oracle.tv(np.full((nz, ny, nx), 4.2), H, eps=0.3) - 0.3) <= 1e-15


def test_tv_gradient_finite_differences():
    rng = np.random.default_rng(1)
    z = rng.uniform(0, 0.02, (4, 5, 6))
    eps = 1e-3
    n = z.size
    g = oracle.tv_grad(z, H, eps) / n  # gradient of the voxel-mean E1_eps
    d = 1e-7
    for idx in [(0, 0, 0), (2, 3, 1), (3, 4, 5), (1, 2, 3)]:
        zp = z.copy(); zp[idx] += d
        zm = z.copy(); zm[idx] -= d
        fd = (oracle.tv(zp, H, eps) - oracle.tv(zm, H, eps)) / (2 * d)
        assert abs(fd - g[idx]) <= 1e-7 * max(abs(g[idx]), 1e-3), (idx, fd, g[idx])


def test_prox_constant_is_fixed_point():
    gk = np.full((4, 5, 6), 0.013)
    z = oracle.tv_prox(gk, gk, H, beta=7.0, eps=1e-3, n_inner=25)
    assert np.array_equal(z, gk)


def test_prox_large_beta_returns_g():
    rng = np.random.default_rng(2)
    gk = rng.uniform(0, 1, (4, 5, 6))
    z = oracle.tv_prox(gk, np.zeros_like(gk), H, beta=1e9, eps=1e-3, n_inner=3)
    assert np.max(np.abs(z - gk)) <= 1e-6


def test_prox_descent_is_monotone():
    rng = np.random.default_rng(3)
    gk = rng.uniform(-0.005, 0.02, (6, 7, 8))
    z0 = rng.uniform(0, 0.02, (6, 7, 8))
    z, phi = oracle.tv_prox(gk, z0, H, beta=50.0, eps=1e-3, n_inner=40, want_phi=True)
    assert np.all(z >= 0.0)
    assert np.all(np.diff(phi) <= 1e-14 * np.abs(phi[:-1]))
    assert phi[-1] < phi[0]


def _exact_tv1d(g, lam):
    """argmin 0.5||z-g||^2 + lam*sum|z[i+1]-z[i]| via its dual
    min_{|p|<=lam} 0.5||g - Delta^T p||^2, solved by scipy's lsq_linear."""
    n = len(g)
    Dt = np.zeros((n, n - 1))
    for i in range(n - 1):
        Dt[i + 1, i] = 1.0
        Dt[i, i] = -1.0
    res = lsq_linear(Dt, g, bounds=(-lam, lam), tol=1e-14, max_iter=10000, method="bvls")
    return g - Dt @ res.x


def test_prox_1d_tends_to_exact_tv_denoising():
    """On a 1-D volume (ny = nz = 1) Step 2 minimises
    (1/N)[sum|z_{i+1}-z_i|_eps/h + (beta/2)||z-g||^2]; as eps -> 0 (with the
    inner count large enough to converge) it reaches exact 1-D TV denoising
    with lam = 1/(beta h), at first order in eps (measured constant ~3:
    errors 2.0e-2, 3.0e-3, 9.6e-4 at eps = 1e-2, 1e-3, 3e-4)."""
    rng = np.random.default_rng(4)
    n = 40
    clean = np.repeat([0.2, 1.0, 0.5, 0.8], n // 4)
    g = np.maximum(clean + 0.1 * rng.standard_normal(n), 0.0)
    h = np.array([1.0, 1.0, 1.0])
    beta = 4.0
    zstar = _exact_tv1d(g, 1.0 / (beta * h[0]))
    errs = []
    for eps in (1e-2, 1e-3):
        s = oracle.prox_step(h, beta, eps)
        k = int(40.0 / (s * beta))
        z = oracle.tv_prox(g.reshape(1, 1, n), g.reshape(1, 1, n), h, beta, eps, k)
        errs.append(np.max(np.abs(z.ravel() - zstar)))
    assert errs[0] <= 3.5e-2 and errs[1] <= 3.5e-3, errs
    assert errs[1] < errs[0] / 5.0, errs


def test_default_inner_rule():
    h = np.array([2.0, 2.0, 2.0])
    beta, eps = 40.0, 1e-3
    k = oracle.default_inner(h, beta, eps)
    s = oracle.prox_step(h, beta, eps)
    assert k == min(200, math.ceil(3 * (1 + 4 * 0.75 / (eps * beta))))
    assert (1 - s * beta) ** k <= math.exp(-3) * 1.0000001 or k == 200
