"""Pins of the oracle's solver (Algorithm A1 with the coarse-to-fine
schedule): textbook special cases (projected Landweber when the TV weight is
zero, the exact fixed point of consistent data), the monotone energy and
non-negativity guaranteed by the step-size rule, the power iteration against
a dense eigen-solver, the multi-grid transfers on linear fields, and the
divergence of the paper's literal beta ~ 10 mu in millimetre units."""

import math

import numpy as np
import pytest

import oracle
from workloads import Geometry, analytic_projections, noisy_log_projections, \
    shepp_logan_standin


def _small_data(g, seed=7):
    # the 64^3 stand-in phantom scaled into the 24^3 x 4 mm grid's FOV
    ph = shepp_logan_standin(1000)
    return noisy_log_projections(analytic_projections(g, ph), 1e5, seed)


def test_landweber_special_case(small_geom):
    """TV weight 0 and one inner step of size 1/beta: Step 2 returns g, so
    each outer iteration is f <- max(0, f - tau P^T (P f - Y)) with
    tau = (mu/beta) * 2 N_vox / N_meas."""
    g = small_geom
    Y = _small_data(g)
    mu, beta = 1e-3, 0.05
    out = oracle.fbs_solve(g, Y, mu, [3], beta=[beta], n_inner=[1], tv_weight=0.0)
    tau = (mu / beta) * 2.0 * g.n_vox / g.n_meas
    f = np.zeros(g.vol_shape)
    for _ in range(3):
        f = np.maximum(0.0, f - tau * oracle.backproject(g, oracle.project(g, f) - Y))
    assert np.max(np.abs(out["f"] - f)) <= 1e-14 * max(1.0, np.max(np.abs(f))) * 100


def test_consistent_data_fixed_point(small_geom):
    """Y = P f_true, TV off, f0 = f_true: every iterate equals f_true."""
    g = small_geom
    rng = np.random.default_rng(11)
    f_true = rng.uniform(0.0, 0.02, g.vol_shape)
    Y = oracle.project(g, f_true)
    out = oracle.fbs_solve(g, Y, 1e-3, [4], f0=f_true, beta=[0.05], n_inner=[1],
                           tv_weight=0.0)
    assert np.max(np.abs(out["f"] - f_true)) <= 1e-14


@pytest.mark.parametrize("levels", [[6], [3, 3]])
def test_monotone_energy_and_nonnegative(small_geom, levels):
    """With beta = 1.1 * L_N (power iteration) the smoothed energy E_eps
    never increases over the outer iterations of a level, and f >= 0."""
    g = small_geom
    Y = _small_data(g)
    out = oracle.fbs_solve(g, Y, 1e-3, levels, trace=True)
    assert np.all(out["f"] >= 0.0)
    tr = out["trace"]
    row = 0
    for n in levels:
        e = tr[row:row + n + 1, 1]
        assert np.all(np.diff(e) <= 1e-14 * np.abs(e[:-1])), e
        assert e[-1] < e[0]
        row += n + 1
    # report = energies of the returned volume, matches the last trace row
    assert np.allclose(out["report"], tr[-1], rtol=1e-13, atol=0)


def test_power_iteration_against_dense_eigensolver():
    g = Geometry(6, 5, 4, 3.0, 3.0, 4.0, 9, 6, 3.0, 3.0, 300.0, 450.0, 3,
                 angles=(0.0, 2.0, 4.1))
    nvox = g.n_vox
    A = np.zeros((g.n_meas, nvox))
    for v in range(nvox):
        e = np.zeros(nvox)
        e[v] = 1.0
        A[:, v] = oracle.project(g, e.reshape(g.vol_shape)).ravel()
    lam_max = np.linalg.eigvalsh(A.T @ A)[-1]
    lam = oracle.power_lambda(g, 30)
    assert lam <= lam_max * (1 + 1e-12)
    assert lam >= 0.99 * lam_max, (lam, lam_max)


def test_literal_beta_ten_mu_diverges(small_geom):
    """The paper's empirical beta ~ 10 mu is tied to its (unstated) units.
    With lengths in mm the data step tau = (mu/beta) 2 N_vox/N_meas times the
    largest eigenvalue of P^T P is thousands, far above the stability limit
    2, and the update overshoots: the energy jumps by orders of magnitude.
    (Step 2 is taken exactly here, TV weight 0, so that only the data step
    is tested; with TV on, a few inner steps of size 1/Lipschitz barely move
    z at this beta, which hides the instability rather than curing it.)
    The rule beta = 1.1 L_N on the same data decreases the energy."""
    g = small_geom
    Y = _small_data(g)
    mu = 1e-3
    lam = oracle.power_lambda(g, 30)
    tau = (mu / (10 * mu)) * 2.0 * g.n_vox / g.n_meas
    assert tau * lam > 1000.0
    bad = oracle.fbs_solve(g, Y, mu, [4], beta=[10 * mu], n_inner=[1], tv_weight=0.0,
                           trace=True)["trace"][:, 3]
    assert bad.max() > 100.0 * bad[0], bad
    good = oracle.fbs_solve(g, Y, mu, [4], n_inner=[1], tv_weight=0.0, trace=True)["trace"][:, 3]
    assert np.all(np.diff(good) <= 0.0) and good[-1] < 0.5 * good[0], good


def test_prolongation_reproduces_linear_fields():
    cz, cy, cx = 5, 6, 7
    hc = np.array([2.0, 3.0, 4.0])  # coarse spacing; fine spacing is half
    xc = [(np.arange(n) - (n - 1) / 2) * hc[a] for a, n in enumerate((cx, cy, cz))]
    fine = (2 * cz, 2 * cy, 2 * cx)
    xf = [(np.arange(2 * n) - (2 * n - 1) / 2) * hc[a] / 2 for a, n in enumerate((cx, cy, cz))]
    a0, a = 0.3, np.array([0.01, -0.02, 0.005])
    zc, yc, xcc = np.meshgrid(xc[2], xc[1], xc[0], indexing="ij")
    fc = a0 + a[0] * xcc + a[1] * yc + a[2] * zc
    ff = oracle.prolong(fc, fine)
    zf, yf, xff = np.meshgrid(xf[2], xf[1], xf[0], indexing="ij")
    want = a0 + a[0] * xff + a[1] * yf + a[2] * zf
    inner = (slice(1, -1), slice(1, -1), slice(1, -1))
    assert np.max(np.abs(ff[inner] - want[inner])) <= 1e-14
    assert np.max(np.abs(oracle.prolong(np.full((cz, cy, cx), 0.7), fine) - 0.7)) <= 1e-15
    # restriction (2x2x2 mean) and detector binning (2x2 mean) of a linear
    # field sample the same field at the coarse centres
    assert np.max(np.abs(oracle.restrict(want) - fc)) <= 1e-14
    y = np.broadcast_to(want[0], (3,) + want.shape[1:]).copy()
    want_bin = fc[0] + a[2] * (xf[2][0] - xc[2][0])  # fine slice 0 sits below coarse 0
    assert np.max(np.abs(oracle.bin_detector(y) - want_bin[None])) <= 1e-14


def test_clip_inside_vs_after_agree_near_convergence():
    """Clipping inside every inner step (used) and clipping once after the
    inner loop (the literal order of Algorithm A1) give nearly the same
    prox when g is mostly non-negative."""
    rng = np.random.default_rng(9)
    h = np.array([2.0, 2.0, 2.0])
    gk = rng.uniform(-0.002, 0.02, (6, 6, 6))
    beta, eps = 40.0, 1e-3
    k = 2000
    z0 = np.maximum(gk, 0)
    a = oracle.tv_prox(gk, z0, h, beta, eps, k, clip_mode=0)
    b = oracle.tv_prox(gk, z0, h, beta, eps, k, clip_mode=1)
    assert np.max(np.abs(a - b)) <= 2e-3
    assert np.all(a >= 0) and np.all(b >= 0)
