"""Pins of the oracle's data term E2 and of the scale of Step 1.

Eq. (1) defines E2 = (1/(N_theta A)) sum_theta ||P^theta f - Y^theta||^2, the
squared residual integrated over each imager of area A and averaged over the
views; with the integral replaced by the pixel sum times the pixel area the
discrete E2 is the mean of the squared residual over all N_meas = N_theta nu nv
pixels.  Step 1 of Algorithm A1 moves f by (mu V / beta) times the functional
derivative of E2; with the derivative at a voxel equal to the partial
derivative over the voxel volume, the update is f - tau P^T (P f - Y) with
tau = (mu / beta) 2 N_vox / N_meas.

The closed forms below fix the denominator of E2 (constant data, a single
non-zero residual, and the grid independence the area and volume
normalisations promise), and a finite-difference test fixes the scale of
Step 1 against E2 itself.  The geometries have N_vox != N_meas, so a swapped
or missing count cannot pass."""

import math

import numpy as np
import pytest

import oracle
from workloads import Geometry

# (geometry, N_vox, N_meas): both counts differ from each other
GEOMS = [
    Geometry(10, 8, 6, 3.0, 3.0, 4.0, 16, 12, 3.2, 3.2, 300.0, 450.0, 3),    # 480 vs 576
    Geometry(12, 12, 12, 2.5, 2.5, 2.5, 20, 10, 2.8, 3.6, 400.0, 600.0, 5),  # 1728 vs 1000
    Geometry(9, 7, 5, 2.0, 2.0, 3.0, 11, 9, 2.0, 2.0, 250.0, 400.0, 7,
             angles=(0.1, 0.9, 1.7, 2.6, 3.3, 4.4, 5.9)),                      # 315 vs 693
]


@pytest.mark.parametrize("g", GEOMS)
@pytest.mark.parametrize("c", [0.7, -2.5])
def test_e2_of_constant_data_is_its_square(g, c):
    """f = 0 and Y = c on every pixel: the residual is -c everywhere and its
    pixel mean square is c^2, whatever the counts of voxels and pixels."""
    assert g.n_vox != g.n_meas
    Y = np.full(g.proj_shape, c)
    e2, r = oracle.data_energy(g, np.zeros(g.vol_shape), Y)
    assert np.array_equal(r, -Y)
    # a sequential sum of N_meas equal terms: rounding below N_meas * 2^-53
    assert abs(e2 - c * c) <= 1e-12 * c * c


@pytest.mark.parametrize("g", GEOMS)
def test_e2_of_single_residual(g):
    """One non-zero pixel r in the residual: E2 = r^2 / N_meas."""
    rng = np.random.default_rng(4)
    for _ in range(3):
        Y = np.zeros(g.proj_shape)
        k, j, i = (int(rng.integers(n)) for n in g.proj_shape)
        rv = float(rng.uniform(0.5, 3.0))
        Y[k, j, i] = rv
        e2, _ = oracle.data_energy(g, np.zeros(g.vol_shape), Y)
        assert abs(e2 - rv * rv / g.n_meas) <= 1e-15 * rv * rv / g.n_meas


def _blob(g, centre, sigma):
    """A Gaussian sampled at the voxel centres (the grid centred on the axis)."""
    ax = [(np.arange(n) - (n - 1) / 2) * h for n, h in ((g.nx, g.hx), (g.ny, g.hy), (g.nz, g.hz))]
    z, y, x = np.meshgrid(ax[2], ax[1], ax[0], indexing="ij")
    d2 = (x - centre[0]) ** 2 + (y - centre[1]) ** 2 + (z - centre[2]) ** 2
    return 0.02 * np.exp(-0.5 * d2 / sigma ** 2)


def test_e2_independent_of_pixel_and_voxel_size():
    """E2 approximates the imager integral over the area A (and the volume
    enters only through the line integrals), so for a smooth object and
    Y = 0 it barely changes when the pixel pitch halves on the same imager
    (four times the pixels) or the voxel spacing halves on the same volume
    (eight times the voxels).  A sum instead of a mean, or a division by
    the voxel count, would move it by a factor of four or eight."""
    base = dict(sad=500.0, sdd=750.0, n_views=4)
    g = Geometry(24, 24, 18, 2.0, 2.0, 2.0, 32, 24, 2.4, 2.4, **base)
    g_pix = Geometry(24, 24, 18, 2.0, 2.0, 2.0, 64, 48, 1.2, 1.2, **base)
    g_vox = Geometry(48, 48, 36, 1.0, 1.0, 1.0, 32, 24, 2.4, 2.4, **base)
    centre, sigma = (1.5, -2.0, 1.0), 6.0
    e = {}
    for name, gg in (("base", g), ("pix", g_pix), ("vox", g_vox)):
        e[name], _ = oracle.data_energy(gg, _blob(gg, centre, sigma), np.zeros(gg.proj_shape))
    assert e["base"] > 0.0
    # the pixel mean of a smooth imager function: O(pitch^2) change
    assert abs(e["pix"] / e["base"] - 1.0) <= 0.005, e
    # trilinear interpolation of the blob: O((h / sigma)^2) change, 1.4% here
    assert abs(e["vox"] / e["base"] - 1.0) <= 0.03, e


@pytest.mark.parametrize("g", GEOMS)
def test_step1_scale_is_the_functional_derivative_of_e2(g):
    """Step 1 with TV off (one exact prox step) maps f0 to
    f1 = f0 - (mu V / beta) dE2/df.  With dE2/df(x_v) = (1/h^3) dE2/df_v,
    (f0 - f1) beta / (mu N_vox) must equal the gradient of the pinned E2,
    checked along random directions by central differences (exact up to
    rounding, E2 being quadratic).  f0 stays well above zero, so the
    non-negativity projection does not act."""
    rng = np.random.default_rng(21)
    f_true = rng.uniform(0.01, 0.02, g.vol_shape)
    Y = oracle.project(g, f_true) + rng.normal(0.0, 0.02, g.proj_shape)
    f0 = f_true + rng.uniform(-0.002, 0.002, g.vol_shape)
    mu, beta = 1e-3, 10.0
    f1 = oracle.fbs_solve(g, Y, mu, [1], f0=f0, beta=[beta], n_inner=[1], tv_weight=0.0)["f"]
    assert np.all(f1 > 0.0)
    grad = (f0 - f1) * beta / (mu * g.n_vox)
    for _ in range(3):
        d = rng.normal(0.0, 1.0, g.vol_shape)
        t = 1e-3
        ep, _ = oracle.data_energy(g, f0 + t * d, Y)
        em, _ = oracle.data_energy(g, f0 - t * d, Y)
        fd = (ep - em) / (2.0 * t)
        an = float(np.sum(grad * d))
        assert abs(an - fd) <= 1e-7 * max(abs(fd), 1e-300), (an, fd)


@pytest.mark.parametrize("g", GEOMS[:2])
def test_landweber_special_case_unequal_counts(g):
    """TV weight 0, one inner step of size 1/beta: each outer iteration is
    projected Landweber, f <- max(0, f - tau P^T (P f - Y)), with tau from
    this geometry's own counts."""
    rng = np.random.default_rng(5)
    Y = oracle.project(g, rng.uniform(0.0, 0.02, g.vol_shape)) + \
        rng.normal(0.0, 0.05, g.proj_shape)
    mu, beta = 1e-3, 0.5
    out = oracle.fbs_solve(g, Y, mu, [3], beta=[beta], n_inner=[1], tv_weight=0.0)
    tau = (mu / beta) * 2.0 * g.n_vox / g.n_meas
    f = np.zeros(g.vol_shape)
    for _ in range(3):
        f = np.maximum(0.0, f - tau * oracle.backproject(g, oracle.project(g, f) - Y))
    assert np.max(np.abs(out["f"] - f)) <= 1e-12 * max(1.0, np.max(np.abs(f)))


@pytest.mark.parametrize("g", GEOMS[:2])
def test_report_energy_recomposed_from_pinned_parts(g):
    """The solver's report (E, E_eps, E1, E2) of its returned volume equals
    E1 from the pinned TV (ramp and step closed forms), E2 from the pinned
    data term, and E = E1 + mu E2, E_eps = E1_eps + mu E2."""
    rng = np.random.default_rng(8)
    Y = oracle.project(g, rng.uniform(0.0, 0.02, g.vol_shape)) + \
        rng.normal(0.0, 0.02, g.proj_shape)
    mu, eps = 2e-3, 1e-3
    out = oracle.fbs_solve(g, Y, mu, [3], eps=eps)
    f = out["f"]
    h = np.array([g.hx, g.hy, g.hz])
    e2, _ = oracle.data_energy(g, f, Y)
    e1, e1e = oracle.tv(f, h, 0.0), oracle.tv(f, h, eps)
    E, Ee, E1, E2 = out["report"]
    assert math.isclose(E2, e2, rel_tol=1e-13)
    assert math.isclose(E1, e1, rel_tol=1e-13)
    assert math.isclose(E, e1 + mu * e2, rel_tol=1e-13)
    assert math.isclose(Ee, e1e + mu * e2, rel_tol=1e-13)
