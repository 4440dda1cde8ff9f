"""Pins of the oracle's Eq. (2) operator (the paper's gather-form gradient,
scaled like the matrix transpose) and of the solver's Eq. (2) mode.

- On the central ray of a view, the imager point is the detector centre and
  the weight L^3/(L0 l^2) reduces to the squared magnification SDD^2/l^2
  (the inverse-square law): exact.
- A voxel whose imager point falls between four pixel centres reads their
  mean (bilinear weights 1/4): exact.
- For a smooth residual the operator converges, at first order in the
  pixel pitch, to the matrix transpose P^T (pinned independently by brute
  force and dot tests), because both approximate the same continuum
  adjoint.
- With inverse-crime data and the phantom as the start, the residual is
  zero, so the Eq. (2) solver (TV off) leaves f unchanged.
"""

import numpy as np

import oracle
from workloads import Geometry, tiny_geometry


def _axis_geometry(nu, nv):
    return Geometry(5, 9, 5, 1.0, 1.0, 1.0, nu, nv, 1.0, 1.0, 100.0, 150.0, 1, angles=(0.0,))


def test_central_ray_inverse_square():
    g = _axis_geometry(5, 5)
    y = np.zeros(g.proj_shape)
    y[0, 2, 2] = 1.0  # the centre pixel
    out = oracle.eq2_backproject(g, y)
    for j in range(g.ny):
        l = (j - 0.5 * (g.ny - 1)) * g.hy + g.sad  # source at (0, -SAD, 0)
        assert abs(out[2, j, 2] - (g.sdd / l) ** 2) <= 1e-13 * (g.sdd / l) ** 2


def test_between_four_pixels_reads_their_mean():
    g = _axis_geometry(4, 4)  # the centre lies between pixels 1 and 2 on both axes
    rng = np.random.default_rng(7)
    y = rng.uniform(-1.0, 1.0, g.proj_shape)
    y[0, 1, 1], y[0, 1, 2], y[0, 2, 1], y[0, 2, 2] = 1.0, 2.0, 3.0, 4.0
    out = oracle.eq2_backproject(g, y)
    for j in range(g.ny):
        l = (j - 0.5 * (g.ny - 1)) * g.hy + g.sad
        want = 2.5 * (g.sdd / l) ** 2
        assert abs(out[2, j, 2] - want) <= 1e-13 * want


def test_converges_to_the_matrix_transpose():
    errs = []
    for scale in (1, 2, 4):
        g = Geometry(24, 24, 24, 2.0, 2.0, 2.0, 48 * scale, 36 * scale, 3.2 / scale,
                     3.2 / scale, 300.0, 450.0, 4, angles=(0.1, 1.3, 2.9, 4.4))
        u = (np.arange(g.nu) - 0.5 * (g.nu - 1)) * g.au
        v = (np.arange(g.nv) - 0.5 * (g.nv - 1)) * g.av
        U, V = np.meshgrid(u, v)
        y = np.stack([np.exp(-((U - 10 * np.cos(k)) ** 2 + (V - 5 * k) ** 2) / (2 * 30.0 ** 2))
                      for k in range(4)])
        a, b = oracle.backproject(g, y), oracle.eq2_backproject(g, y)
        sl = (slice(4, 20),) * 3
        errs.append(np.linalg.norm((a - b)[sl]) / np.linalg.norm(a[sl]))
    assert errs[0] > 1.8 * errs[1] > 3.2 * errs[2], errs  # first order in the pitch
    assert errs[2] < 5e-3, errs


def test_eq2_solver_keeps_an_exact_solution():
    g = tiny_geometry()
    rng = np.random.default_rng(8)
    f = rng.uniform(0.0, 0.02, g.vol_shape)
    Y = oracle.project(g, f)
    out = oracle.fbs_solve(g, Y, 1e-3, (3,), f0=f, beta=(1.0,), n_inner=(4,),
                           tv_weight=0.0, gradient="eq2")
    assert np.array_equal(out["f"], f)


def test_off_centre_bilinear_fractions():
    """Voxel (1, 0, 0) mm at theta = 0 projects to u* = 1.5 mm (SDD/SAD =
    1.5); with 2 mm pixels centred at -4..4 mm that is index 2.75, so it
    reads 1/4 of pixel 2 and 3/4 of pixel 3 (and likewise along v for the
    voxel (0, 0, 1) mm)."""
    g = Geometry(5, 5, 5, 1.0, 1.0, 1.0, 5, 5, 2.0, 2.0, 100.0, 150.0, 1, angles=(0.0,))
    L = np.sqrt(150.0 ** 2 + 1.5 ** 2)
    l2 = 100.0 ** 2 + 1.0
    w = L ** 3 / (150.0 * l2) * (1.0 / 4.0)  # h^3/(au av) = 1/4
    y = np.zeros(g.proj_shape)
    y[0, 2, 2], y[0, 2, 3] = 1.0, 0.0
    out = oracle.eq2_backproject(g, y)
    assert abs(out[2, 2, 3] - 0.25 * w) <= 1e-13 * w   # x = +1 mm: i = 3
    y = np.zeros(g.proj_shape)
    y[0, 2, 2], y[0, 3, 2] = 0.0, 1.0
    out = oracle.eq2_backproject(g, y)
    assert abs(out[3, 2, 2] - 0.75 * w) <= 1e-13 * w   # z = +1 mm: k = 3
