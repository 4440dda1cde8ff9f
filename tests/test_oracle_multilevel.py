"""Pins of the oracle's deeper multigrid and its stopping rule: where each
coarser level's cells and pixels sit (linear fields through the 2x2x2 and
2x2 means, odd sizes included), the volume-centre shift (a padded grid
holding the same function gives the same projections), a three-level solve
against the composition of single-level solves and transfers, the relative
change rule against independent fixed-count solves, and the monotone
energy over three levels."""

import dataclasses

import numpy as np
import pytest

import oracle
from workloads import Geometry, analytic_projections, noisy_log_projections, \
    shepp_logan_standin


def _centres(n, h, off):
    return (np.arange(n) - (n - 1) / 2.0) * h + off


@pytest.mark.parametrize("dims", [(8, 6, 4, 10, 8), (7, 6, 5, 9, 7), (9, 11, 3, 5, 13)])
def test_coarse_cells_sit_at_block_centres(dims):
    nx, ny, nz, nu, nv = dims
    g = Geometry(nx, ny, nz, 2.0, 2.5, 3.0, nu, nv, 1.5, 1.7, 400.0, 600.0, 2,
                 u_off=3.1, v_off=-0.7, x_off=1.3, y_off=-2.2, z_off=0.4)
    c = oracle.coarse_geometry(g)
    assert (c.nx, c.ny, c.nz, c.nu, c.nv) == (nx // 2, ny // 2, nz // 2, nu // 2, nv // 2)
    assert (c.hx, c.au, c.step) == (4.0, 3.0, 2.0 * oracle.step_of(g))
    a0, a = 0.3, (0.011, -0.023, 0.0057)
    # a linear field sampled at the fine voxel centres, 2x2x2-averaged, is
    # the same field at the coarse cell centres
    z, y, x = np.meshgrid(_centres(nz, g.hz, g.z_off), _centres(ny, g.hy, g.y_off),
                          _centres(nx, g.hx, g.x_off), indexing="ij")
    zc, yc, xc = np.meshgrid(_centres(c.nz, c.hz, c.z_off), _centres(c.ny, c.hy, c.y_off),
                             _centres(c.nx, c.hx, c.x_off), indexing="ij")
    fine = a0 + a[0] * x + a[1] * y + a[2] * z
    want = a0 + a[0] * xc + a[1] * yc + a[2] * zc
    assert np.max(np.abs(oracle.restrict(fine) - want)) <= 1e-13
    # the same for detector pixels and 2x2 binning
    v, u = np.meshgrid(_centres(nv, g.av, g.v_off), _centres(nu, g.au, g.u_off), indexing="ij")
    vc, uc = np.meshgrid(_centres(c.nv, c.av, c.v_off), _centres(c.nu, c.au, c.u_off),
                         indexing="ij")
    y2 = np.stack([a0 + a[0] * u + a[1] * v] * 2)
    assert np.max(np.abs(oracle.bin_detector(y2) - (a0 + a[0] * uc + a[1] * vc))) <= 1e-13
    with pytest.raises(ValueError):
        oracle.coarse_geometry(dataclasses.replace(g, nz=1))


def test_volume_shift_equals_padding():
    """A grid shifted by whole voxels holds the same function as a wider
    centred grid with zero planes on one side: same P, same Eq. (2) values
    at the same voxels, and P^T matched on the shifted grid."""
    g = Geometry(12, 10, 8, 2.0, 2.0, 2.5, 30, 24, 2.0, 2.0, 300.0, 450.0, 3,
                 angles=(0.3, 1.9, 4.0), step=0.9, x_off=4.0, z_off=-2.5)
    wide = dataclasses.replace(g, nx=16, nz=10, x_off=0.0, z_off=0.0)
    rng = np.random.default_rng(70)
    f = rng.uniform(0.0, 0.02, g.vol_shape)
    fw = np.zeros(wide.vol_shape)
    fw[:-2, :, 4:] = f                       # x: voxel i -> i + 4, z: k -> k
    a, b = oracle.project(g, f), oracle.project(wide, fw)
    assert np.max(np.abs(a - b)) <= 1e-12 * np.max(np.abs(b))
    y = rng.uniform(-1.0, 1.0, g.proj_shape)
    e = oracle.eq2_backproject(g, y)
    ew = oracle.eq2_backproject(wide, y)[:-2, :, 4:]
    assert np.max(np.abs(e - ew)) <= 1e-12 * np.max(np.abs(ew))
    lhs = float(np.sum(a * y))
    rhs = float(np.sum(f * oracle.backproject(g, y)))
    assert abs(lhs - rhs) <= 1e-12 * abs(lhs)


@pytest.fixture(scope="module")
def odd_case():
    g = Geometry(22, 20, 14, 4.0, 4.0, 4.5, 46, 34, 3.2, 3.2, 1000.0, 1500.0, 8)
    Y = noisy_log_projections(analytic_projections(g, shepp_logan_standin(1000)), 1e5, 71)
    return g, Y


def test_three_levels_equal_composed_single_levels(odd_case):
    g, Y = odd_case
    mu, iters = 1e-3, (2, 2, 2)
    out = oracle.fbs_solve(g, Y, mu, iters, trace=True)
    g1 = oracle.coarse_geometry(g)
    g0 = oracle.coarse_geometry(g1)
    assert (g0.nx, g0.ny, g0.nz, g0.nu, g0.nv) == (5, 5, 3, 11, 8)
    Y1 = oracle.bin_detector(Y)
    Y0 = oracle.bin_detector(Y1)
    f = np.zeros((g0.nz, g0.ny, g0.nx))
    rows = []
    for lev, (gl, Yl, nxt) in enumerate(((g0, Y0, g1), (g1, Y1, g), (g, Y, None))):
        step = oracle.fbs_solve(gl, Yl, mu, (iters[lev],), f0=f, trace=True)
        assert step["used_beta"][0] == out["used_beta"][lev]
        assert step["used_inner"][0] == out["used_inner"][lev]
        rows.append(step["trace"])
        f = step["f"] if nxt is None else oracle.prolong(step["f"], (nxt.nz, nxt.ny, nxt.nx))
    assert np.array_equal(out["f"], f)
    assert np.allclose(out["trace"], np.concatenate(rows), rtol=1e-13, atol=0)
    assert list(out["used_iters"]) == [2, 2, 2]


def test_relative_change_rule_against_fixed_counts(odd_case):
    g, Y = odd_case
    mu = 1e-3
    beta = oracle.fbs_solve(g, Y, mu, (1,))["used_beta"]
    runs = [np.zeros(g.vol_shape)] + [oracle.fbs_solve(g, Y, mu, (k,), beta=beta)["f"]
                                      for k in range(1, 9)]
    ch = [np.linalg.norm(runs[k] - runs[k - 1]) / np.linalg.norm(runs[k]) for k in range(1, 9)]
    assert all(np.diff(ch[1:]) < 0), ch    # the change shrinks after the first step
    for stop in (2, 5):
        tol = 0.5 * (ch[stop - 1] + ch[stop - 2])   # first met at iteration `stop`
        out = oracle.fbs_solve(g, Y, mu, (8,), beta=beta, tol=tol, trace=True)
        assert out["used_iters"][0] == stop
        assert np.array_equal(out["f"], runs[stop])
        assert abs(out["change"][0] - ch[stop - 1]) <= 1e-12 * ch[stop - 1]
        assert out["trace"].shape == (stop + 1, 4)
    # never met: the count is a maximum; tol = 0 is the fixed-count solve
    out = oracle.fbs_solve(g, Y, mu, (3,), beta=beta, tol=1e-12)
    assert out["used_iters"][0] == 3 and np.array_equal(out["f"], runs[3])
    out = oracle.fbs_solve(g, Y, mu, (3,), beta=beta, tol=0.0)
    assert out["used_iters"][0] == 3 and out["change"][0] == 0.0
    # met at once on every level of a three-level solve
    out = oracle.fbs_solve(g, Y, mu, (4, 4, 4), tol=10.0, trace=True)
    assert list(out["used_iters"]) == [1, 1, 1]
    assert out["trace"].shape == (6, 4)     # packed: 2 rows per level
    assert np.allclose(out["trace"][-1], out["report"], rtol=1e-13, atol=0)


def test_monotone_energy_three_levels(odd_case):
    g, Y = odd_case
    out = oracle.fbs_solve(g, Y, 1e-3, (3, 3, 3), trace=True)
    assert np.all(out["f"] >= 0.0)
    row = 0
    for n in (3, 3, 3):
        e = out["trace"][row:row + n + 1, 1]
        assert np.all(np.diff(e) <= 1e-14 * np.abs(e[:-1])), e
        row += n + 1
    with pytest.raises(ValueError):
        oracle.fbs_solve(g, Y, 1e-3, (1, 1, 1, 1, 1))


try:
    from hypothesis import given, settings, strategies as st

    @settings(max_examples=25, deadline=None)
    @given(st.integers(2, 11), st.integers(2, 11), st.integers(2, 11),
           st.integers(2, 13), st.integers(2, 13),
           st.floats(-20.0, 20.0), st.floats(-20.0, 20.0), st.floats(-20.0, 20.0),
           st.floats(-9.0, 9.0), st.floats(-9.0, 9.0))
    def test_coarse_centres_random_sizes_and_shifts(nx, ny, nz, nu, nv, xo, yo, zo, uo, vo):
        """Any sizes (odd or even) and shifts: the 2x2x2 and 2x2 means of a
        linear field sit exactly at the coarse centres; the shifts, the
        dimensions and the pitches of the coarse level follow."""
        g = Geometry(nx, ny, nz, 1.5, 2.0, 2.5, nu, nv, 1.2, 1.4, 500.0, 800.0, 1,
                     u_off=uo, v_off=vo, x_off=xo, y_off=yo, z_off=zo)
        c = oracle.coarse_geometry(g)
        a = (0.013, -0.021, 0.007)
        z, y, x = np.meshgrid(_centres(nz, g.hz, zo), _centres(ny, g.hy, yo),
                              _centres(nx, g.hx, xo), indexing="ij")
        zc, yc, xc = np.meshgrid(_centres(c.nz, c.hz, c.z_off), _centres(c.ny, c.hy, c.y_off),
                                 _centres(c.nx, c.hx, c.x_off), indexing="ij")
        got = oracle.restrict(a[0] * x + a[1] * y + a[2] * z)
        assert np.max(np.abs(got - (a[0] * xc + a[1] * yc + a[2] * zc))) <= 1e-12
        v, u = np.meshgrid(_centres(nv, g.av, vo), _centres(nu, g.au, uo), indexing="ij")
        vc, uc = np.meshgrid(_centres(c.nv, c.av, c.v_off), _centres(c.nu, c.au, c.u_off),
                             indexing="ij")
        got = oracle.bin_detector((a[0] * u + a[1] * v)[None])
        assert np.max(np.abs(got[0] - (a[0] * uc + a[1] * vc))) <= 1e-12
except ImportError:  # pragma: no cover
    pass
