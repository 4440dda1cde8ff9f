"""Pins of the FP64 oracle's projector P and its transpose against things
other than the oracle itself: brute force with a different formulation,
closed forms, Riemann-sum bounds, convergence orders, and the paper's
continuous gradient formula Eq. (2) as an asymptotic identity."""

import math

import numpy as np
import pytest

import oracle
from workloads import Geometry, tiny_geometry, analytic_projections, \
    shepp_logan_standin, voxelise


# ---------------------------------------------------------------- helpers --

def _rays(g, k, theta):
    """Source and unit directions of every pixel of one view, written out
    directly from the scan description (independent of the oracle)."""
    c, s = math.cos(theta), math.sin(theta)
    src = np.array([g.sad * s, -g.sad * c, 0.0])
    out = []
    for j in range(g.nv):
        for i in range(g.nu):
            u = (i - (g.nu - 1) / 2) * g.au
            v = (j - (g.nv - 1) / 2) * g.av
            d = np.array([-(g.sdd - g.sad) * s + u * c, (g.sdd - g.sad) * c + u * s, v])
            e = d - src
            out.append(e / np.linalg.norm(e))
    return src, np.array(out)


def _brute_project(g, f, angles):
    """P by brute force: every sample n*step for n = 0 .. far past the
    volume, interpolant evaluated as sum over ALL voxels of f_v times the
    product of hat functions (no cell lookup, no clipping)."""
    h = np.array([g.hx, g.hy, g.hz])
    n = np.array([g.nx, g.ny, g.nz])
    cen = [(np.arange(n[a]) - (n[a] - 1) / 2) * h[a] for a in range(3)]
    zz, yy, xx = np.meshgrid(cen[2], cen[1], cen[0], indexing="ij")
    vc = np.stack([xx.ravel(), yy.ravel(), zz.ravel()], axis=1)
    fv = f.ravel()
    step = g.step
    nmax = int(math.ceil((g.sad + np.linalg.norm(n * h)) / step)) + 2
    ts = np.arange(nmax + 1) * step
    y = np.zeros((g.n_views, g.nv, g.nu))
    for k, th in enumerate(angles):
        src, dirs = _rays(g, k, th)
        for r, e in enumerate(dirs):
            p = src[None, :] + ts[:, None] * e[None, :]
            w = np.ones((len(ts), len(fv)))
            for a in range(3):
                w *= np.maximum(0.0, 1.0 - np.abs(p[:, a:a + 1] - vc[None, :, a]) / h[a])
            y[k, r // g.nu, r % g.nu] = step * np.sum(w @ fv)
    return y


TINY_ODD = Geometry(4, 3, 5, 2.0, 1.5, 2.5, 5, 3, 2.2, 2.9, 100.0, 150.0, 2,
                    angles=(0.3, 2.1), step=0.7)


# ------------------------------------------------------------------ pins --

def test_project_matches_brute_force():
    g = TINY_ODD
    f = np.random.default_rng(5).uniform(0.0, 1.0, g.vol_shape)
    want = _brute_project(g, f, g.angles)
    got = oracle.project(g, f)
    assert np.max(np.abs(got - want)) <= 1e-13 * np.max(np.abs(want))


def test_dense_transpose_brute_force():
    """The scatter P^T equals the transpose of the brute-force matrix."""
    g = TINY_ODD
    nvox, nmeas = g.n_vox, g.n_meas
    A = np.zeros((nmeas, nvox))
    for v in range(nvox):
        e = np.zeros(nvox)
        e[v] = 1.0
        A[:, v] = _brute_project(g, e.reshape(g.vol_shape), g.angles).ravel()
    for r in range(nmeas):
        e = np.zeros(nmeas)
        e[r] = 1.0
        col = oracle.backproject(g, e.reshape(g.proj_shape)).ravel()
        assert np.max(np.abs(col - A[r])) <= 1e-14 * max(1.0, np.max(np.abs(A)))


def test_impulse_closed_form():
    """Ray along y through the centre of a 5^3 grid with the sample lattice
    on the y knots: the projection of a unit voxel on the ray is h_y times
    the x and z hat weights, i.e. exactly h = 2 for voxels on the ray."""
    g = Geometry(5, 5, 5, 2.0, 2.0, 2.0, 7, 5, 1.0, 1.0, 1000.0, 1500.0, 1,
                 angles=(0.0,), step=1.0)
    ci, cj = 3, 2  # centre pixel of the 7x5 detector
    for (ix, iy, iz), expect in [((2, 0, 2), 2.0), ((2, 2, 2), 2.0), ((2, 4, 2), 2.0),
                                 ((1, 2, 2), 0.0), ((2, 2, 3), 0.0)]:
        f = np.zeros(g.vol_shape)
        f[iz, iy, ix] = 1.0
        y = oracle.project(g, f)
        assert abs(y[0, cj, ci] - expect) <= 1e-14


def test_constant_volume_riemann_bound():
    """P of the all-ones volume along rays that cross only the two x faces
    of the grid: the interpolant is a trapezoid in x with ramps of one
    voxel, so the line integral is N_x h_x / |e_x| and the uniform-sample sum
    differs from it by at most 4 * (|e_x|/h_x) * step^2 / 8."""
    g = Geometry(10, 60, 60, 2.0, 2.0, 2.0, 9, 9, 2.0, 2.0, 1000.0, 1500.0, 1,
                 angles=(math.pi / 2,), step=0.37)
    y = oracle.project(g, np.ones(g.vol_shape))
    src, dirs = _rays(g, 0, math.pi / 2)
    for r, e in enumerate(dirs):
        ex = abs(e[0])
        exact = g.nx * g.hx / ex
        bound = 4.0 * (ex / g.hx) * g.step ** 2 / 8.0
        assert abs(y[0, r // g.nu, r % g.nu] - exact) <= bound + 1e-12


def _gauss_error(n, h, step, sigma=6.0, rho=1.0):
    g = Geometry(n, n, n, h, h, h, 31, 21, 0.6, 0.6, 400.0, 600.0, 2,
                 angles=(0.2, 1.3), step=step)
    c = np.array([2.0, -1.5, 1.0])
    cen = (np.arange(n) - (n - 1) / 2) * h
    zz, yy, xx = np.meshgrid(cen, cen, cen, indexing="ij")
    f = rho * np.exp(-((xx - c[0]) ** 2 + (yy - c[1]) ** 2 + (zz - c[2]) ** 2) / (2 * sigma ** 2))
    y = oracle.project(g, f)
    err = 0.0
    for k, th in enumerate(g.angles):
        src, dirs = _rays(g, k, th)
        proj = np.sum((c - src)[None, :] * dirs, axis=1)
        dist2 = np.sum((src - c) ** 2) - proj ** 2
        exact = rho * sigma * math.sqrt(2 * math.pi) * np.exp(-dist2 / (2 * sigma ** 2))
        err = max(err, np.max(np.abs(y[k].ravel() - exact)))
    return err


def test_gaussian_blob_second_order():
    """Line integrals of a Gaussian blob converge at order 2 in the voxel
    size (trilinear interpolation error), to the closed form
    rho*sigma*sqrt(2 pi)*exp(-d^2/(2 sigma^2))."""
    e1 = _gauss_error(24, 2.0, 1.0)
    e2 = _gauss_error(48, 1.0, 0.5)
    order = math.log2(e1 / e2)
    assert 1.7 <= order <= 2.3, (e1, e2, order)


def test_ellipsoid_phantom_consistent_with_analytic_data():
    """P of the voxelised phantom approaches the exact line integrals of the
    ellipsoids (independent geometry code in the input generator) at first
    order in the voxel size: sharp edges are blurred over one voxel."""
    import dataclasses
    g0 = tiny_geometry()
    ph = shepp_logan_standin(1000)
    errs = []
    for n, h in [(32, 4.0), (64, 2.0), (128, 1.0)]:
        g = dataclasses.replace(g0, nx=n, ny=n, nz=n, hx=h, hy=h, hz=h, n_views=4)
        p_exact = analytic_projections(g, ph)
        y = oracle.project(g, voxelise(g, ph, sub=2))
        errs.append(np.linalg.norm(y - p_exact) / np.linalg.norm(p_exact))
    assert errs[1] < 0.03, errs
    for a, b in zip(errs, errs[1:]):
        assert 1.7 < a / b < 2.4, errs


@pytest.mark.parametrize("seed", [0, 1])
def test_dot_product_adjoint(small_geom, seed):
    rng = np.random.default_rng(seed)
    f = rng.uniform(0, 0.02, small_geom.vol_shape)
    y = rng.uniform(0, 4, small_geom.proj_shape)
    a = math.fsum((oracle.project(small_geom, f) * y).ravel())
    b = math.fsum((f * oracle.backproject(small_geom, y)).ravel())
    assert abs(a - b) <= 1e-12 * abs(a)


try:
    from hypothesis import given, settings, strategies as st

    @settings(max_examples=12, deadline=None)
    @given(st.integers(3, 7), st.integers(3, 7), st.integers(2, 6),
           st.floats(0.5, 3.0), st.floats(0.5, 3.0), st.floats(0.5, 3.0),
           st.integers(3, 9), st.integers(2, 7), st.floats(0.0, 6.28),
           st.floats(0.2, 1.5))
    def test_dot_product_random_geometries(nx, ny, nz, hx, hy, hz, nu, nv, th, step):
        g = Geometry(nx, ny, nz, hx, hy, hz, nu, nv, 1.3, 1.1, 200.0, 330.0, 3,
                     angles=(th, th + 1.0, th + 2.5), step=step)
        rng = np.random.default_rng(nx * 7 + nu)
        f = rng.standard_normal(g.vol_shape)
        y = rng.standard_normal(g.proj_shape)
        a = math.fsum((oracle.project(g, f) * y).ravel())
        b = math.fsum((f * oracle.backproject(g, y)).ravel())
        scale = math.fsum(np.abs(oracle.project(g, np.abs(f)) * np.abs(y)).ravel())
        assert abs(a - b) <= 1e-12 * max(scale, 1e-300)
except ImportError:  # pragma: no cover
    pass


def test_transpose_scale_matches_eq2():
    """Eq. (2): the continuous adjoint of the cone-beam projection at view
    theta weights the residual at (u*, v*) by L^3 / (L0 l^2).  With fine
    detector and sample spacing the discrete transpose of ones therefore
    tends to (h_x h_y h_z / (a_u a_v)) * sum_theta L^3 / (L0 l^2) at voxel
    centres; the error shrinks as the sampling is refined."""
    def rel_err(pitch, step):
        n = 9
        nu = int(round(60.0 / pitch)) | 1
        g = Geometry(n, n, n, 2.0, 2.0, 2.0, nu, nu, pitch, pitch, 200.0, 300.0, 3,
                     angles=(0.1, 2.2, 4.0), step=step)
        bt = oracle.backproject(g, np.ones(g.proj_shape))
        cen = (np.arange(n) - (n - 1) / 2) * 2.0
        errs = []
        for (i, j, k) in [(4, 4, 4), (2, 5, 3), (6, 3, 5), (3, 3, 6)]:
            x = np.array([cen[i], cen[j], cen[k]])
            pred = 0.0
            for th in g.angles:
                src = np.array([g.sad * math.sin(th), -g.sad * math.cos(th), 0.0])
                ew = np.array([-math.sin(th), math.cos(th), 0.0])
                l = np.linalg.norm(x - src)
                depth = np.dot(x - src, ew)
                L = g.sdd * l / depth  # distance from source to (u*, v*)
                pred += L ** 3 / (g.sdd * l ** 2)
            pred *= 8.0 / (pitch * pitch)
            errs.append(abs(bt[k, j, i] - pred) / pred)
        return max(errs)

    e_coarse = rel_err(0.5, 0.25)
    e_fine = rel_err(0.25, 0.125)
    assert e_fine < 2e-3 and e_fine < e_coarse, (e_coarse, e_fine)


def test_sample_count_matches_definition():
    """S counts every n with n*step inside the padded box, summed over rays."""
    g = TINY_ODD
    src_total = 0
    half = np.array([(g.nx + 1) * g.hx, (g.ny + 1) * g.hy, (g.nz + 1) * g.hz]) / 2
    for k, th in enumerate(g.angles):
        src, dirs = _rays(g, k, th)
        for e in dirs:
            ts = np.arange(0, 4000) * g.step
            p = src[None] + ts[:, None] * e[None]
            src_total += int(np.sum(np.all(np.abs(p) <= half[None], axis=1)))
    assert oracle.count_samples(g) == src_total
