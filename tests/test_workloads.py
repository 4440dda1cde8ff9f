"""Checks of the seeded input generators (not part of the method)."""

import math

import numpy as np

from workloads import Ellipsoid, Geometry, analytic_projections, voxelise, \
    shepp_logan_standin, random_head, head_geometry, tiny_geometry, fov_mask, \
    noisy_log_projections
from workloads.phantoms import _chords, ray_directions


def test_sphere_chord_closed_form():
    g = Geometry(8, 8, 8, 1.0, 1.0, 1.0, 9, 7, 2.0, 2.0, 500.0, 800.0, 2, angles=(0.0, 1.0))
    R = 30.0
    sph = Ellipsoid.make((3.0, -2.0, 1.0), (R, R, R), 1.0, phi=0.7, tilt=0.2)
    p = analytic_projections(g, [sph])
    for k, th in enumerate(g.angles):
        src, dirs = ray_directions(g, th)
        c = np.array([3.0, -2.0, 1.0])
        t = (c - src) @ dirs.reshape(-1, 3).T
        d2 = np.sum((c - src) ** 2) - t ** 2
        want = 2.0 * np.sqrt(np.maximum(R * R - d2, 0.0))
        assert np.max(np.abs(p[k].ravel() - want)) <= 1e-10


def test_rotated_ellipsoid_chord_quadrature():
    e = Ellipsoid.make((4.0, -6.0, 2.0), (30.0, 18.0, 12.0), 1.0, phi=0.6, tilt=0.4)
    rng = np.random.default_rng(3)
    r = e.rotation()
    for _ in range(5):
        src = np.array([rng.uniform(-5, 5), -400.0, rng.uniform(-5, 5)])
        d = np.array([rng.uniform(-0.02, 0.02), 1.0, rng.uniform(-0.02, 0.02)])
        d /= np.linalg.norm(d)
        chord = float(_chords(src[None], d[None], e)[0])
        ts = np.linspace(300.0, 500.0, 2_000_001)
        pts = src[None] + ts[:, None] * d[None]
        b = ((pts - np.array(e.centre)) @ r) / np.array(e.axes)
        inside = np.sum(b * b, axis=1) <= 1.0
        quad = inside.sum() * (ts[1] - ts[0])
        assert abs(quad - chord) <= 2e-4 * max(chord, 1.0) + 2e-4


def test_phantoms_fit_the_field_of_view():
    g = tiny_geometry()
    vx = voxelise(g, shepp_logan_standin(1000), sub=2)
    assert vx.max() <= 0.02 + 1e-12 and vx.min() >= -1e-12
    assert np.all(vx[~fov_mask(g)] == 0.0)
    gh = head_geometry(40)
    ph = random_head(gh, 1001)
    assert 12 <= len(ph) <= 22
    # exact values in {0, 0.02, 0.04}: sample points
    rng = np.random.default_rng(0)
    pts = rng.uniform(-120, 120, size=(20000, 3))
    val = np.zeros(len(pts))
    for e in ph:
        b = ((pts - np.array(e.centre)) @ e.rotation()) / np.array(e.axes)
        val += e.rho * (np.sum(b * b, axis=1) <= 1.0)
    assert set(np.round(val, 12)).issubset({0.0, 0.02, 0.04})


def test_noise_is_seeded_and_clamped():
    p = np.full((2, 3, 4), 12.0)  # exp(-12)*1e4 ~ 0.06 counts: many zeros
    a = noisy_log_projections(p, 1e4, 5, sigma=5.0)
    b = noisy_log_projections(p, 1e4, 5, sigma=5.0)
    assert np.array_equal(a, b)
    assert a.max() <= math.log(1e4) + 1e-12
