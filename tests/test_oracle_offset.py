"""Pins of the detector offset (u_off, v_off) in the oracle: moving the
detector by whole pixel pitches is the same as renumbering the pixels, for
the projector and for the Eq. (2) residual lookup, and P stays matched to
its transpose on an offset (half-fan) geometry."""

import dataclasses

import numpy as np

import oracle
from workloads import Geometry

BASE = Geometry(20, 18, 12, 2.0, 2.0, 2.5, 40, 30, 2.0, 2.0, 300.0, 450.0, 3,
                angles=(0.2, 2.0, 4.1))


def test_projector_pixel_shift():
    rng = np.random.default_rng(50)
    f = rng.uniform(0.0, 0.02, BASE.vol_shape)
    p0 = oracle.project(BASE, f)
    g1 = dataclasses.replace(BASE, u_off=2 * BASE.au, v_off=-BASE.av)
    p1 = oracle.project(g1, f)
    # pixel (i, j) of g1 sits where pixel (i + 2, j - 1) of BASE sits
    a, b = p1[:, 1:, :-2], p0[:, :-1, 2:]
    assert np.max(np.abs(a - b)) <= 1e-12 * np.max(np.abs(b))


def test_eq2_pixel_shift():
    rng = np.random.default_rng(51)
    y0 = rng.uniform(-1.0, 1.0, BASE.proj_shape)
    y0[:, :, :3] = 0.0            # columns the shifted detector does not see
    g1 = dataclasses.replace(BASE, u_off=3 * BASE.au)
    y1 = np.zeros_like(y0)
    y1[:, :, :-3] = y0[:, :, 3:]  # the same values at the same places
    a, b = oracle.eq2_backproject(g1, y1), oracle.eq2_backproject(BASE, y0)
    assert np.max(np.abs(a - b)) <= 1e-12 * np.max(np.abs(b))


def test_half_fan_dot_product():
    g = dataclasses.replace(BASE, u_off=0.3 * BASE.nu * BASE.au)
    rng = np.random.default_rng(52)
    f = rng.uniform(0.0, 1.0, g.vol_shape)
    y = rng.uniform(-1.0, 1.0, g.proj_shape)
    lhs = float(np.sum(oracle.project(g, f) * y))
    rhs = float(np.sum(f * oracle.backproject(g, y)))
    assert abs(lhs - rhs) <= 1e-12 * abs(lhs)
