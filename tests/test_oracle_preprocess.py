"""Pins of the oracle's log transform of detector counts (the step before
the method): Beer-Lambert counts I = I0 exp(-p) give back p, an open beam
gives 0, counts below the floor are clamped, and a flat field replaces the
single open-beam count pixel by pixel."""

import numpy as np

import oracle


def test_beer_lambert_counts_give_the_line_integral():
    p = np.linspace(0.0, 6.0, 61)
    i0 = 5e4
    y = oracle.log_counts(i0 * np.exp(-p), i0=i0)
    assert np.max(np.abs(y - p)) <= 1e-12


def test_open_beam_and_floor():
    i0 = 1e4
    y = oracle.log_counts(np.array([i0, 0.0, -3.0, 0.5, 2.0]), i0=i0, min_count=1.0)
    assert y[0] == 0.0
    assert y[1] == y[2] == y[3] == np.log(i0)      # clamped to one count
    assert abs(y[4] - np.log(i0 / 2.0)) <= 1e-15


def test_flat_field_per_pixel():
    rng = np.random.default_rng(3)
    flat = rng.uniform(2e4, 6e4, (4, 5))
    p = rng.uniform(0.0, 3.0, (4, 5))
    y = oracle.log_counts(flat * np.exp(-p), flat=flat)
    assert np.max(np.abs(y - p)) <= 1e-12
