"""Detector noise model for the synthetic scans (the paper's low-mAs regime).

Counts I ~ Poisson(I0 * exp(-p)) plus optional Gaussian electronic noise of
standard deviation sigma counts; the measured line integral is
Y = ln(I0 / max(I, 1)), so zero or negative counts are clamped to one.
"""

from __future__ import annotations

import numpy as np


def noisy_log_projections(p: np.ndarray, i0: float, seed: int,
                          sigma: float = 0.0) -> np.ndarray:
    """Noisy line integrals from exact ones ``p`` (FP64 in, FP64 out)."""
    rng = np.random.Generator(np.random.PCG64(seed))
    counts = rng.poisson(i0 * np.exp(-p)).astype(np.float64)
    if sigma > 0.0:
        counts += rng.normal(0.0, sigma, size=counts.shape)
    return np.log(i0 / np.maximum(counts, 1.0))
