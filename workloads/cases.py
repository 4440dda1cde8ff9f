"""Complete seeded reconstruction cases: geometry, phantom, data, settings."""

from __future__ import annotations

import dataclasses
import math
from typing import List, Optional

import numpy as np

from .geometry import Geometry, tiny_geometry, head_geometry, diff_geometry, \
    diff_fd_geometry
from .phantoms import Ellipsoid, analytic_projections, shepp_logan_standin, \
    random_head, voxelise
from .noise import noisy_log_projections


@dataclasses.dataclass
class Case:
    name: str
    geom: Geometry
    phantom: List[Ellipsoid]
    Y: np.ndarray            # (n_views, nv, nu) FP64 measured line integrals
    mu: float
    iters: tuple             # outer iterations per level, coarse first
    eps: float = 1e-3        # TV smoothing (1/mm^2)
    truth: Optional[np.ndarray] = None  # voxelised phantom, filled on demand

    def voxelised(self) -> np.ndarray:
        if self.truth is None:
            self.truth = voxelise(self.geom, self.phantom)
        return self.truth


def make_case(name, geom, phantom, i0, noise_seed, mu, iters, sigma=0.0,
              eps=1e-3) -> Case:
    p = analytic_projections(geom, phantom)
    y = noisy_log_projections(p, i0, noise_seed, sigma)
    return Case(name, geom, phantom, y, mu, tuple(iters), eps)


def tiny_case() -> Case:
    """64^3 @ 2 mm, Shepp-Logan-style stand-in, 16 views, I0 = 1e5, mu = 1e-3,
    one level, 10 iterations."""
    g = tiny_geometry()
    return make_case("tiny", g, shepp_logan_standin(1000), 1e5, 2000, 1e-3, (10,))


def head_case(n_views: int = 40, iters=(20, 20)) -> Case:
    """512x512x70 head, 40 views, I0 = 5e4, mu = 1e-3, two levels of 20."""
    g = head_geometry(n_views)
    return make_case("head%d" % n_views, g, random_head(g, 1001), 5e4, 2001,
                     1e-3, iters)


def lowdose_case(n_views: int, i0: float, mu: float, iters=(30, 30)) -> Case:
    """Low-dose sweep point: 20/30 views, I0 in {1e4, 2.5e4}, electronic
    noise sigma = 5 counts, mu in {5e-4, 1e-3, 2e-3}, 60 iterations."""
    g = head_geometry(n_views)
    return make_case("lowdose_v%d_i%g_mu%g" % (n_views, i0, mu), g,
                     random_head(g, 1001), i0, 2002, mu, iters, sigma=5.0)


def diff_inputs(fd: bool = False, seed: int = 3000):
    """Random positive volume f ~ U(0, 0.02)/mm and data y ~ U(0, 4) for the
    differentiable-projector checks (128^3 case, or the 32^3 FD case)."""
    g = diff_fd_geometry() if fd else diff_geometry()
    rng = np.random.Generator(np.random.PCG64(seed))
    f = rng.uniform(0.0, 0.02, size=g.vol_shape)
    y = rng.uniform(0.0, 4.0, size=g.proj_shape)
    return g, f, y


def fov_mask(g: Geometry) -> np.ndarray:
    """Voxels inside the transaxial field of view seen by every view and the
    axial range seen by every view (boolean, (nz, ny, nx)), for a centred
    detector (u_off = v_off = 0) over a full turn."""
    half_u = g.nu * g.au / 2.0
    fov_r = g.sad * half_u / math.hypot(g.sdd, half_u)
    x = (np.arange(g.nx) - (g.nx - 1) / 2.0) * g.hx + g.x_off
    y = (np.arange(g.ny) - (g.ny - 1) / 2.0) * g.hy + g.y_off
    z = (np.arange(g.nz) - (g.nz - 1) / 2.0) * g.hz + g.z_off
    r = np.sqrt(x[None, :] ** 2 + y[:, None] ** 2)
    half_v = g.nv * g.av / 2.0
    zmax = half_v * (g.sad - r) / g.sdd
    return (r[None] <= fov_r) & (np.abs(z)[:, None, None] <= zmax[None])
