"""Scan geometries of the synthetic workloads (sizes only, no method arithmetic)."""

from __future__ import annotations

import dataclasses
import math
from typing import Optional, Tuple

import numpy as np


@dataclasses.dataclass(frozen=True)
class Geometry:
    """A circular cone-beam scan of a voxel grid.

    nx, ny, nz / hx, hy, hz: voxel counts and spacings (mm), x fastest.
    nu, nv / au, av: detector pixel counts and pitches (mm), u fastest.
    sad, sdd: source-to-axis and source-to-imager distances (mm).
    n_views: number of projections; angles: optional explicit angles (rad),
    default equally spaced over a full rotation.
    step: ray sample spacing (mm); 0 selects half the smallest voxel spacing.
    u_off, v_off: detector shift in its plane (mm); u_off != 0 is a
    half-fan (offset-detector) scan.
    x_off, y_off, z_off: centre of the voxel grid (mm); 0 puts it on the
    rotation axis, level with the source.
    """

    nx: int
    ny: int
    nz: int
    hx: float
    hy: float
    hz: float
    nu: int
    nv: int
    au: float
    av: float
    sad: float
    sdd: float
    n_views: int
    angles: Optional[Tuple[float, ...]] = None
    step: float = 0.0
    u_off: float = 0.0
    v_off: float = 0.0
    x_off: float = 0.0
    y_off: float = 0.0
    z_off: float = 0.0

    @property
    def vol_shape(self):
        """numpy shape of a volume, (nz, ny, nx)."""
        return (self.nz, self.ny, self.nx)

    @property
    def proj_shape(self):
        """numpy shape of a projection stack, (n_views, nv, nu)."""
        return (self.n_views, self.nv, self.nu)

    @property
    def n_vox(self) -> int:
        return self.nx * self.ny * self.nz

    @property
    def n_meas(self) -> int:
        return self.n_views * self.nu * self.nv

    def with_views(self, n_views: int) -> "Geometry":
        return dataclasses.replace(self, n_views=n_views, angles=None)


def angles_of(g: Geometry) -> np.ndarray:
    """View angles in radians (explicit list, else 2*pi*k/n_views)."""
    if g.angles is not None:
        a = np.asarray(g.angles, dtype=np.float64)
        if a.shape != (g.n_views,):
            raise ValueError("angles must have n_views entries")
        return a
    return 2.0 * math.pi * np.arange(g.n_views, dtype=np.float64) / g.n_views


def tiny_geometry() -> Geometry:
    """64^3 volume at 2 mm, 16 views, 128x96 detector at 1.6 mm."""
    return Geometry(64, 64, 64, 2.0, 2.0, 2.0, 128, 96, 1.6, 1.6,
                    1000.0, 1500.0, 16)


def head_geometry(n_views: int = 40) -> Geometry:
    """The paper's experiment size: 512x512x70 volume, 512x384 imager.

    Voxels 0.88 x 0.88 x 2.5 mm, pixels 0.776 mm, SAD 1000, SDD 1500.
    """
    return Geometry(512, 512, 70, 0.88, 0.88, 2.5, 512, 384, 0.776, 0.776,
                    1000.0, 1500.0, n_views)


def diff_geometry() -> Geometry:
    """128^3 at 1.5 mm, 60 views, 256x192 detector at 1.6 mm."""
    return Geometry(128, 128, 128, 1.5, 1.5, 1.5, 256, 192, 1.6, 1.6,
                    1000.0, 1500.0, 60)


def diff_fd_geometry() -> Geometry:
    """The same object at 32^3 / 6 mm with a 64x48 detector at 6.4 mm."""
    return Geometry(32, 32, 32, 6.0, 6.0, 6.0, 64, 48, 6.4, 6.4,
                    1000.0, 1500.0, 60)


def serving_geometries():
    """The three request volume classes of the serving mix (20 views each;
    callers change the view count with ``with_views``)."""
    return {
        "128^3": diff_geometry().with_views(20),
        "256x256x64": Geometry(256, 256, 64, 1.0, 1.0, 2.5, 256, 192,
                               1.552, 1.552, 1000.0, 1500.0, 20),
        "512x512x70": head_geometry(20),
    }
