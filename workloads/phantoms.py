"""Ellipsoid phantoms, their exact cone-beam line integrals, and voxelisation.

An ellipsoid e has centre c, semi-axes (a, b, c), a rotation R whose columns
are its axes in world coordinates, and an additive density rho (1/mm).  The
attenuation of a phantom is the sum of rho_e times the indicator of e.

The line integral of one ellipsoid along the ray s + t*e (|e| = 1) is its
chord length: with q = diag(1/a,1/b,1/c) R^T (s - c) and
w = diag(1/a,1/b,1/c) R^T e, |q + t w|^2 = 1 has roots whose distance is
2*sqrt(b^2 - alpha*gamma)/alpha, where alpha = w.w, b = q.w, gamma = q.q - 1
(zero when the discriminant is not positive).
"""

from __future__ import annotations

import dataclasses
import math
from typing import List, Sequence

import numpy as np

from .geometry import Geometry, angles_of


@dataclasses.dataclass(frozen=True)
class Ellipsoid:
    centre: tuple
    axes: tuple
    rot: tuple  # 3x3 rotation, row-major nested tuples; columns = body axes
    rho: float

    @staticmethod
    def make(centre, axes, rho, phi=0.0, tilt=0.0):
        """Ellipsoid rotated by phi about z, then tilted by `tilt` about x."""
        cp, sp = math.cos(phi), math.sin(phi)
        ct, st = math.cos(tilt), math.sin(tilt)
        rz = np.array([[cp, -sp, 0.0], [sp, cp, 0.0], [0.0, 0.0, 1.0]])
        rx = np.array([[1.0, 0.0, 0.0], [0.0, ct, -st], [0.0, st, ct]])
        r = rx @ rz
        return Ellipsoid(tuple(float(v) for v in centre),
                         tuple(float(v) for v in axes),
                         tuple(tuple(float(v) for v in row) for row in r),
                         float(rho))

    def rotation(self) -> np.ndarray:
        return np.array(self.rot, dtype=np.float64)


def _chords(src: np.ndarray, dirs: np.ndarray, e: Ellipsoid) -> np.ndarray:
    """Chord length of rays src + t*dirs (dirs unit, shape (..., 3))."""
    r = e.rotation()
    inv_ax = 1.0 / np.asarray(e.axes, dtype=np.float64)
    q = ((src - np.asarray(e.centre)) @ r) * inv_ax
    w = (dirs @ r) * inv_ax
    alpha = np.sum(w * w, axis=-1)
    b = np.sum(q * w, axis=-1)
    gamma = np.sum(q * q, axis=-1) - 1.0
    disc = b * b - alpha * gamma
    out = np.zeros(disc.shape, dtype=np.float64)
    pos = disc > 0.0
    out[pos] = 2.0 * np.sqrt(disc[pos]) / alpha[pos]
    return out


def ray_directions(g: Geometry, theta: float):
    """Source position and unit ray directions (nv, nu, 3) for one view."""
    c, s = math.cos(theta), math.sin(theta)
    src = np.array([g.sad * s, -g.sad * c, 0.0])
    det_c = np.array([-(g.sdd - g.sad) * s, (g.sdd - g.sad) * c, 0.0])
    e_u = np.array([c, s, 0.0])
    e_v = np.array([0.0, 0.0, 1.0])
    u = (np.arange(g.nu) - (g.nu - 1) / 2.0) * g.au + g.u_off
    v = (np.arange(g.nv) - (g.nv - 1) / 2.0) * g.av + g.v_off
    d = det_c[None, None, :] + u[None, :, None] * e_u + v[:, None, None] * e_v
    dirs = d - src
    dirs /= np.linalg.norm(dirs, axis=-1, keepdims=True)
    return src, dirs


def analytic_projections(g: Geometry, phantom: Sequence[Ellipsoid]) -> np.ndarray:
    """Exact line integrals of the phantom, shape (n_views, nv, nu), FP64."""
    out = np.zeros(g.proj_shape, dtype=np.float64)
    for k, th in enumerate(angles_of(g)):
        src, dirs = ray_directions(g, th)
        acc = np.zeros((g.nv, g.nu))
        for e in phantom:
            acc += e.rho * _chords(src[None, None, :], dirs, e)
        out[k] = acc
    return out


def voxelise(g: Geometry, phantom: Sequence[Ellipsoid], sub: int = 0) -> np.ndarray:
    """Phantom averaged over sub^3 points per voxel, shape (nz, ny, nx), FP64.

    sub = 0 picks 4 for volumes up to 128^3 and 2 otherwise.
    """
    if sub <= 0:
        sub = 4 if g.n_vox <= 128 ** 3 else 2
    out = np.zeros(g.vol_shape, dtype=np.float64)
    offs = (np.arange(sub) + 0.5) / sub - 0.5
    cx = (np.arange(g.nx) - (g.nx - 1) / 2.0) * g.hx + g.x_off
    cy = (np.arange(g.ny) - (g.ny - 1) / 2.0) * g.hy + g.y_off
    cz = (np.arange(g.nz) - (g.nz - 1) / 2.0) * g.hz + g.z_off
    for e in phantom:
        r = e.rotation()
        ext = np.abs(r) @ np.asarray(e.axes)  # half-extent of the bounding box
        lo = np.asarray(e.centre) - ext
        hi = np.asarray(e.centre) + ext
        ix = np.nonzero((cx + g.hx / 2 >= lo[0]) & (cx - g.hx / 2 <= hi[0]))[0]
        iy = np.nonzero((cy + g.hy / 2 >= lo[1]) & (cy - g.hy / 2 <= hi[1]))[0]
        iz = np.nonzero((cz + g.hz / 2 >= lo[2]) & (cz - g.hz / 2 <= hi[2]))[0]
        if len(ix) == 0 or len(iy) == 0 or len(iz) == 0:
            continue
        inv_ax = 1.0 / np.asarray(e.axes)
        px = (cx[ix][:, None] + offs[None, :] * g.hx).ravel()
        py = (cy[iy][:, None] + offs[None, :] * g.hy).ravel()
        for kz in iz:
            acc = np.zeros((len(iy), len(ix)))
            for oz in offs:
                pz = cz[kz] + oz * g.hz
                d0 = px[None, :] - e.centre[0]
                d1 = py[:, None] - e.centre[1]
                d2 = pz - e.centre[2]
                b0 = (d0 * r[0, 0] + d1 * r[1, 0] + d2 * r[2, 0]) * inv_ax[0]
                b1 = (d0 * r[0, 1] + d1 * r[1, 1] + d2 * r[2, 1]) * inv_ax[1]
                b2 = (d0 * r[0, 2] + d1 * r[1, 2] + d2 * r[2, 2]) * inv_ax[2]
                inside = (b0 * b0 + b1 * b1 + b2 * b2) <= 1.0
                acc += inside.reshape(len(iy), sub, len(ix), sub).sum(axis=(1, 3))
            out[kz, iy[0]:iy[-1] + 1, ix[0]:ix[-1] + 1] += e.rho * acc / sub ** 3
    return out


def shepp_logan_standin(seed: int = 1000) -> List[Ellipsoid]:
    """A seeded Shepp-Logan-style stand-in (not the published table).

    An outer shell of 0.02/mm, an inner body of 0.016/mm and eight small
    non-overlapping low-contrast inner ellipsoids (+-0.002 or +-0.003/mm);
    everything lies within r <= 58 mm and |z| <= 44 mm, inside the cone-beam
    field of view of the 64^3 / 2 mm / 128x96 detector scan.
    """
    rng = np.random.Generator(np.random.PCG64(seed))
    ph = [Ellipsoid.make((0, 0, 0), (56, 46, 44), 0.02),
          Ellipsoid.make((0, -1, 0), (52, 42, 40), -0.004)]
    placed = []
    while len(placed) < 8:
        ax = rng.uniform(4.0, 12.0, size=3)
        cen = rng.uniform([-36, -28, -26], [36, 28, 26])
        rad = float(ax.max())
        # stay inside the inner body with a margin, and apart from the others
        if (cen[0] / (52 - rad - 2)) ** 2 + (cen[1] / (42 - rad - 2)) ** 2 \
                + (cen[2] / (40 - rad - 2)) ** 2 > 1.0:
            continue
        if any(np.linalg.norm(cen - c2) < rad + r2 + 1.0 for c2, r2 in placed):
            continue
        placed.append((cen, rad))
        rho = float(rng.choice([0.002, -0.002, 0.003, -0.003]))
        ph.append(Ellipsoid.make(cen, ax, rho, phi=float(rng.uniform(0, math.pi)),
                                 tilt=float(rng.uniform(-0.3, 0.3))))
    return ph


def random_ellipsoid_object(g: Geometry, seed: int, n_inner=(10, 20),
                            fill: float = 0.85) -> List[Ellipsoid]:
    """A seeded random-ellipsoid head inside the scan's field of view.

    Skull shell +0.04/mm with a brain of -0.02/mm inside it (net 0.02/mm),
    and 10-20 non-overlapping inner ellipsoids of air (-0.02) or bone (+0.02),
    so every voxel value is exactly one of {0, 0.02, 0.04} (before
    partial-volume averaging).  The object fills `fill` of the smaller of the
    grid half-extent and the transaxial field-of-view radius, and fits the
    axial extent seen by every view.
    """
    rng = np.random.Generator(np.random.PCG64(seed))
    half_u = g.nu * g.au / 2.0
    fov_r = g.sad * half_u / math.hypot(g.sdd, half_u)
    half_x, half_y = g.nx * g.hx / 2.0, g.ny * g.hy / 2.0
    half_z = min(g.nz * g.hz / 2.0, g.nv * g.av / 2.0 * g.sad / g.sdd * (1 - fov_r / g.sad))
    rx = fill * min(half_x, fov_r) * rng.uniform(0.80, 0.86)
    ry = fill * min(half_y, fov_r) * rng.uniform(0.95, 1.0)
    rz = fill * half_z * rng.uniform(0.9, 0.95)
    phi = float(rng.uniform(-0.1, 0.1))
    skull = Ellipsoid.make((0, 0, 0), (rx, ry, rz), 0.04, phi=phi)
    t = min(rx, ry) * 0.08
    bx, by, bz = rx - t, ry - t, rz - t * min(1.0, rz / rx)
    brain = Ellipsoid.make((0, 0, 0), (bx, by, bz), -0.02, phi=phi)
    ph = [skull, brain]
    n = int(rng.integers(n_inner[0], n_inner[1] + 1))
    placed = []
    tries = 0
    while len(placed) < n and tries < 20000:
        tries += 1
        ax = rng.uniform(0.05, 0.22, size=3) * np.array([bx, by, bz])
        cen = rng.uniform(-1, 1, size=3) * np.array([bx, by, bz]) * 0.8
        rad = float(ax.max())
        m = 1.0 + 0.02 * min(bx, by)
        if (cen[0] / max(bx - rad * m, 1e-9)) ** 2 + (cen[1] / max(by - rad * m, 1e-9)) ** 2 \
                + (cen[2] / max(bz - rad * m, 1e-9)) ** 2 > 1.0:
            continue
        if any(np.linalg.norm(cen - c2) < rad + r2 + 0.5 for c2, r2 in placed):
            continue
        placed.append((cen, rad))
        rho = 0.02 if rng.random() < 0.5 else -0.02
        ph.append(Ellipsoid.make(cen, ax, rho, phi=float(rng.uniform(0, math.pi)),
                                 tilt=float(rng.uniform(-0.4, 0.4))))
    return ph


def random_head(g: Geometry, seed: int = 1001) -> List[Ellipsoid]:
    return random_ellipsoid_object(g, seed)
