"""Seeded synthetic inputs for cone-beam TV reconstruction.

This package generates inputs only: scan geometries with the sizes of the
paper's experiments (Sec. "digital NCAT phantom": 512x512x70 volume, 512x384
imager, 20-40 views over 360 degrees; CatPhan experiment: low mAs), ellipsoid
phantoms, their exact (analytic) cone-beam line integrals, and detector noise.

It contains none of the reconstruction method's arithmetic: no discrete
projector, no adjoint, no TV, no solver.  Both the HIP library and the FP64
reference take the arrays produced here as plain inputs.

Geometry conventions (shared by every consumer, stated here once):
  * lengths in mm, attenuation in 1/mm; rotation axis z through the isocentre;
  * view k at angle theta_k (default 2*pi*k/n_views); the source sits at
    R(theta)(0, -SAD, 0), the detector centre at R(theta)(0, SDD-SAD, 0), the
    detector u axis is R(theta)(1, 0, 0) and its v axis is z;
  * detector pixel (i, j) centre: u = (i - (nu-1)/2)*au, v = (j - (nv-1)/2)*av;
  * voxel (i, j, k) centre: ((i-(nx-1)/2)hx, (j-(ny-1)/2)hy, (k-(nz-1)/2)hz),
    stored x fastest; projections stored [view][v][u], u fastest.
"""

from .geometry import Geometry, tiny_geometry, head_geometry, diff_geometry, \
    diff_fd_geometry, serving_geometries, angles_of
from .phantoms import Ellipsoid, shepp_logan_standin, random_head, \
    random_ellipsoid_object, analytic_projections, voxelise
from .noise import noisy_log_projections
from .cases import Case, make_case, tiny_case, head_case, lowdose_case, \
    diff_inputs, fov_mask

__all__ = [
    "Geometry", "tiny_geometry", "head_geometry", "diff_geometry",
    "diff_fd_geometry", "serving_geometries", "angles_of", "Ellipsoid",
    "shepp_logan_standin", "random_head", "random_ellipsoid_object",
    "analytic_projections", "voxelise", "noisy_log_projections", "Case",
    "make_case", "tiny_case", "head_case", "lowdose_case", "diff_inputs",
    "fov_mask",
]
