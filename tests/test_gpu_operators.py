"""GPU parity of the projector P and its gather-form transpose P^T against
the FP64 oracle (relative L2 <= 1e-5 in float32), dot tests, determinism,
edge cases and the full head-size geometry on all of its views."""

import dataclasses
import math
import sys

import numpy as np
import pytest

import oracle
from workloads import Geometry, tiny_geometry, head_geometry, diff_geometry

from gpu_util import require_gpu, rel_l2, to_dev, to_np

pytestmark = pytest.mark.gpu

TOL = 1e-5

RAGGED = Geometry(70, 45, 33, 2.1, 2.3, 2.7, 97, 61, 2.4, 2.2, 700.0, 1100.0, 7,
                  angles=(0.05, 0.9, 1.7, 2.6, 3.3, 4.4, 5.9))


def _plan(g):
    import paper_1002_3675_amd as cb
    return cb.Plan(g)


def _log(msg):
    print(msg, flush=True)
    sys.stdout.flush()


@pytest.mark.parametrize("name,g", [("tiny", tiny_geometry()), ("ragged", RAGGED)])
def test_project_matches_oracle(name, g):
    require_gpu()
    _log("project parity %s" % name)
    rng = np.random.default_rng(10)
    f = rng.uniform(0.0, 0.02, g.vol_shape)
    plan = _plan(g)
    y = to_np(plan.project(to_dev(f)))
    want = oracle.project(g, f.astype(np.float32).astype(np.float64))
    assert rel_l2(y, want) <= TOL, rel_l2(y, want)
    assert plan.samples == oracle.count_samples(g) or \
        abs(plan.samples - oracle.count_samples(g)) <= 1e-6 * plan.samples


@pytest.mark.parametrize("name,g", [("tiny", tiny_geometry()), ("ragged", RAGGED)])
def test_backproject_matches_oracle(name, g):
    require_gpu()
    _log("backproject parity %s" % name)
    rng = np.random.default_rng(11)
    y = rng.uniform(0.0, 4.0, g.proj_shape).astype(np.float32).astype(np.float64)
    plan = _plan(g)
    f = to_np(plan.backproject(to_dev(y)))
    want = oracle.backproject(g, y)
    assert rel_l2(f, want) <= TOL, rel_l2(f, want)


# Slices of more than 2^23 voxels (2900 x 2900, 2902^2 padded): offsets of
# the padded volume's planes exceed 24-bit integer products.  "staged":
# voxels large against a pixel's footprint, so the projector stages its
# chunk boxes in LDS; "global": voxels small, so its chunks read the volume
# from memory.
WIDE = {
    "staged": Geometry(2900, 2900, 2, 1.0, 1.0, 1.0, 40, 6, 0.4, 0.4, 2500.0, 3000.0, 2,
                       angles=(0.3, 1.9)),
    "global": Geometry(2900, 2900, 2, 0.1, 0.1, 0.1, 40, 6, 12.8, 0.1, 600.0, 1000.0, 2,
                       angles=(0.3, 1.9)),
}


@pytest.mark.parametrize("name", sorted(WIDE))
def test_wide_slices_match_oracle(name):
    require_gpu()
    g = WIDE[name]
    _log("wide-slice parity %s" % name)
    assert (g.nx + 2) * (g.ny + 2) > 2 ** 23
    if name == "global":
        # lower bound of a piece's box (as in fallback_margins): beyond the LDS box
        import paper_1002_3675_amd as cb
        cfg = cb.kernel_config()
        half = 0.5 * math.sqrt((g.nx * g.hx) ** 2 + (g.ny * g.hy) ** 2 + (g.nz * g.hz) ** 2)
        span_u = cfg["tile_u"] * g.au * (g.sad - half) / g.sdd / g.hx
        depth = cfg["tile_chunk"] * 0.5 * g.hx / math.sqrt(3.0) / g.hx
        assert math.floor(span_u) * (g.nz + 2) * math.floor(depth) > cfg["tile_lds_floats"]
    rng = np.random.default_rng(15)
    f = rng.uniform(0.0, 0.02, g.vol_shape).astype(np.float32).astype(np.float64)
    plan = _plan(g)
    y = to_np(plan.project(to_dev(f)))
    want = oracle.project(g, f)
    assert np.count_nonzero(want) > want.size // 4
    assert rel_l2(y, want) <= TOL, rel_l2(y, want)
    r = rng.uniform(0.0, 4.0, g.proj_shape).astype(np.float32).astype(np.float64)
    b = to_np(plan.backproject(to_dev(r)))
    want_b = oracle.backproject(g, r)
    assert rel_l2(b, want_b) <= TOL, rel_l2(b, want_b)


def test_projector_row_pitch_beyond_the_compiled_ones():
    """The projector's staged loop is compiled for odd LDS row pitches 5 to
    41.  Thin x voxels (0.25 mm) seen across a 16-pixel tile of 1 mm
    footprint, with rays along y, need boxes about 60-75 cells wide in x
    (still inside the LDS box: 4 mm of samples deep, two detector rows),
    which take the generic loop."""
    require_gpu()
    g = Geometry(96, 24, 4, 0.25, 1.0, 1.0, 32, 2, 2.0, 2.0, 100.0, 200.0, 2,
                 angles=(0.0, math.pi))
    rng = np.random.default_rng(14)
    f = rng.uniform(0.0, 0.02, g.vol_shape).astype(np.float32).astype(np.float64)
    y = to_np(_plan(g).project(to_dev(f)))
    want = oracle.project(g, f)
    assert np.count_nonzero(want) > want.size // 2
    assert rel_l2(y, want) <= TOL, rel_l2(y, want)


def test_transpose_samples_a_hair_below_a_cell_face():
    """An odd 3 x 3 detector has a central ray exactly parallel to -y (view
    pi) or -x (view pi/2); with 0.1-voxel steps its in-segment coordinates
    land a hair (below 2^-25) under a cell face, where the weight rounds up
    to exactly 1.  The cell pass's fast membership test rejects those
    samples and its second pass adds them back; without that pass this
    transpose is 3e-3 away from the oracle's."""
    require_gpu()
    g = Geometry(16, 16, 3, 1.0, 1.0, 1.0, 3, 3, 1.0, 1.0, 200.0, 400.0, 8,
                 angles=(math.pi, math.pi / 2) * 4, step=0.1)
    rng = np.random.default_rng(3)
    y = rng.uniform(0.5, 4.0, g.proj_shape).astype(np.float32).astype(np.float64)
    f = to_np(_plan(g).backproject(to_dev(y)))
    want = oracle.backproject(g, y)
    assert rel_l2(f, want) <= TOL, rel_l2(f, want)


def test_backproject_signed_residual():
    """Mixed-sign input (a residual) still meets the tolerance."""
    require_gpu()
    g = tiny_geometry()
    rng = np.random.default_rng(12)
    y = rng.standard_normal(g.proj_shape).astype(np.float32).astype(np.float64)
    f = to_np(_plan(g).backproject(to_dev(y)))
    want = oracle.backproject(g, y)
    assert rel_l2(f, want) <= TOL, rel_l2(f, want)


def test_float32_dot_product():
    require_gpu()
    g = tiny_geometry()
    plan = _plan(g)
    rng = np.random.default_rng(13)
    f = to_dev(rng.uniform(0, 0.02, g.vol_shape))
    y = to_dev(rng.uniform(0, 4, g.proj_shape))
    a = math.fsum((to_np(plan.project(f)) * to_np(y)).ravel())
    b = math.fsum((to_np(f) * to_np(plan.backproject(y))).ravel())
    assert abs(a - b) <= 2e-6 * abs(a), (a, b)


def test_float64_kernels_match_oracle_tightly():
    require_gpu()
    import torch
    g = RAGGED
    plan = _plan(g)
    rng = np.random.default_rng(14)
    f = rng.uniform(0, 0.02, g.vol_shape)
    y = rng.uniform(0, 4, g.proj_shape)
    yp = to_np(plan.project(to_dev(f, torch.float64)))
    assert rel_l2(yp, oracle.project(g, f)) <= 1e-12
    fb = to_np(plan.backproject(to_dev(y, torch.float64)))
    assert rel_l2(fb, oracle.backproject(g, y)) <= 1e-12


def test_deterministic_bitwise():
    require_gpu()
    import torch
    g = tiny_geometry()
    plan = _plan(g)
    rng = np.random.default_rng(15)
    y = to_dev(rng.standard_normal(g.proj_shape))
    f = to_dev(rng.uniform(0, 0.02, g.vol_shape))
    a, b = plan.backproject(y), plan.backproject(y)
    assert torch.equal(a, b)
    assert torch.equal(plan.project(f), plan.project(f))


def test_edge_cases():
    require_gpu()
    import torch
    # zero volume -> zero projections; single view; 1-voxel-thick grid
    g = Geometry(9, 7, 1, 3.0, 3.0, 3.0, 11, 3, 4.0, 4.0, 400.0, 700.0, 1, angles=(0.4,))
    plan = _plan(g)
    assert float(plan.project(torch.zeros(g.vol_shape, device="cuda")).abs().max()) == 0.0
    rng = np.random.default_rng(16)
    f = rng.uniform(0, 1, g.vol_shape)
    assert rel_l2(to_np(plan.project(to_dev(f))), oracle.project(g, f)) <= TOL
    y = rng.uniform(0, 1, g.proj_shape)
    assert rel_l2(to_np(plan.backproject(to_dev(y))), oracle.backproject(g, y)) <= TOL
    # detector that misses the grid entirely: all-zero output, no fault
    g2 = Geometry(8, 8, 8, 1.0, 1.0, 1.0, 4, 4, 1.0, 1.0, 300.0, 500.0, 2, angles=(0.0, 1.0))
    g2 = dataclasses.replace(g2, nv=2, av=400.0)  # both rows far above/below the grid
    p2 = _plan(g2)
    assert float(p2.project(torch.ones(g2.vol_shape, device="cuda")).abs().max()) == 0.0
    assert float(p2.backproject(torch.ones(g2.proj_shape, device="cuda")).abs().max()) == 0.0
    # shape and dtype errors are raised, not run
    with pytest.raises(ValueError):
        plan.project(torch.zeros((1, 2, 3), device="cuda"))
    with pytest.raises(TypeError):
        plan.project(torch.zeros(g.vol_shape, device="cuda", dtype=torch.float16))


def test_head_size_projection_all_views():
    """512x512x70 grid, 512x384 detector, all 40 views (the 45-degree views
    5, 15, 25, 35 included, where the staged boxes are widest): the whole
    projection stack against the oracle, and every view on its own."""
    require_gpu()
    g = head_geometry(40)
    plan = _plan(g)
    rng = np.random.default_rng(17)
    f = rng.uniform(0, 0.02, g.vol_shape).astype(np.float32)
    _log("head projection, 40 views")
    y = to_np(plan.project(to_dev(f)))
    want = oracle.project(g, f.astype(np.float64))
    assert rel_l2(y, want) <= TOL, rel_l2(y, want)
    per_view = [rel_l2(y[k], want[k]) for k in range(g.n_views)]
    assert max(per_view) <= TOL, per_view


def test_head_size_backprojection_all_views():
    """The full 512x512x70 transpose of data on all 40 views against the
    oracle's scatter transpose: the whole volume, and every z plane on its
    own (the first and last included)."""
    require_gpu()
    g = head_geometry(40)
    plan = _plan(g)
    rng = np.random.default_rng(18)
    y = rng.uniform(-1.0, 4.0, g.proj_shape).astype(np.float32)
    _log("head transpose, 40 views")
    f = to_np(plan.backproject(to_dev(y)))
    want = oracle.backproject(g, y.astype(np.float64))
    assert rel_l2(f, want) <= TOL, rel_l2(f, want)
    per_plane = [rel_l2(f[k], want[k]) for k in range(g.nz)]
    assert max(per_plane) <= TOL, per_plane


def test_diff_size_projection_matches_oracle():
    """128^3, 60 views, 256x192 (the differentiation workload)."""
    require_gpu()
    g = diff_geometry()
    plan = _plan(g)
    rng = np.random.default_rng(20)
    f = rng.uniform(0, 0.02, g.vol_shape).astype(np.float32).astype(np.float64)
    y = to_np(plan.project(to_dev(f)))
    assert rel_l2(y, oracle.project(g, f)) <= TOL


def test_thick_slice_serving_size_matches_oracle():
    """256x256x64 at 1 x 1 x 2.5 mm with a 256x192 detector at 1.552 mm (the
    serving mix's middle class), on six views including the diagonals: the
    projector's pieces group into runs of several lengths here, some of
    them unfitting, and the transpose's footprints are narrower than at
    the head size."""
    require_gpu()
    from workloads import serving_geometries
    g0 = serving_geometries()["256x256x64"]
    g = dataclasses.replace(g0, n_views=6,
                            angles=(0.0, math.pi / 4, 1.1, 2.9, 3 * math.pi / 4 + 0.1, 5.0))
    _log("thick-slice parity %dx%dx%d" % (g.nx, g.ny, g.nz))
    plan = _plan(g)
    rng = np.random.default_rng(23)
    f = rng.uniform(0, 0.02, g.vol_shape).astype(np.float32).astype(np.float64)
    y = to_np(plan.project(to_dev(f)))
    assert rel_l2(y, oracle.project(g, f)) <= TOL
    r = rng.uniform(-1, 4, g.proj_shape).astype(np.float32).astype(np.float64)
    b = to_np(plan.backproject(to_dev(r)))
    assert rel_l2(b, oracle.backproject(g, r)) <= TOL


def test_diff_size_transpose_matches_oracle():
    """128^3, 60 views, 256x192 (the differentiation workload)."""
    require_gpu()
    g = diff_geometry()
    plan = _plan(g)
    rng = np.random.default_rng(19)
    y = rng.uniform(0, 4, g.proj_shape).astype(np.float32).astype(np.float64)
    f = to_np(plan.backproject(to_dev(y)))
    assert rel_l2(f, oracle.backproject(g, y)) <= TOL


# Geometries that force each operator's fallback path (the sizes they
# exceed come from the library, cbct_kernel_config; the lower bounds below
# are checked on the host by fallback_margins and by
# tests/test_kernel_config.py).
# P^T: 2 mm voxels seen through 0.2 mm pixels at magnification ~1.4, so a
# full brick's footprint is hundreds of pixels wide and more than ten rows
# tall, far beyond the LDS table: every full brick reads its rays from the
# global ray table.
PT_FALLBACK = Geometry(16, 16, 16, 2.0, 2.0, 2.0, 256, 256, 0.2, 0.2, 300.0, 450.0, 3,
                       angles=(0.3, 1.9, 4.0))
# P: 8 mm pixels over 1 mm voxels, so the rays of one tile fan over the
# whole grid cross-section and no piece's box fits the LDS box: every tap is
# read from the bordered volume in global memory.
P_FALLBACK = Geometry(64, 64, 64, 1.0, 1.0, 1.0, 24, 16, 8.0, 8.0, 300.0, 450.0, 3,
                      angles=(0.2, 2.2, 4.5))


def fallback_margins(cfg):
    """Host lower bounds of (full-brick footprint in pixels over the LDS
    table, projector chunk box in cells over the LDS box) for PT_FALLBACK
    and P_FALLBACK; both must exceed 1 for the fallbacks to be taken."""
    g = PT_FALLBACK
    # nearest and farthest points of the grid from the source
    half = 0.5 * math.sqrt((g.nx * g.hx) ** 2 + (g.ny * g.hy) ** 2)
    m_min = g.sdd / (g.sad + half)
    # a brick of bx x by cells (full bricks: smaller than the grid) spans at
    # least min(bx hx, by hy) perpendicular to any ray in xy, and bz hz in z
    bx, by, bz = cfg["brick_x"], cfg["brick_y"], cfg["brick_z"]
    cols = min(bx * g.hx, by * g.hy) * m_min / g.au
    rows = bz * g.hz * m_min / g.av
    pt = (math.floor(cols) * math.floor(rows)) / cfg["table_pixels"]
    g = P_FALLBACK
    # a tile's rays span tile * pitch * d / sdd at distance d from the
    # source; inside the grid d >= sad - half, and the box is clipped to
    # the bordered grid; a piece (the samples of the smallest box) advances
    # piece * step along the ray, at least piece * step / sqrt(3) along its
    # dominant axis
    half = 0.5 * math.sqrt((g.nx * g.hx) ** 2 + (g.ny * g.hy) ** 2 + (g.nz * g.hz) ** 2)
    d = g.sad - half
    span_u = min(cfg["tile_u"] * g.au * d / g.sdd / g.hx, g.nx + 2)
    span_v = min(cfg["tile_v"] * g.av * d / g.sdd / g.hz, g.nz + 2)
    step = 0.5 * min(g.hx, g.hy, g.hz)
    depth = cfg["tile_chunk"] * step / math.sqrt(3.0) / max(g.hx, g.hy)
    p = (math.floor(span_u) * math.floor(span_v) * math.floor(depth)) / cfg["tile_lds_floats"]
    return pt, p


@pytest.mark.parametrize("name,g", [("pt_fallback", PT_FALLBACK), ("p_fallback", P_FALLBACK)])
def test_fallback_paths_match_oracle(name, g):
    torch = require_gpu()
    _log("fallback parity %s" % name)
    rng = np.random.default_rng(12)
    f = rng.uniform(0.0, 0.02, g.vol_shape)
    y = rng.uniform(-1.0, 4.0, g.proj_shape)
    p = _plan(g)
    got_p = to_np(p.project(to_dev(f)))
    want_p = oracle.project(g, f.astype(np.float32).astype(np.float64))
    assert rel_l2(got_p, want_p) <= TOL, rel_l2(got_p, want_p)
    got_t = to_np(p.backproject(to_dev(y)))
    want_t = oracle.backproject(g, y.astype(np.float32).astype(np.float64))
    assert rel_l2(got_t, want_t) <= TOL, rel_l2(got_t, want_t)
    # the float32 dot test ties the two paths together
    fd, yd = to_dev(f, torch.float64), to_dev(y, torch.float64)
    lhs = float((p.project(fd.float()).double() * yd).sum())
    rhs = float((fd * p.backproject(yd.float()).double()).sum())
    assert abs(lhs - rhs) <= 2e-6 * max(abs(lhs), abs(rhs)), (lhs, rhs)


def test_fma_rate_probe_is_plausible():
    """The measured ALU ceiling the rooflines cite: positive, and not above
    the published vector peaks (157.3 TFLOP/s float32 with packed math,
    78.6 float64)."""
    require_gpu()
    import paper_1002_3675_amd as cb
    f32 = cb.probe_fma_rate(False)
    f64 = cb.probe_fma_rate(True)
    assert 1.0 < f32 <= 157.3 * 1.05, f32
    assert 1.0 < f64 <= 78.6 * 1.05, f64


def test_kernel_timing_records_only_the_selected_kinds():
    """Event timing restricted to the cell pass records its launches only;
    timing every kind records the projector too; the results do not depend
    on timing."""
    torch = require_gpu()
    import paper_1002_3675_amd as cb
    g = tiny_geometry()
    plan = _plan(g)
    rng = np.random.default_rng(24)
    f = to_dev(rng.uniform(0.0, 0.02, g.vol_shape))
    y = to_dev(rng.uniform(0.0, 4.0, g.proj_shape))
    ref_p, ref_t = plan.project(f), plan.backproject(y)
    try:
        cb.kernel_timing(True, kernels=["cells"])
        p1, t1 = plan.project(f), plan.backproject(y)
        torch.cuda.synchronize()
        cb.kernel_timing(False)
        kt = cb.kernel_times()
        assert kt["cells"][0] == 1 and kt["cells"][1] > 0.0
        assert kt["project"][0] == 0 and kt["gather"][0] == 0
        cb.kernel_timing(True)
        plan.project(f)
        plan.backproject(y)
        torch.cuda.synchronize()
        cb.kernel_timing(False)
        kt = cb.kernel_times()
        assert kt["project"][0] == 1 and kt["cells"][0] == 1 and kt["gather"][0] == 1
    finally:
        cb.kernel_timing(False)
    assert torch.equal(p1, ref_p) and torch.equal(t1, ref_t)


def test_transpose_tables_are_prepared_once_and_shared_by_streams():
    """The plan prepares the transpose's geometry tables on its first call
    (here on a side stream) and every later call, on any stream, waits for
    them: results are bitwise those of a fresh plan."""
    torch = require_gpu()
    g = RAGGED
    rng = np.random.default_rng(21)
    y = to_dev(rng.uniform(-1.0, 4.0, g.proj_shape))
    want = _plan(g).backproject(y)
    plan = _plan(g)
    s1, s2 = torch.cuda.Stream(), torch.cuda.Stream()
    s1.wait_stream(torch.cuda.current_stream())
    s2.wait_stream(torch.cuda.current_stream())
    with torch.cuda.stream(s1):
        a = plan.backproject(y)
    with torch.cuda.stream(s2):
        b = plan.backproject(y)
    torch.cuda.synchronize()
    assert torch.equal(a, want) and torch.equal(b, want)
    assert torch.equal(plan.backproject(y), want)
