"""The C ABI library loads and exports every symbol include/cbct.h
declares, and the ctypes mirrors of its structs have the C layout
(no compute calls: these run without a GPU)."""

import ctypes
import dataclasses
import os
import re
import subprocess
import tempfile

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "cbct.h")


def _declared():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(cbct_[a-z0-9_]+)\s*\(", text)))


def _built():
    from paper_1002_3675_amd import _native
    if not os.path.exists(_native.LIB_PATH):
        from paper_1002_3675_amd import build
        build.build()
    return _native


def test_every_declared_symbol_is_exported():
    _native = _built()
    names = _declared()
    assert len(names) >= 20
    h = ctypes.CDLL(_native.LIB_PATH)
    for n in names:
        assert hasattr(h, n), n
    # and the Python binding declares a signature for each of them
    assert sorted(_native.SIGNATURES) == names


def test_struct_layout_matches_c():
    _native = _built()
    src = r"""
#include <stddef.h>
#include <stdio.h>
#include "cbct.h"
#define P(s, f) printf(#s "." #f " %zu\n", offsetof(s, f));
int main(void) {
  printf("cbct_geom %zu\n", sizeof(cbct_geom));
  P(cbct_geom, hx) P(cbct_geom, nu) P(cbct_geom, au) P(cbct_geom, n_views)
  P(cbct_geom, angles) P(cbct_geom, step) P(cbct_geom, u_off) P(cbct_geom, v_off)
  P(cbct_geom, x_off) P(cbct_geom, y_off) P(cbct_geom, z_off)
  printf("MAX_LEVELS.value %d\n", CBCT_MAX_LEVELS);
  printf("cbct_fbs_params %zu\n", sizeof(cbct_fbs_params));
  P(cbct_fbs_params, iters) P(cbct_fbs_params, beta) P(cbct_fbs_params, eps)
  P(cbct_fbs_params, n_inner) P(cbct_fbs_params, trace_energy)
  P(cbct_fbs_params, gradient) P(cbct_fbs_params, tol)
  printf("cbct_fbs_report %zu\n", sizeof(cbct_fbs_report));
  P(cbct_fbs_report, beta_used) P(cbct_fbs_report, n_inner_used)
  P(cbct_fbs_report, level_iters) P(cbct_fbs_report, iters_done)
  P(cbct_fbs_report, change) P(cbct_fbs_report, trace)
  return 0;
}
"""
    with tempfile.TemporaryDirectory() as d:
        c = os.path.join(d, "l.c")
        open(c, "w").write(src)
        exe = os.path.join(d, "l")
        subprocess.check_call(["gcc", "-I", os.path.join(ROOT, "include"), c, "-o", exe])
        out = subprocess.check_output([exe]).decode().split("\n")
    want = {}
    for line in out:
        if line.strip():
            k, v = line.split()
            want[k] = int(v)
    S = {"cbct_geom": _native.cbct_geom, "cbct_fbs_params": _native.cbct_fbs_params,
         "cbct_fbs_report": _native.cbct_fbs_report}
    assert want.pop("MAX_LEVELS.value") == _native.MAX_LEVELS
    for k, v in want.items():
        if "." in k:
            s, f = k.split(".")
            assert getattr(S[s], f).offset == v, k
        else:
            assert ctypes.sizeof(S[k]) == v, k


def test_error_strings_without_gpu():
    _native = _built()
    lib = _native.lib()
    assert lib.cbct_strerror(0) == b"success"
    assert lib.cbct_strerror(-1) == b"invalid argument"
    # invalid geometry is rejected before any device call
    g = _native.cbct_geom(0, 1, 1, 1, 1, 1, 1, 1, 1, 1, 10, 20, 1, None, 0)
    h = ctypes.c_void_p()
    assert lib.cbct_plan_create(ctypes.byref(g), ctypes.byref(h)) == _native.CBCT_EINVAL
    assert b"positive" in lib.cbct_last_error()
    g = _native.cbct_geom(8, 8, 8, 1, 1, 1, 4, 4, 1, 1, 20, 10, 1, None, 0)
    assert lib.cbct_plan_create(ctypes.byref(g), ctypes.byref(h)) == _native.CBCT_EINVAL
    assert lib.cbct_fbs_footprint(ctypes.byref(g), None) == 0


def test_kernel_timing_selection_is_host_state():
    """Selecting kernel kinds for event timing touches no device: unknown
    kinds are refused, known masks and stopping are accepted, and reading
    with no records gives zero launches."""
    _native = _built()
    lib = _native.lib()
    assert lib.cbct_kernel_timing_select(1 << len(_native.KERNELS)) == _native.CBCT_EINVAL
    assert lib.cbct_kernel_timing_select(1 << _native.KERNELS.index("cells")) == 0
    assert lib.cbct_kernel_timing_select(0) == 0
    assert lib.cbct_kernel_timing(1) == 0
    assert lib.cbct_kernel_timing(0) == 0
    n, t = ctypes.c_int64(-1), ctypes.c_double(-1.0)
    assert lib.cbct_kernel_timing_read(_native.KERNELS.index("cells"), ctypes.byref(n),
                                       ctypes.byref(t)) == 0
    assert n.value == 0 and t.value == 0.0


def test_representation_limits_are_rejected_before_the_device():
    """The transpose keeps cell indices and segment numbers in 16 bits:
    grids above 32000 voxels per axis, or a step so small that sample
    indices pass 8e6, are refused at plan creation (no GPU needed)."""
    _native = _built()
    lib = _native.lib()
    h = ctypes.c_void_p()
    g = _native.cbct_geom(32001, 1, 1, 0.001, 1, 1, 16, 16, 1, 1, 100, 200, 1, None, 0)
    assert lib.cbct_plan_create(ctypes.byref(g), ctypes.byref(h)) == _native.CBCT_EINVAL
    assert b"32000" in lib.cbct_last_error()
    g = _native.cbct_geom(8, 8, 8, 1, 1, 1, 16, 16, 1, 1, 100, 200, 1, None, 1e-5)
    assert lib.cbct_plan_create(ctypes.byref(g), ctypes.byref(h)) == _native.CBCT_EINVAL
    assert b"step too small" in lib.cbct_last_error()


def test_footprint_is_host_arithmetic():
    import paper_1002_3675_amd as cb
    from workloads import head_geometry
    g = head_geometry(40)
    one = cb.footprint(g, cb.FbsParams(iters=(20,)))
    two = cb.footprint(g, cb.FbsParams(iters=(20, 20)))
    nvox, nmeas = g.n_vox, g.n_meas
    # at least Y, f, g, z, r and the cell workspace of the fine level
    assert one >= 4 * (3 * nvox + 2 * nmeas + 8 * 513 * 513 * 71)
    assert two > one


def test_footprint_counts_the_power_iteration_when_beta_is_estimated():
    import paper_1002_3675_amd as cb
    from workloads import head_geometry
    g = head_geometry(40)
    given = cb.footprint(g, cb.FbsParams(iters=(20, 20), beta=[500.0, 500.0]))
    est = cb.footprint(g, cb.FbsParams(iters=(20, 20)))
    partly = cb.footprint(g, cb.FbsParams(iters=(20, 20), beta=[500.0, 0.0]))
    # the fine level's power iteration: two volumes, a projection stack, the
    # bordered volume and the cell workspace
    extra = 4 * (2 * g.n_vox + g.n_meas + 514 * 514 * 72) + 4 * 8 * 513 * 513 * 71
    assert est - given >= extra
    assert partly == est


def test_solver_parameters_are_checked_on_the_host():
    """Levels, tolerance and shifts are validated before any device call:
    footprint() returns 0 for what init would refuse."""
    import paper_1002_3675_amd as cb
    from workloads import Geometry, head_geometry
    g = head_geometry(40)
    assert cb.footprint(g, cb.FbsParams(iters=(5, 5, 5, 5))) > \
        cb.footprint(g, cb.FbsParams(iters=(5, 5, 5))) > cb.footprint(g, cb.FbsParams(iters=(5, 5)))
    assert cb.footprint(g, cb.FbsParams(iters=(5, 5), tol=1e-3)) > \
        cb.footprint(g, cb.FbsParams(iters=(5, 5)))
    with pytest.raises(ValueError):
        cb.FbsParams(iters=(1, 1, 1, 1, 1)).to_c()
    assert cb.footprint(g, cb.FbsParams(iters=(5, 5), trace_energy="final")) > 0
    bad = cb.FbsParams(iters=(5, 5)).to_c()
    bad.trace_energy = 3
    from paper_1002_3675_amd import _native
    c, _ang = cb._to_c(g)
    assert _native.lib().cbct_fbs_footprint(ctypes.byref(c), ctypes.byref(bad)) == 0
    with pytest.raises(ValueError):
        cb.FbsParams(trace_energy="every").to_c()
    assert cb.footprint(g, cb.FbsParams(iters=(5, 5), tol=-1.0)) == 0
    assert cb.footprint(g, cb.FbsParams(iters=(5, 5), tol=float("nan"))) == 0
    small = Geometry(6, 6, 3, 4.0, 4.0, 4.0, 16, 12, 3.2, 3.2, 1000.0, 1500.0, 4)
    assert cb.footprint(small, cb.FbsParams(iters=(1, 1))) > 0    # 3 -> 1 plane
    assert cb.footprint(small, cb.FbsParams(iters=(1, 1, 1))) == 0  # 1 -> 0 planes
    # a coarser level's zero-bordered grid is wider: it too must lie inside
    # the source orbit (half diagonal 71.4 mm at the fine level, 72.1 coarse)
    tight = Geometry(100, 100, 8, 1.0, 1.0, 1.0, 64, 16, 2.0, 2.0, 72.0, 150.0, 4)
    assert cb.footprint(tight, cb.FbsParams(iters=(1,))) > 0
    assert cb.footprint(tight, cb.FbsParams(iters=(1, 1))) == 0
    # a shifted grid must still lie inside the source orbit
    assert cb.footprint(dataclasses.replace(g, x_off=900.0), cb.FbsParams(iters=(5,))) == 0
    assert cb.footprint(dataclasses.replace(g, z_off=float("inf")), cb.FbsParams(iters=(5,))) == 0
