"""FP64 CPU reference ("oracle") for TV-regularised cone-beam reconstruction.

TEST INFRASTRUCTURE ONLY: imported by the tests, the smoke check and the CPU
baseline leg of the benchmark, never by the reconstruction library.  It shares
no code with the HIP path.  The arithmetic lives in ``oracle.c`` (plain C99 +
OpenMP, double precision); this module builds it with gcc on first use and
wraps it with ctypes.  Inputs are numpy arrays (converted to float64) and a
geometry object with the attributes nx, ny, nz, hx, hy, hz, nu, nv, au, av,
sad, sdd, n_views, angles (None or a sequence), step (<= 0 for half the
smallest voxel spacing) and, optionally, the detector shift u_off, v_off and
the volume centre x_off, y_off, z_off (mm, default 0).

Parity status: every function here is pinned by tests/test_oracle_*.py against
closed forms, brute force or textbook special cases, except the end-to-end
reconstructions against the paper's figures and times, which the paper does
not print ("parity unpinned" for those comparisons).
"""

from __future__ import annotations

import ctypes
import os
import subprocess
import threading

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "oracle.c")
_LIB_PATH = os.path.join(_HERE, "liboracle.so")
_lock = threading.Lock()
_lib = None

_D = ctypes.POINTER(ctypes.c_double)
_I = ctypes.POINTER(ctypes.c_int)


def build(force: bool = False) -> str:
    """Compile oracle.c into liboracle.so (gcc, -O2, OpenMP, no FMA)."""
    if force or not os.path.exists(_LIB_PATH) or \
            os.path.getmtime(_LIB_PATH) < os.path.getmtime(_SRC):
        tmp = _LIB_PATH + ".tmp%d" % os.getpid()
        subprocess.check_call(["gcc", "-std=c99", "-O2", "-fopenmp", "-fPIC",
                               "-shared", "-D_GNU_SOURCE", "-o", tmp, _SRC, "-lm"])
        os.replace(tmp, _LIB_PATH)
    return _LIB_PATH


def _load():
    global _lib
    with _lock:
        if _lib is None:
            build()
            lib = ctypes.CDLL(_LIB_PATH)
            lib.or_project.argtypes = [_I, _D, _D, _D, _D]
            lib.or_backproject.argtypes = [_I, _D, _D, _D, _D]
            lib.or_count_samples.argtypes = [_I, _D, _D]
            lib.or_count_samples.restype = ctypes.c_longlong
            lib.or_grad.argtypes = [_I, _D, _D, _D, _D, _D]
            lib.or_grad_adjoint.argtypes = [_I, _D, _D, _D, _D, _D]
            lib.or_tv.argtypes = [_I, _D, _D, ctypes.c_double]
            lib.or_tv.restype = ctypes.c_double
            lib.or_tv_grad.argtypes = [_I, _D, _D, ctypes.c_double, _D]
            lib.or_prox_step.argtypes = [_D, ctypes.c_double, ctypes.c_double, ctypes.c_double]
            lib.or_prox_step.restype = ctypes.c_double
            lib.or_tv_prox.argtypes = [_I, _D, _D, _D, ctypes.c_double, ctypes.c_double,
                                       ctypes.c_int, ctypes.c_double, ctypes.c_int,
                                       ctypes.c_double, _D]
            lib.or_data_energy.argtypes = [_I, _D, _D, _D, _D, _D]
            lib.or_data_energy.restype = ctypes.c_double
            lib.or_power_lambda.argtypes = [_I, _D, _D, ctypes.c_int]
            lib.or_power_lambda.restype = ctypes.c_double
            lib.or_bin_detector.argtypes = [ctypes.c_int, ctypes.c_int, ctypes.c_int, _D, _D]
            lib.or_restrict.argtypes = [_I, _D, _D]
            lib.or_prolong.argtypes = [_I, _I, _D, _D]
            lib.or_default_inner.argtypes = [_D, ctypes.c_double, ctypes.c_double]
            lib.or_default_inner.restype = ctypes.c_int
            lib.or_fbs_solve.argtypes = [_I, _D, _D, _D, _D, ctypes.c_double, ctypes.c_int,
                                         _I, _D, ctypes.c_double, _I, ctypes.c_double,
                                         ctypes.c_double, ctypes.c_int, ctypes.c_int, _D, _D,
                                         _D, _D]
            lib.or_coarse.argtypes = [_I, _D, _I, _D]
            lib.or_coarse.restype = ctypes.c_int
            lib.or_fbs_solve.restype = ctypes.c_int
            lib.or_eq2_backproject.argtypes = [_I, _D, _D, _D, _D]
            lib.or_threads.argtypes = []
            lib.or_threads.restype = ctypes.c_int
            _lib = lib
    return _lib


def threads() -> int:
    """OpenMP threads the oracle's loops use."""
    return int(_load().or_threads())


def _dp(a):
    return a.ctypes.data_as(_D) if a is not None else None


def _f64(a):
    return np.ascontiguousarray(a, dtype=np.float64)


def _pack(g):
    dims = np.array([g.nx, g.ny, g.nz, g.nu, g.nv, g.n_views], dtype=np.int32)
    par = np.array([g.hx, g.hy, g.hz, g.au, g.av, g.sad, g.sdd, g.step]
                   + [float(getattr(g, k, 0.0))
                      for k in ("u_off", "v_off", "x_off", "y_off", "z_off")], dtype=np.float64)
    ang = None if getattr(g, "angles", None) is None else _f64(g.angles)
    return dims, par, ang


def _vshape(g):
    return (g.nz, g.ny, g.nx)


def _pshape(g):
    return (g.n_views, g.nv, g.nu)


def step_of(g) -> float:
    return g.step if g.step > 0 else 0.5 * min(g.hx, g.hy, g.hz)


def project(g, f):
    """y = P f (FP64)."""
    lib = _load()
    dims, par, ang = _pack(g)
    f = _f64(f).reshape(_vshape(g))
    y = np.empty(_pshape(g))
    lib.or_project(dims.ctypes.data_as(_I), _dp(par), _dp(ang), _dp(f), _dp(y))
    return y


def backproject(g, y):
    """f = P^T y (FP64, scatter form)."""
    lib = _load()
    dims, par, ang = _pack(g)
    y = _f64(y).reshape(_pshape(g))
    f = np.empty(_vshape(g))
    lib.or_backproject(dims.ctypes.data_as(_I), _dp(par), _dp(ang), _dp(y), _dp(f))
    return f


def eq2_backproject(g, y):
    """Eq. (2) of the paper as an operator on residuals y, on the scale of
    the matrix transpose: sum over views of L^3/(L0 l^2) times the bilinear
    interpolant of y at the voxel's imager point, times hx hy hz/(au av)."""
    lib = _load()
    dims, par, ang = _pack(g)
    y = _f64(y).reshape(_pshape(g))
    f = np.empty(_vshape(g))
    lib.or_eq2_backproject(dims.ctypes.data_as(_I), _dp(par), _dp(ang), _dp(y), _dp(f))
    return f


def log_counts(counts, i0=None, flat=None, min_count=1.0):
    """Line integrals from detector counts (the log transform before the
    method): y = ln(I0 / max(I, min_count)), with I0 the open-beam count,
    per pixel from a flat field or one number for all pixels."""
    counts = _f64(counts)
    ref = _f64(flat) if flat is not None else float(i0)
    return np.log(ref / np.maximum(counts, float(min_count)))


def count_samples(g) -> int:
    lib = _load()
    dims, par, ang = _pack(g)
    return int(lib.or_count_samples(dims.ctypes.data_as(_I), _dp(par), _dp(ang)))


def _vd(z):
    nz, ny, nx = z.shape
    return np.array([nx, ny, nz], dtype=np.int32)


def grad(z, h):
    """D z as (gx, gy, gz)."""
    lib = _load()
    z = _f64(z)
    h = _f64(h)
    out = [np.empty_like(z) for _ in range(3)]
    lib.or_grad(_vd(z).ctypes.data_as(_I), _dp(h), _dp(z), *[_dp(o) for o in out])
    return tuple(out)


def grad_adjoint(p, h):
    """D^T (px, py, pz)."""
    lib = _load()
    px, py, pz = (_f64(a) for a in p)
    h = _f64(h)
    out = np.empty_like(px)
    lib.or_grad_adjoint(_vd(px).ctypes.data_as(_I), _dp(h), _dp(px), _dp(py), _dp(pz), _dp(out))
    return out


def tv(z, h, eps=0.0) -> float:
    """E1 = mean_v sqrt(|Dz|_v^2 + eps^2)."""
    lib = _load()
    z = _f64(z)
    h = _f64(h)
    return float(lib.or_tv(_vd(z).ctypes.data_as(_I), _dp(h), _dp(z), eps))


def tv_grad(z, h, eps):
    """D^T (Dz / |Dz|_eps) = N_vox * gradient of the smoothed E1."""
    lib = _load()
    z = _f64(z)
    h = _f64(h)
    out = np.empty_like(z)
    lib.or_tv_grad(_vd(z).ctypes.data_as(_I), _dp(h), _dp(z), eps, _dp(out))
    return out


def prox_step(h, beta, eps, tv_weight=1.0) -> float:
    lib = _load()
    return float(lib.or_prox_step(_dp(_f64(h)), beta, eps, tv_weight))


def default_inner(h, beta, eps) -> int:
    lib = _load()
    return int(lib.or_default_inner(_dp(_f64(h)), beta, eps))


def tv_prox(g_aux, z0, h, beta, eps, n_inner, step=0.0, clip_mode=0,
            tv_weight=1.0, want_phi=False):
    """Steps 2-3 of Algorithm A1 from z0; returns z (and the Phi trace)."""
    lib = _load()
    ga = _f64(g_aux)
    z = _f64(z0).copy()
    h = _f64(h)
    phi = np.empty(n_inner + 1) if want_phi else None
    lib.or_tv_prox(_vd(z).ctypes.data_as(_I), _dp(h), _dp(ga), _dp(z), beta, eps,
                   n_inner, step, clip_mode, tv_weight, _dp(phi))
    return (z, phi) if want_phi else z


def data_energy(g, f, Y):
    """(E2, residual P f - Y)."""
    lib = _load()
    dims, par, ang = _pack(g)
    f = _f64(f).reshape(_vshape(g))
    Y = _f64(Y).reshape(_pshape(g))
    r = np.empty(_pshape(g))
    e2 = lib.or_data_energy(dims.ctypes.data_as(_I), _dp(par), _dp(ang), _dp(f), _dp(Y), _dp(r))
    return float(e2), r


def power_lambda(g, n_iter=30) -> float:
    lib = _load()
    dims, par, ang = _pack(g)
    return float(lib.or_power_lambda(dims.ctypes.data_as(_I), _dp(par), _dp(ang), n_iter))


def beta_rule(g, mu, lam) -> float:
    """beta = 1.1 * mu * (2 N_vox / N_meas) * lambda."""
    nvox = g.nx * g.ny * g.nz
    nmeas = g.n_views * g.nu * g.nv
    return 1.1 * mu * 2.0 * nvox / nmeas * lam


def bin_detector(y):
    lib = _load()
    y = _f64(y)
    nviews, nv, nu = y.shape
    out = np.empty((nviews, nv // 2, nu // 2))
    lib.or_bin_detector(nu, nv, nviews, _dp(y), _dp(out))
    return out


def restrict(f):
    lib = _load()
    f = _f64(f)
    nz, ny, nx = f.shape
    out = np.empty((nz // 2, ny // 2, nx // 2))
    lib.or_restrict(np.array([nx, ny, nz], dtype=np.int32).ctypes.data_as(_I), _dp(f), _dp(out))
    return out


def prolong(fc, fine_shape):
    lib = _load()
    fc = _f64(fc)
    cz, cy, cx = fc.shape
    nz, ny, nx = fine_shape
    out = np.empty(fine_shape)
    lib.or_prolong(np.array([cx, cy, cz], dtype=np.int32).ctypes.data_as(_I),
                   np.array([nx, ny, nz], dtype=np.int32).ctypes.data_as(_I), _dp(fc), _dp(out))
    return out


def coarse_geometry(g):
    """Geometry of the next coarser multigrid level (a plain namespace):
    half the voxels and pixels per axis, spacings, pitches and step doubled,
    cells and pixels at the centres of the blocks they average."""
    import types
    dims, par, _ = _pack(g)
    cd = np.zeros(6, dtype=np.int32)
    cp = np.zeros(13)
    if _load().or_coarse(dims.ctypes.data_as(_I), _dp(par), cd.ctypes.data_as(_I), _dp(cp)):
        raise ValueError("oracle coarse_geometry: a size would fall below 1")
    return types.SimpleNamespace(
        nx=int(cd[0]), ny=int(cd[1]), nz=int(cd[2]), hx=cp[0], hy=cp[1], hz=cp[2],
        nu=int(cd[3]), nv=int(cd[4]), au=cp[3], av=cp[4], sad=cp[5], sdd=cp[6],
        n_views=g.n_views, angles=getattr(g, "angles", None),
        step=cp[7], u_off=cp[8], v_off=cp[9],
        x_off=cp[10], y_off=cp[11], z_off=cp[12])


def fbs_solve(g, Y, mu, iters, f0=None, beta=None, eps=1e-3, n_inner=None,
              tv_weight=1.0, clip_mode=0, trace=False, gradient="matched", tol=0.0):
    """Algorithm A1 with the coarse-to-fine schedule.

    iters: outer iterations per level, coarse first (1 to 4 levels); with
    tol > 0 a level stops after the first iteration whose relative change
    ||f_{k+1} - f_k|| / ||f_{k+1}|| is <= tol, and iters are maxima.
    Returns dict(f, used_beta, used_inner, used_iters, change (last relative
    change per level), report=(E, E_eps, E1, E2), trace (packed rows:
    used_iters[l] + 1 per level)).
    """
    lib = _load()
    dims, par, ang = _pack(g)
    Y = _f64(Y).reshape(_pshape(g))
    f = np.zeros(_vshape(g)) if f0 is None else _f64(f0).reshape(_vshape(g)).copy()
    nl = len(iters)
    it = np.array(iters, dtype=np.int32)
    b = np.zeros(nl) if beta is None else _f64(beta)
    k = np.zeros(nl, dtype=np.int32) if n_inner is None else np.array(n_inner, dtype=np.int32)
    used = np.zeros(3 * nl)
    change = np.zeros(nl)
    tr = np.zeros((int(sum(iters)) + nl, 4)) if trace else None
    rep = np.zeros(4)
    gm = {"matched": 0, "eq2": 1}[gradient]
    rc = lib.or_fbs_solve(dims.ctypes.data_as(_I), _dp(par), _dp(ang), _dp(Y), _dp(f), mu, nl,
                          it.ctypes.data_as(_I), _dp(b), eps, k.ctypes.data_as(_I), tol,
                          tv_weight, clip_mode, gm, _dp(used), _dp(change), _dp(tr), _dp(rep))
    if rc != 0:
        raise ValueError("oracle fbs_solve: invalid arguments")
    made = used[2 * nl:].astype(int)
    if tr is not None:
        tr = tr[:int(made.sum()) + nl]
    return dict(f=f, used_beta=used[:nl].copy(), used_inner=used[nl:2 * nl].astype(int),
                used_iters=made, change=change, report=rep, trace=tr)
