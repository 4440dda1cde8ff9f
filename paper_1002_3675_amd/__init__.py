"""MI355X-native TV-regularised cone-beam CT reconstruction.

Python binding of libcbct.so (include/cbct.h).  Every step of the
reconstruction runs in the library's HIP kernels; this module only
marshals arguments: PyTorch provides device memory and the stream.  There
is no CPU fallback: without the built library, or without a GPU, the
calls raise.

    plan = Plan(geom)                 # geometry -> per-view tables
    y = plan.project(f)               # P f          (float32 / float64)
    f = plan.backproject(y)           # P^T y        (gather, no atomics)
    y = Project.apply(f, plan)        # differentiable P
    f, rep = fbs_solve(plan, Y, FbsParams(mu=1e-3, iters=(20, 20)))

The method is forward-backward splitting for min E1 + mu*E2 s.t. f >= 0
(Eq. (1) and Algorithm A1 of Jia et al., cone-beam CT reconstruction via
total variation).
"""

from __future__ import annotations

import ctypes
import dataclasses
from typing import Optional, Sequence, Tuple, Union

from . import _native
from ._native import CbctError, cbct_fbs_params, cbct_fbs_report, cbct_geom, check

__all__ = ["Geometry", "Plan", "FbsParams", "FbsReport", "FbsState", "fbs_solve",
           "tv_prox", "tv_energy", "Project", "footprint", "CbctError"]


@dataclasses.dataclass(frozen=True)
class Geometry:
    """Scan and grid (mm): see include/cbct.h for the conventions."""
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

    @staticmethod
    def of(g) -> "Geometry":
        """Copy any object with the same attribute names."""
        ang = getattr(g, "angles", None)
        return Geometry(int(g.nx), int(g.ny), int(g.nz), float(g.hx), float(g.hy),
                        float(g.hz), int(g.nu), int(g.nv), float(g.au), float(g.av),
                        float(g.sad), float(g.sdd), int(g.n_views),
                        None if ang is None else tuple(float(a) for a in ang),
                        float(getattr(g, "step", 0.0)),
                        *(float(getattr(g, k, 0.0))
                          for k in ("u_off", "v_off", "x_off", "y_off", "z_off")))

    @property
    def vol_shape(self):
        return (self.nz, self.ny, self.nx)

    @property
    def proj_shape(self):
        return (self.n_views, self.nv, self.nu)


def _to_c(g: Geometry):
    """cbct_geom plus the angle buffer that must outlive the call."""
    ang = None
    c = cbct_geom(g.nx, g.ny, g.nz, g.hx, g.hy, g.hz, g.nu, g.nv, g.au, g.av, g.sad, g.sdd,
                  g.n_views, None, g.step, g.u_off, g.v_off, g.x_off, g.y_off, g.z_off)
    if g.angles is not None:
        ang = (ctypes.c_double * g.n_views)(*g.angles)
        c.angles = ctypes.cast(ang, ctypes.POINTER(ctypes.c_double))
    return c, ang


def _torch():
    import torch
    return torch


def _stream_of(t):
    torch = _torch()
    return ctypes.c_void_p(torch.cuda.current_stream(t.device).cuda_stream)


def _check_tensor(t, shape, dtype, name):
    torch = _torch()
    if not isinstance(t, torch.Tensor) or not t.is_cuda:
        raise TypeError("%s must be a CUDA (HIP) tensor" % name)
    if t.dtype != dtype:
        raise TypeError("%s must be %s, got %s" % (name, dtype, t.dtype))
    if tuple(t.shape) != tuple(shape):
        raise ValueError("%s must have shape %s, got %s" % (name, tuple(shape), tuple(t.shape)))
    if not t.is_contiguous():
        raise ValueError("%s must be contiguous" % name)


def _ptr(t):
    return ctypes.c_void_p(t.data_ptr())


class Plan:
    """A cbct_plan: immutable per-geometry tables on the current device."""

    def __init__(self, geom, device=None):
        torch = _torch()
        self.geom = Geometry.of(geom)
        self.device = torch.device("cuda", torch.cuda.current_device()) if device is None \
            else torch.device(device)
        c, ang = _to_c(self.geom)
        h = ctypes.c_void_p()
        with torch.cuda.device(self.device):
            check(_native.lib().cbct_plan_create(ctypes.byref(c), ctypes.byref(h)),
                  "cbct_plan_create")
        self._h = h
        self._lib = _native.lib()

    def __del__(self):
        h = getattr(self, "_h", None)
        if h is not None and h.value:
            self._lib.cbct_plan_destroy(h)
            self._h = None

    @property
    def handle(self):
        return self._h

    @property
    def samples(self) -> int:
        """Ray samples S taken by one projection."""
        return int(self._lib.cbct_plan_samples(self._h))

    @property
    def step(self) -> float:
        out = cbct_geom()
        check(self._lib.cbct_plan_geom(self._h, ctypes.byref(out)), "cbct_plan_geom")
        return out.step

    def _new(self, shape, dtype):
        torch = _torch()
        return torch.empty(shape, dtype=dtype, device=self.device)

    def project(self, f, out=None):
        """y = P f (float32 or float64)."""
        torch = _torch()
        fn = {torch.float32: self._lib.cbct_project,
              torch.float64: self._lib.cbct_project_f64}.get(f.dtype)
        if fn is None:
            raise TypeError("f must be float32 or float64")
        _check_tensor(f, self.geom.vol_shape, f.dtype, "f")
        y = self._new(self.geom.proj_shape, f.dtype) if out is None else out
        _check_tensor(y, self.geom.proj_shape, f.dtype, "out")
        with torch.cuda.device(self.device):
            check(fn(self._h, _ptr(f), _ptr(y), _stream_of(f)), "cbct_project")
        return y

    def project_residual(self, f, Y, r=None, sumsq=None):
        """r = P f - Y; sumsq (float64 device scalar tensor) gets sum r^2."""
        torch = _torch()
        _check_tensor(f, self.geom.vol_shape, torch.float32, "f")
        _check_tensor(Y, self.geom.proj_shape, torch.float32, "Y")
        r = self._new(self.geom.proj_shape, torch.float32) if r is None else r
        _check_tensor(r, self.geom.proj_shape, torch.float32, "r")
        sp = ctypes.c_void_p(None)
        if sumsq is not None:
            _check_tensor(sumsq, (1,), torch.float64, "sumsq")
            sp = _ptr(sumsq)
        with torch.cuda.device(self.device):
            check(self._lib.cbct_project_residual(self._h, _ptr(f), _ptr(Y), _ptr(r), sp,
                                                  _stream_of(f)), "cbct_project_residual")
        return r

    def backproject(self, y, out=None):
        """f = P^T y (float32 or float64)."""
        torch = _torch()
        fn = {torch.float32: self._lib.cbct_backproject,
              torch.float64: self._lib.cbct_backproject_f64}.get(y.dtype)
        if fn is None:
            raise TypeError("y must be float32 or float64")
        _check_tensor(y, self.geom.proj_shape, y.dtype, "y")
        f = self._new(self.geom.vol_shape, y.dtype) if out is None else out
        _check_tensor(f, self.geom.vol_shape, y.dtype, "out")
        with torch.cuda.device(self.device):
            check(fn(self._h, _ptr(y), _ptr(f), _stream_of(y)), "cbct_backproject")
        return f

    def backproject_eq2(self, y, out=None):
        """The paper's Eq. (2) applied to residuals y, on the transpose's
        scale (float32): the cheap, unmatched approximation of P^T y."""
        torch = _torch()
        _check_tensor(y, self.geom.proj_shape, torch.float32, "y")
        f = self._new(self.geom.vol_shape, torch.float32) if out is None else out
        _check_tensor(f, self.geom.vol_shape, torch.float32, "out")
        with torch.cuda.device(self.device):
            check(self._lib.cbct_backproject_eq2(self._h, _ptr(y), _ptr(f), _stream_of(y)),
                  "cbct_backproject_eq2")
        return f

    def backproject_update(self, r, f, tau, out=None):
        """g = f - tau * P^T r (Step 1 of Algorithm A1)."""
        torch = _torch()
        _check_tensor(r, self.geom.proj_shape, torch.float32, "r")
        _check_tensor(f, self.geom.vol_shape, torch.float32, "f")
        g = self._new(self.geom.vol_shape, torch.float32) if out is None else out
        with torch.cuda.device(self.device):
            check(self._lib.cbct_backproject_update(self._h, _ptr(r), _ptr(f), float(tau),
                                                    _ptr(g), _stream_of(r)),
                  "cbct_backproject_update")
        return g

    def power_lambda(self, n_iter=30) -> float:
        """Largest eigenvalue of P^T P (power iteration, cached)."""
        torch = _torch()
        lam = ctypes.c_double()
        with torch.cuda.device(self.device):
            s = ctypes.c_void_p(torch.cuda.current_stream(self.device).cuda_stream)
            check(self._lib.cbct_plan_lambda(self._h, int(n_iter), ctypes.byref(lam), s),
                  "cbct_plan_lambda")
        return lam.value


def _grid_c(shape, h):
    nz, ny, nx = shape
    return cbct_geom(nx, ny, nz, float(h[0]), float(h[1]), float(h[2]), 1, 1, 1.0, 1.0,
                     2.0, 3.0, 1, None, 0.0)


def tv_prox(g, z0, h, beta, eps, n_inner, step=0.0, nonneg=True, noalloc=False, out=None):
    """Steps 2-3 of Algorithm A1 on the GPU; returns z (a new tensor, or
    `out` filled).  noalloc=True calls cbct_tv_prox_noalloc (no device
    allocation in the library; grids up to 2^24 voxels)."""
    torch = _torch()
    _check_tensor(g, g.shape, torch.float32, "g")
    _check_tensor(z0, g.shape, torch.float32, "z0")
    if out is None:
        z = z0.clone()
    else:
        _check_tensor(out, g.shape, torch.float32, "out")
        z = out
        if z.data_ptr() != z0.data_ptr():
            z.copy_(z0)
    c = _grid_c(g.shape, h)
    name = "cbct_tv_prox_noalloc" if noalloc else "cbct_tv_prox"
    with torch.cuda.device(g.device):
        check(getattr(_native.lib(), name)(ctypes.byref(c), _ptr(g), _ptr(z), float(beta),
                                           float(eps), int(n_inner), float(step),
                                           int(bool(nonneg)), _stream_of(g)), name)
    return z


def tv_energy(f, h, eps=0.0):
    """(E1, E1_eps): voxel means of |Df| and sqrt(|Df|^2 + eps^2)."""
    torch = _torch()
    _check_tensor(f, f.shape, torch.float32, "f")
    c = _grid_c(f.shape, h)
    out = (ctypes.c_double * 2)()
    with torch.cuda.device(f.device):
        check(_native.lib().cbct_tv_energy(ctypes.byref(c), _ptr(f), float(eps), out,
                                           _stream_of(f)), "cbct_tv_energy")
    return out[0], out[1]


@dataclasses.dataclass
class FbsParams:
    """Solver settings (see cbct_fbs_params): E = E1 + mu E2."""
    mu: float = 1e-3
    iters: Sequence[int] = (10,)          # per level, coarse first
    beta: Optional[Sequence[float]] = None  # None / <= 0 -> power-iteration rule
    eps: float = 1e-3
    n_inner: Optional[Sequence[int]] = None  # None / <= 0 -> default rule
    trace_energy: Union[bool, str] = False  # True: E per iteration; "final": E at the end only
    gradient: str = "matched"             # "matched" (P^T) or "eq2" (the paper's Eq. (2))
    tol: float = 0.0                      # > 0: stop a level at this relative change

    def trace_mode(self) -> int:
        """cbct_fbs_params.trace_energy: 0 none, 1 per iteration, 2 final E."""
        if isinstance(self.trace_energy, str):
            if self.trace_energy != "final":
                raise ValueError("trace_energy must be a bool or 'final'")
            return 2
        return int(bool(self.trace_energy))

    def to_c(self):
        n = len(self.iters)
        if not 1 <= n <= _native.MAX_LEVELS:
            raise ValueError("iters must have 1 to %d entries" % _native.MAX_LEVELS)
        p = cbct_fbs_params()
        p.mu = float(self.mu)
        p.n_levels = n
        for l in range(n):
            p.iters[l] = int(self.iters[l])
            p.beta[l] = float(self.beta[l]) if self.beta is not None else 0.0
            p.n_inner[l] = int(self.n_inner[l]) if self.n_inner is not None else 0
        p.eps = float(self.eps)
        p.trace_energy = self.trace_mode()
        if self.gradient not in ("matched", "eq2"):
            raise ValueError("gradient must be 'matched' or 'eq2'")
        p.gradient = 1 if self.gradient == "eq2" else 0
        p.tol = float(self.tol)
        return p


@dataclasses.dataclass
class FbsReport:
    E: float
    E_eps: float
    E1: float
    E2: float
    beta_used: Tuple[float, ...]
    n_inner_used: Tuple[int, ...]
    iters_done: int
    trace: Optional[list] = None          # packed: level_iters[l] + 1 rows per level
    level_iters: Tuple[int, ...] = ()     # outer iterations made per level
    change: Tuple[float, ...] = ()        # last relative change per level (tol > 0)


def _report(rep, n_levels, trace_buf):
    made = tuple(rep.level_iters[:n_levels])
    tr = None
    if trace_buf is not None:
        n_rows = sum(m + 1 for m in made)
        tr = [tuple(trace_buf[4 * i:4 * i + 4]) for i in range(n_rows)]
    return FbsReport(rep.E, rep.E_eps, rep.E1, rep.E2, tuple(rep.beta_used[:n_levels]),
                     tuple(rep.n_inner_used[:n_levels]), rep.iters_done, tr, made,
                     tuple(rep.change[:n_levels]))


def fbs_solve(plan: Plan, Y, params: FbsParams, f0=None):
    """Reconstruct from Y (float32 device tensor [n_views][nv][nu]).
    Returns (f, FbsReport); f starts from f0 (default zeros)."""
    torch = _torch()
    _check_tensor(Y, plan.geom.proj_shape, torch.float32, "Y")
    f = torch.zeros(plan.geom.vol_shape, dtype=torch.float32, device=Y.device) if f0 is None \
        else f0.clone()
    _check_tensor(f, plan.geom.vol_shape, torch.float32, "f0")
    p = params.to_c()
    rep = cbct_fbs_report()
    n_rows = sum(int(i) + 1 for i in params.iters)
    buf = None
    if params.trace_mode() == 1:
        buf = (ctypes.c_double * (4 * n_rows))()
        rep.trace = ctypes.cast(buf, ctypes.POINTER(ctypes.c_double))
    with torch.cuda.device(Y.device):
        check(_native.lib().cbct_fbs_solve(plan.handle, _ptr(Y), _ptr(f), ctypes.byref(p),
                                           ctypes.byref(rep), _stream_of(Y)), "cbct_fbs_solve")
    return f, _report(rep, len(params.iters), buf)


class FbsState:
    """Step API: a solve that advances a few iterations at a time."""

    def __init__(self, plan: Plan, Y, f, params: FbsParams, stream=None):
        torch = _torch()
        _check_tensor(Y, plan.geom.proj_shape, torch.float32, "Y")
        _check_tensor(f, plan.geom.vol_shape, torch.float32, "f")
        self.plan, self.Y, self.f, self.params = plan, Y, f, params
        self.stream = stream
        self._p = params.to_c()
        self._lib = _native.lib()
        h = ctypes.c_void_p()
        with torch.cuda.device(Y.device):
            check(self._lib.cbct_fbs_init(plan.handle, _ptr(Y), _ptr(f), ctypes.byref(self._p),
                                          ctypes.byref(h), self._stream()), "cbct_fbs_init")
        self._h = h

    def _stream(self):
        torch = _torch()
        s = self.stream if self.stream is not None else torch.cuda.current_stream(self.Y.device)
        return ctypes.c_void_p(s.cuda_stream)

    def step(self, n=1):
        torch = _torch()
        with torch.cuda.device(self.Y.device):
            check(self._lib.cbct_fbs_step(self._h, int(n), self._stream()), "cbct_fbs_step")

    @property
    def finished(self) -> bool:
        rc = self._lib.cbct_fbs_finished(self._h)
        if rc < 0:
            check(rc, "cbct_fbs_finished")
        return rc == 1

    def report(self) -> FbsReport:
        rep = cbct_fbs_report()
        check(self._lib.cbct_fbs_report_get(self._h, ctypes.byref(rep)), "cbct_fbs_report_get")
        return _report(rep, len(self.params.iters), None)

    def close(self):
        if getattr(self, "_h", None) is not None and self._h.value:
            self._lib.cbct_fbs_free(self._h)
            self._h = None

    def __del__(self):
        self.close()


def kernel_timing(enable: bool, kernels=None):
    """Start (clearing old records) or stop per-kernel HIP-event timing.
    kernels: names from _native.KERNELS to record (default all); the
    others then run without events."""
    if kernels is None or not enable:
        check(_native.lib().cbct_kernel_timing(int(bool(enable))), "cbct_kernel_timing")
        return
    mask = 0
    for k in kernels:
        mask |= 1 << _native.KERNELS.index(k)
    check(_native.lib().cbct_kernel_timing_select(mask), "cbct_kernel_timing_select")


def kernel_times():
    """{kernel: (launches, total_ms)} recorded since kernel_timing(True)."""
    out = {}
    for i, name in enumerate(_native.KERNELS):
        n = ctypes.c_int64()
        t = ctypes.c_double()
        check(_native.lib().cbct_kernel_timing_read(i, ctypes.byref(n), ctypes.byref(t)),
              "cbct_kernel_timing_read")
        out[name] = (int(n.value), float(t.value))
    return out


def log_counts(counts, i0=None, flat=None, min_count: float = 1.0, out=None):
    """Line integrals from detector counts (float32 device tensors):
    ln(ref / max(counts, min_count)), ref = the flat field or i0."""
    torch = _torch()
    _check_tensor(counts, counts.shape, torch.float32, "counts")
    if flat is not None:
        _check_tensor(flat, counts.shape, torch.float32, "flat")
    elif i0 is None:
        raise ValueError("give i0 or a flat field")
    y = torch.empty_like(counts) if out is None else out
    _check_tensor(y, counts.shape, torch.float32, "out")
    with torch.cuda.device(counts.device):
        check(_native.lib().cbct_log_counts(_ptr(counts), _ptr(flat) if flat is not None else None,
                                            float(i0 or 0.0), float(min_count), _ptr(y),
                                            int(counts.numel()), _stream_of(counts)),
              "cbct_log_counts")
    return y


def kernel_config() -> dict:
    """Tunable sizes of the float kernels (cbct_kernel_config)."""
    buf = (ctypes.c_int32 * 8)()
    n = _native.lib().cbct_kernel_config(buf, 8)
    if n < 0:
        check(n, "cbct_kernel_config")
    names = ("tile_u", "tile_v", "tile_chunk", "tile_lds_floats", "brick_x", "brick_y",
             "brick_z", "table_pixels")
    return {k: int(buf[i]) for i, k in enumerate(names)}


def projector_tile_margin(geom) -> int:
    """Cells by which the projector widens a tile's corner-ray box
    (cbct_projector_tile_margin; host arithmetic)."""
    c, _ang = _to_c(geom)
    out = ctypes.c_int32()
    check(_native.lib().cbct_projector_tile_margin(ctypes.byref(c), ctypes.byref(out)),
          "cbct_projector_tile_margin")
    return int(out.value)


def probe_fma_rate(fp64: bool = False) -> float:
    """Sustained non-packed FMA rate of the current device in TFLOP/s
    (float32, or float64 with fp64=True): the measured ALU ceiling."""
    torch = _torch()
    out = ctypes.c_double()
    check(_native.lib().cbct_probe_fma_rate(int(bool(fp64)), ctypes.byref(out),
                                            ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)),
          "cbct_probe_fma_rate")
    return float(out.value)


def footprint(geom, params: FbsParams) -> int:
    """Device bytes of a solve, including the caller's Y and f."""
    c, ang = _to_c(Geometry.of(geom))
    p = params.to_c()
    return int(_native.lib().cbct_fbs_footprint(ctypes.byref(c), ctypes.byref(p)))


def _make_project_function():
    torch = _torch()

    class Project(torch.autograd.Function):
        """Differentiable cone-beam projection: forward P f, backward P^T g,
        both by the library's kernels (the backward is the hand-written
        gather-form transpose, not autograd of the forward)."""

        @staticmethod
        def forward(ctx, f, plan):
            ctx.plan = plan
            return plan.project(f.contiguous())

        @staticmethod
        def backward(ctx, gy):
            return ctx.plan.backproject(gy.contiguous()), None

    return Project


class _LazyProject:
    _cls = None

    def __getattr__(self, name):
        if _LazyProject._cls is None:
            _LazyProject._cls = _make_project_function()
        return getattr(_LazyProject._cls, name)


Project = _LazyProject()
