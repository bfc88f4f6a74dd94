"""MI355X (gfx950) absolute-value preconditioned MINRES for complex-shifted
Laplacian systems (Lin, Li & Hon, arXiv:2408.00488).

Thin Python binding of the C ABI in include/csl.h (libcsl.so, built in-tree
by ``python -m paper_2408_00488_amd.build``).  The binding only marshals
arguments: torch tensors provide device memory and the current stream; every
step of the solve runs in the library's HIP kernels.  There is no CPU
fallback: without the built library every call raises.

Vectors are complex128 CUDA tensors of shape ``(n_0, ..., n_{d-1})`` (C
order, last axis contiguous); the coefficient is a float64 CUDA tensor of
the same shape.
"""
from __future__ import annotations

import ctypes
import os
from dataclasses import dataclass

__all__ = [
    "CSLError", "Problem", "Batch", "create_problem", "destroy_problem",
    "apply_A", "apply_Pinv", "minres_solve", "minres_solve_noalloc", "minres_adjoint",
    "batch_create", "batch_solve", "batch_destroy", "CSLSolve", "solve",
    "library_path", "load_library",
]

_HERE = os.path.dirname(os.path.abspath(__file__))
_LIBNAME = "libcsl.so"

STATUS_NAMES = {0: "OK", 1: "ERR_ARG", 2: "ERR_SINGULAR", 3: "ERR_NOT_CONVERGED",
                4: "ERR_BREAKDOWN", 5: "ERR_NONFINITE", 6: "ERR_HIP", 7: "ERR_OOM",
                8: "ERR_TIMEOUT"}


class CSLError(RuntimeError):
    def __init__(self, status: int, message: str, info=None):
        super().__init__(f"{STATUS_NAMES.get(status, status)}: {message}")
        self.status = status
        self.info = info


class _Grid(ctypes.Structure):
    _fields_ = [("dim", ctypes.c_int), ("n", ctypes.c_int * 3),
                ("length", ctypes.c_double * 3)]


class _ProblemOpts(ctypes.Structure):
    _fields_ = [("abar_rule", ctypes.c_int), ("pinv_prec", ctypes.c_int),
                ("abar", ctypes.c_double), ("tile_elems", ctypes.c_int),
                ("dst_engine", ctypes.c_int), ("reserved", ctypes.c_int * 2)]


class _SolveOpts(ctypes.Structure):
    _fields_ = [("tol", ctypes.c_double), ("maxit", ctypes.c_int),
                ("check_true_residual", ctypes.c_int), ("timeout_ms", ctypes.c_int),
                ("reserved", ctypes.c_int * 3)]


class _SolveInfo(ctypes.Structure):
    _fields_ = [("status", ctypes.c_int), ("iters", ctypes.c_int),
                ("relres_est", ctypes.c_double), ("relres_true", ctypes.c_double)]


class _BatchOpts(ctypes.Structure):
    _fields_ = [("tol", ctypes.c_double), ("maxit", ctypes.c_int),
                ("check_true_residual", ctypes.c_int), ("timeout_ms", ctypes.c_int),
                ("grid_size", ctypes.c_int), ("use_graph", ctypes.c_int),
                ("tile_points", ctypes.c_int), ("lds_bytes", ctypes.c_int),
                ("block_threads", ctypes.c_int)]


class _BatchTuning(ctypes.Structure):
    _fields_ = [("tile_points", ctypes.c_int), ("lds_bytes", ctypes.c_int),
                ("grid_size", ctypes.c_int), ("candidates", ctypes.c_int),
                ("ms", ctypes.c_double), ("ms_default", ctypes.c_double),
                ("block_threads", ctypes.c_int), ("tile_elems", ctypes.c_int)]


def _tuning_dict(t: _BatchTuning) -> dict:
    return {"tile_points": t.tile_points, "lds_bytes": t.lds_bytes,
            "grid_size": t.grid_size, "block_threads": t.block_threads,
            "candidates": t.candidates, "ms": t.ms, "ms_default": t.ms_default,
            "tile_elems": t.tile_elems}


_lib = None


def library_path() -> str:
    return os.path.join(_HERE, _LIBNAME)


def load_library():
    """Load libcsl.so (raises if it has not been built)."""
    global _lib
    if _lib is not None:
        return _lib
    path = library_path()
    if not os.path.exists(path):
        raise RuntimeError(f"{path} is missing: build it with "
                           "`python -m paper_2408_00488_amd.build`")
    L = ctypes.CDLL(path)
    vp, dp, ip = ctypes.c_void_p, ctypes.POINTER(ctypes.c_double), ctypes.c_int
    L.create_problem.argtypes = [ctypes.POINTER(_Grid), vp, ctypes.c_double, ctypes.c_double,
                                 ctypes.POINTER(_ProblemOpts), vp, ctypes.POINTER(vp)]
    L.destroy_problem.argtypes = [vp]
    L.problem_info.argtypes = [vp, dp, dp, dp]
    L.problem_dst_engines.argtypes = [vp, ctypes.POINTER(ctypes.c_int)]
    L.problem_set_schedule.argtypes = [vp, ctypes.c_int, ctypes.c_int, ctypes.c_int, ctypes.c_int,
                                       vp]
    L.problem_schedule.argtypes = [vp, ctypes.POINTER(_BatchTuning)]
    L.batch_schedule.argtypes = [vp, ctypes.POINTER(_BatchTuning)]
    L.problem_tune.argtypes = [vp, vp, vp, ctypes.POINTER(_BatchTuning), vp]
    L.apply_A.argtypes = [vp, vp, vp, vp]
    L.apply_Pinv.argtypes = [vp, vp, vp, vp]
    L.minres_solve.argtypes = [vp, vp, vp, ctypes.POINTER(_SolveOpts),
                               ctypes.POINTER(_SolveInfo), vp]
    L.minres_solve_noalloc.argtypes = [ctypes.POINTER(_Grid), vp, ctypes.c_double,
                                       ctypes.c_double, ctypes.POINTER(_ProblemOpts), vp, vp,
                                       ctypes.POINTER(_SolveOpts), ctypes.POINTER(_SolveInfo), vp]
    L.minres_adjoint.argtypes = [vp, vp, vp, vp, vp, vp, vp, ctypes.POINTER(_SolveOpts),
                                 ctypes.POINTER(_SolveInfo), vp]
    L.batch_create.argtypes = [ctypes.POINTER(vp), ip, ctypes.POINTER(_BatchOpts),
                               ctypes.POINTER(vp)]
    L.batch_solve.argtypes = [vp, ctypes.POINTER(vp), ctypes.POINTER(vp),
                              ctypes.POINTER(_SolveInfo), vp]
    L.batch_adjoint.argtypes = [vp, ctypes.POINTER(vp), ctypes.POINTER(vp), ctypes.POINTER(vp),
                                vp, vp, vp, ctypes.POINTER(_SolveOpts),
                                ctypes.POINTER(_SolveInfo), vp]
    L.batch_destroy.argtypes = [vp]
    L.batch_tune.argtypes = [vp, ctypes.POINTER(vp), ctypes.POINTER(vp),
                             ctypes.POINTER(_BatchTuning), vp]
    L.problem_clone.argtypes = [vp, vp, ctypes.POINTER(vp)]
    L.problem_lanczos.argtypes = [vp, dp, dp, ip, ctypes.POINTER(ctypes.c_int), vp]
    L.problem_ritz.argtypes = [vp, dp, ip, ctypes.POINTER(ctypes.c_int), vp]
    L.paradiag_create.argtypes = [ctypes.POINTER(_Grid), vp, ip, ctypes.c_double,
                                  ctypes.c_double, ctypes.POINTER(_ProblemOpts),
                                  ctypes.POINTER(_BatchOpts), vp, ctypes.POINTER(vp)]
    L.paradiag_shift.argtypes = [vp, ip, dp, dp]
    L.paradiag_transform.argtypes = [vp, vp, vp, ip, vp]
    L.paradiag_solve.argtypes = [vp, vp, vp, ctypes.POINTER(_SolveInfo), vp]
    L.paradiag_tune.argtypes = [vp, vp, ctypes.POINTER(_BatchTuning), vp]
    L.paradiag_batch.argtypes = [vp, ctypes.POINTER(vp)]
    L.paradiag_destroy.argtypes = [vp]
    L.csl_last_error.restype = ctypes.c_char_p
    L.csl_version.restype = ctypes.c_int
    for fn in ("create_problem", "destroy_problem", "problem_info", "problem_dst_engines",
               "problem_set_schedule", "problem_tune", "problem_schedule", "batch_schedule",
               "apply_A", "apply_Pinv",
               "minres_solve", "minres_adjoint", "batch_create", "batch_solve",
               "batch_tune", "batch_destroy", "problem_clone", "problem_lanczos", "problem_ritz",
               "paradiag_create", "paradiag_shift",
               "paradiag_transform", "paradiag_solve", "paradiag_tune", "paradiag_batch",
               "paradiag_destroy"):
        getattr(L, fn).restype = ctypes.c_int
    _lib = L
    return L


def _check(status: int, info=None):
    if status != 0:
        msg = load_library().csl_last_error().decode(errors="replace")
        raise CSLError(status, msg, info)


def _torch():
    import torch
    return torch


def _stream(device=None):
    torch = _torch()
    return ctypes.c_void_p(torch.cuda.current_stream(device).cuda_stream)


def _ptr(t):
    return ctypes.c_void_p(t.data_ptr())


def _info_dict(i: _SolveInfo) -> dict:
    return {"status": i.status, "status_name": STATUS_NAMES.get(i.status, str(i.status)),
            "iters": i.iters, "relres_est": i.relres_est, "relres_true": i.relres_true}


_ABAR = {"mean": 0, "geomean": 1, "given": 2}
_DST = {"auto": 0, "fft": 1, "gemm": 2, "gemm16": 3}
_DST_NAMES = {1: "fft", 2: "gemm", 3: "gemm16"}


class Problem:
    """Handle of one complex-shifted system (K + lambda I) z = f on a grid
    with nodal coefficient ``a`` (float64 CUDA tensor, 2-D or 3-D)."""

    def __init__(self, a, alpha: float, beta: float, lengths=None,
                 abar_rule: str = "mean", abar: float | None = None,
                 pinv_fp32: bool = False, tile_elems: int = 0, dst: str = "auto"):
        torch = _torch()
        L = load_library()
        if not (isinstance(a, torch.Tensor) and a.is_cuda and a.dtype == torch.float64):
            raise TypeError("a must be a float64 CUDA tensor")
        if a.dim() not in (2, 3):
            raise ValueError("a must be 2-D or 3-D")
        self.a = a.contiguous()
        self.shape = tuple(self.a.shape)
        self.device = self.a.device
        self.alpha = float(alpha)
        self.beta = float(beta)
        self.pinv_fp32 = bool(pinv_fp32)
        g = _Grid()
        g.dim = self.a.dim()
        for k in range(3):
            g.n[k] = self.shape[k] if k < g.dim else 0
            g.length[k] = float(lengths[k]) if (lengths is not None and k < g.dim) else 1.0
        o = _ProblemOpts()
        o.abar_rule = _ABAR[abar_rule]
        o.pinv_prec = 1 if pinv_fp32 else 0
        o.abar = float(abar) if abar is not None else 0.0
        o.tile_elems = int(tile_elems)
        o.dst_engine = _DST[dst]
        h = ctypes.c_void_p()
        with torch.cuda.device(self.device):
            _check(L.create_problem(ctypes.byref(g), _ptr(self.a), self.alpha, self.beta,
                                    ctypes.byref(o), _stream(self.device), ctypes.byref(h)))
        self._h = h
        ab, mn, mx = ctypes.c_double(), ctypes.c_double(), ctypes.c_double()
        _check(L.problem_info(h, ctypes.byref(ab), ctypes.byref(mn), ctypes.byref(mx)))
        self.abar, self.a_min, self.a_max = ab.value, mn.value, mx.value
        self._dim = g.dim
        self._read_engines()

    def _read_engines(self):
        eng = (ctypes.c_int * 3)()
        _check(load_library().problem_dst_engines(self._h, eng))
        #: sine-transform engine per axis: "fft" or "gemm"
        self.dst_engines = tuple(_DST_NAMES[eng[k]] for k in range(self._dim))

    @property
    def handle(self):
        if self._h is None:
            raise RuntimeError("problem destroyed")
        return self._h

    def clone(self) -> "Problem":
        """A problem with the same set-up and workspaces of its own (see
        problem_clone): batch it with this one to solve several right-hand
        sides of the same shifted system in one launch."""
        torch = _torch()
        h = ctypes.c_void_p()
        with torch.cuda.device(self.device):
            _check(load_library().problem_clone(self.handle, _stream(self.device), ctypes.byref(h)))
        q = Problem.__new__(Problem)
        q.__dict__.update({k: v for k, v in self.__dict__.items() if k != "_h"})
        q._h = h
        return q

    def set_schedule(self, tile_points: int = 0, lds_bytes: int = 0, block_threads: int = 0,
                     tile_elems: int = 0):
        """Schedule of this problem's own solves (see problem_set_schedule)."""
        _check(load_library().problem_set_schedule(self.handle, int(tile_points), int(lds_bytes),
                                                   int(block_threads), int(tile_elems),
                                                   _stream(self.device)))

    @property
    def schedule(self) -> dict:
        """Schedule in use for this problem's own solves."""
        t = _BatchTuning()
        _check(load_library().problem_schedule(self.handle, ctypes.byref(t)))
        return _tuning_dict(t)

    def lanczos(self):
        """(delta, gamma) of the last completed solve as float64 NumPy arrays
        (see problem_lanczos)."""
        import numpy as np
        L = load_library()
        k = ctypes.c_int()
        _check(L.problem_lanczos(self.handle, None, None, 0, ctypes.byref(k), _stream(self.device)))
        d = np.empty(k.value)
        g = np.empty(k.value)
        dp = ctypes.POINTER(ctypes.c_double)
        _check(L.problem_lanczos(self.handle, d.ctypes.data_as(dp), g.ctypes.data_as(dp), k.value,
                                 ctypes.byref(k), _stream(self.device)))
        return d, g

    def ritz_values(self):
        """Ritz values of P^{-1} A from the last completed solve, ascending
        (see problem_ritz)."""
        import numpy as np
        L = load_library()
        k = ctypes.c_int()
        _check(L.problem_ritz(self.handle, None, 0, ctypes.byref(k), _stream(self.device)))
        th = np.empty(k.value)
        _check(L.problem_ritz(self.handle, th.ctypes.data_as(ctypes.POINTER(ctypes.c_double)),
                              k.value, ctypes.byref(k), _stream(self.device)))
        return th

    def tune(self, f, z=None) -> dict:
        """Time candidate schedules of minres_solve on f and keep the fastest."""
        torch = _torch()
        self._vec(f, "f")
        if z is None:
            z = torch.empty_like(f)
        self._vec(z, "z")
        t = _BatchTuning()
        _check(load_library().problem_tune(self.handle, _ptr(f), _ptr(z), ctypes.byref(t),
                                           _stream(self.device)))
        self._read_engines()   # the tuner may move a matrix-core axis to the FFT
        return _tuning_dict(t)

    def close(self):
        if getattr(self, "_h", None) is not None:
            load_library().destroy_problem(self._h)
            self._h = None

    def __del__(self):  # pragma: no cover - best effort
        try:
            self.close()
        except Exception:
            pass

    def _vec(self, x, name):
        torch = _torch()
        if not (isinstance(x, torch.Tensor) and x.is_cuda and x.dtype == torch.complex128):
            raise TypeError(f"{name} must be a complex128 CUDA tensor")
        if tuple(x.shape) != self.shape:
            raise ValueError(f"{name} has shape {tuple(x.shape)}, expected {self.shape}")
        if not x.is_contiguous():
            raise ValueError(f"{name} must be contiguous")
        return x


def create_problem(a, alpha, beta, **kw) -> Problem:
    return Problem(a, alpha, beta, **kw)


def destroy_problem(p: Problem):
    p.close()


def apply_A(p: Problem, x, y=None):
    """y = A x (block form; complex storage y = (K + lambda I) conj(x))."""
    torch = _torch()
    p._vec(x, "x")
    if y is None:
        y = torch.empty_like(x)
    p._vec(y, "y")
    _check(load_library().apply_A(p.handle, _ptr(x), _ptr(y), _stream(p.device)))
    return y


def apply_Pinv(p: Problem, x, y=None):
    """y = P^{-1} x through the sine transforms."""
    torch = _torch()
    p._vec(x, "x")
    if y is None:
        y = torch.empty_like(x)
    p._vec(y, "y")
    _check(load_library().apply_Pinv(p.handle, _ptr(x), _ptr(y), _stream(p.device)))
    return y


def _solve_opts(tol, maxit, check_true, timeout_ms):
    o = _SolveOpts()
    o.tol = float(tol)
    o.maxit = int(maxit)
    o.check_true_residual = 1 if check_true else 0
    o.timeout_ms = int(timeout_ms)
    return o


def minres_solve(p: Problem, f, z=None, tol=1e-8, maxit=1000, check_true=True,
                 timeout_ms=0, want_info=True, raise_on_error=True):
    """Solve (K + lambda I) z = f.  Returns (z, info dict or None)."""
    torch = _torch()
    p._vec(f, "f")
    if z is None:
        z = torch.empty_like(f)
    p._vec(z, "z")
    o = _solve_opts(tol, maxit, check_true, timeout_ms)
    info = _SolveInfo()
    st = load_library().minres_solve(p.handle, _ptr(f), _ptr(z), ctypes.byref(o),
                                     ctypes.byref(info) if want_info else None,
                                     _stream(p.device))
    d = _info_dict(info) if want_info else None
    if raise_on_error and st != 0:
        _check(st, d)
    return z, d


def minres_solve_noalloc(a, alpha: float, beta: float, f, z=None, lengths=None,
                         abar_rule: str = "mean", abar: float | None = None,
                         pinv_fp32: bool = False, tol=1e-8, maxit=1000, check_true=True,
                         timeout_ms=0, want_info=True, raise_on_error=True):
    """Solve (K + lambda I) z = f once without a problem handle, through the
    library's allocation-free entry point (its workspace is a static device
    array; n + 1 a power of two on every axis).  Returns (z, info or None)."""
    torch = _torch()
    if not (isinstance(a, torch.Tensor) and a.is_cuda and a.dtype == torch.float64):
        raise TypeError("a must be a float64 CUDA tensor")
    if a.dim() not in (2, 3) or not a.is_contiguous():
        raise ValueError("a must be a contiguous 2-D or 3-D tensor")
    shape = tuple(a.shape)
    for name, v in (("f", f), ("z", z)):
        if v is None:
            continue
        if not (isinstance(v, torch.Tensor) and v.is_cuda and v.dtype == torch.complex128
                and tuple(v.shape) == shape and v.is_contiguous() and v.device == a.device):
            raise ValueError(f"{name} must be a contiguous complex128 CUDA tensor of shape "
                             f"{shape} on {a.device}")
    if z is None:
        z = torch.empty_like(f)
    g = _Grid()
    g.dim = a.dim()
    for k in range(3):
        g.n[k] = shape[k] if k < g.dim else 0
        g.length[k] = float(lengths[k]) if (lengths is not None and k < g.dim) else 1.0
    po = _ProblemOpts()
    po.abar_rule = _ABAR[abar_rule]
    po.pinv_prec = 1 if pinv_fp32 else 0
    po.abar = float(abar) if abar is not None else 0.0
    po.dst_engine = _DST["fft"]
    o = _solve_opts(tol, maxit, check_true, timeout_ms)
    info = _SolveInfo()
    with torch.cuda.device(a.device):
        st = load_library().minres_solve_noalloc(
            ctypes.byref(g), _ptr(a), float(alpha), float(beta), ctypes.byref(po), _ptr(f),
            _ptr(z), ctypes.byref(o), ctypes.byref(info) if want_info else None,
            _stream(a.device))
    d = _info_dict(info) if want_info else None
    if raise_on_error and st != 0:
        _check(st, d)
    return z, d


def minres_adjoint(p: Problem, z, gz, tol=1e-8, maxit=1000, check_true=True,
                   timeout_ms=0, ga=None, raise_on_error=True):
    """Adjoint solve: returns (grads, info) with grads = dict(f=..., alpha=...,
    beta=..., a=...) (alpha/beta as 0-dim CUDA tensors; a accumulated into
    ``ga`` if given, else a fresh zero tensor)."""
    torch = _torch()
    p._vec(z, "z")
    p._vec(gz, "gz")
    gf = torch.empty_like(gz)
    gab = torch.zeros(2, dtype=torch.float64, device=p.device)
    if ga is None:
        ga = torch.zeros(p.shape, dtype=torch.float64, device=p.device)
    o = _solve_opts(tol, maxit, check_true, timeout_ms)
    info = _SolveInfo()
    st = load_library().minres_adjoint(
        p.handle, _ptr(z), _ptr(gz), _ptr(gf), ctypes.c_void_p(gab.data_ptr()),
        ctypes.c_void_p(gab.data_ptr() + 8), _ptr(ga), ctypes.byref(o), ctypes.byref(info),
        _stream(p.device))
    d = _info_dict(info)
    if raise_on_error and st != 0:
        _check(st, d)
    return {"f": gf, "alpha": gab[0], "beta": gab[1], "a": ga}, d


class Batch:
    """Several problems solved by one persistent launch (optionally a graph)."""

    def __init__(self, problems, tol=1e-8, maxit=1000, check_true=True, timeout_ms=0,
                 grid_size=0, use_graph=True, tile_points=0, lds_bytes=0, block_threads=0):
        self.problems = list(problems)
        arr = (ctypes.c_void_p * len(self.problems))(*[p.handle for p in self.problems])
        o = _BatchOpts()
        o.tol = float(tol)
        o.maxit = int(maxit)
        o.check_true_residual = 1 if check_true else 0
        o.timeout_ms = int(timeout_ms)
        o.grid_size = int(grid_size)
        o.use_graph = 1 if use_graph else 0
        o.tile_points = int(tile_points)
        o.lds_bytes = int(lds_bytes)
        o.block_threads = int(block_threads)
        h = ctypes.c_void_p()
        _check(load_library().batch_create(arr, len(self.problems), ctypes.byref(o),
                                           ctypes.byref(h)))
        self._h = h
        self.device = self.problems[0].device

    def close(self):
        if getattr(self, "_h", None) is not None:
            load_library().batch_destroy(self._h)
            self._h = None

    def __del__(self):  # pragma: no cover
        try:
            self.close()
        except Exception:
            pass

    def solve(self, fs, zs=None, want_info=True, raise_on_error=True):
        torch = _torch()
        n = len(self.problems)
        if len(fs) != n:
            raise ValueError("need one right-hand side per system")
        if zs is None:
            zs = [torch.empty_like(f) for f in fs]
        for p, f, z in zip(self.problems, fs, zs):
            p._vec(f, "f")
            p._vec(z, "z")
        fa = (ctypes.c_void_p * n)(*[f.data_ptr() for f in fs])
        za = (ctypes.c_void_p * n)(*[z.data_ptr() for z in zs])
        infos = (_SolveInfo * n)()
        st = load_library().batch_solve(self._h, fa, za, infos if want_info else None,
                                        _stream(self.device))
        d = [_info_dict(i) for i in infos] if want_info else None
        if raise_on_error and st != 0:
            _check(st, d)
        return zs, d

    def adjoint(self, zs, gzs, ga=None, tol=1e-8, maxit=1000, check_true=True, timeout_ms=0,
                want_info=True, raise_on_error=True):
        """Adjoint of every system at once (batch_adjoint): zs the forward
        solutions, gzs = dL/dRe z + i dL/dIm z per system.  Returns (grads,
        infos) with grads = dict(f=[per system], alpha=tensor(count),
        beta=tensor(count), a=ga): the coefficient gradient summed over the
        systems (accumulated into ``ga`` if given, else a fresh zero tensor;
        every system must be on one grid)."""
        torch = _torch()
        n = len(self.problems)
        if len(zs) != n or len(gzs) != n:
            raise ValueError("need one solution and one loss gradient per system")
        for p, z, gz in zip(self.problems, zs, gzs):
            p._vec(z, "z")
            p._vec(gz, "gz")
        gfs = [torch.empty_like(gz) for gz in gzs]
        gab = torch.zeros((2, n), dtype=torch.float64, device=self.device)
        if ga is None:
            ga = torch.zeros(self.problems[0].shape, dtype=torch.float64, device=self.device)
        elif not (isinstance(ga, torch.Tensor) and ga.dtype == torch.float64 and ga.is_contiguous()
                  and tuple(ga.shape) == self.problems[0].shape and ga.device == self.device):
            raise ValueError("ga must be a contiguous float64 tensor of the grid's shape")
        za = (ctypes.c_void_p * n)(*[z.data_ptr() for z in zs])
        ga_arr = (ctypes.c_void_p * n)(*[g.data_ptr() for g in gzs])
        fa = (ctypes.c_void_p * n)(*[g.data_ptr() for g in gfs])
        o = _solve_opts(tol, maxit, check_true, timeout_ms)
        infos = (_SolveInfo * n)()
        st = load_library().batch_adjoint(
            self._h, za, ga_arr, fa, ctypes.c_void_p(gab.data_ptr()),
            ctypes.c_void_p(gab.data_ptr() + 8 * n), _ptr(ga), ctypes.byref(o),
            infos if want_info else None, _stream(self.device))
        d = [_info_dict(i) for i in infos] if want_info else None
        if raise_on_error and st != 0:
            _check(st, d)
        return {"f": gfs, "alpha": gab[0], "beta": gab[1], "a": ga}, d

    def tune(self, fs, zs=None) -> dict:
        """Time the candidate schedules on these right-hand sides and keep
        the fastest (see batch_tune); returns the chosen schedule."""
        torch = _torch()
        n = len(self.problems)
        if len(fs) != n:
            raise ValueError("need one right-hand side per system")
        if zs is None:
            zs = [torch.empty_like(f) for f in fs]
        for p, f, z in zip(self.problems, fs, zs):
            p._vec(f, "f")
            p._vec(z, "z")
        fa = (ctypes.c_void_p * n)(*[f.data_ptr() for f in fs])
        za = (ctypes.c_void_p * n)(*[z.data_ptr() for z in zs])
        t = _BatchTuning()
        _check(load_library().batch_tune(self._h, fa, za, ctypes.byref(t),
                                         _stream(self.device)))
        return _tuning_dict(t)

    @property
    def schedule(self) -> dict:
        """Schedule in use for this batch."""
        t = _BatchTuning()
        _check(load_library().batch_schedule(self._h, ctypes.byref(t)))
        return _tuning_dict(t)


class ParaDiag:
    """All-at-once solve of implicit Euler (step tau, L steps) for u' + K u = g
    with the alpha-circulant time factor: u = (kron(C, I) + kron(I, K))^-1 r
    through the step transform and one batched solve of the L shifted
    systems (see paradiag_create).  All-at-once vectors are complex128 CUDA
    tensors of shape (L,) + grid shape."""

    def __init__(self, a, steps: int, tau: float, alpha_c: float, lengths=None,
                 abar_rule: str = "mean", pinv_fp32: bool = False, dst: str = "auto",
                 tol=1e-8, maxit=1000, check_true=True, timeout_ms=0, use_graph=True,
                 tile_points=0, lds_bytes=0, block_threads=0):
        torch = _torch()
        if not (isinstance(a, torch.Tensor) and a.is_cuda and a.dtype == torch.float64):
            raise TypeError("a must be a float64 CUDA tensor")
        if a.dim() not in (2, 3):
            raise ValueError("a must be 2-D or 3-D")
        self.a = a.contiguous()
        self.shape = tuple(self.a.shape)
        self.device = self.a.device
        self.steps = int(steps)
        g = _Grid()
        g.dim = self.a.dim()
        for k in range(3):
            g.n[k] = self.shape[k] if k < g.dim else 0
            g.length[k] = float(lengths[k]) if (lengths is not None and k < g.dim) else 1.0
        po = _ProblemOpts()
        po.abar_rule = _ABAR[abar_rule]
        po.pinv_prec = 1 if pinv_fp32 else 0
        po.dst_engine = _DST[dst]
        bo = _BatchOpts()
        bo.tol = float(tol)
        bo.maxit = int(maxit)
        bo.check_true_residual = 1 if check_true else 0
        bo.timeout_ms = int(timeout_ms)
        bo.use_graph = 1 if use_graph else 0
        bo.tile_points = int(tile_points)
        bo.lds_bytes = int(lds_bytes)
        bo.block_threads = int(block_threads)
        h = ctypes.c_void_p()
        with torch.cuda.device(self.device):
            _check(load_library().paradiag_create(
                ctypes.byref(g), _ptr(self.a), self.steps, float(tau), float(alpha_c),
                ctypes.byref(po), ctypes.byref(bo), _stream(self.device), ctypes.byref(h)))
        self._h = h

    def close(self):
        if getattr(self, "_h", None) is not None:
            load_library().paradiag_destroy(self._h)
            self._h = None

    def __del__(self):  # pragma: no cover
        try:
            self.close()
        except Exception:
            pass

    def _vec(self, x, name):
        torch = _torch()
        if not (isinstance(x, torch.Tensor) and x.is_cuda and x.dtype == torch.complex128
                and x.is_contiguous() and x.device == self.device
                and tuple(x.shape) == (self.steps,) + self.shape):
            raise ValueError(f"{name} must be a contiguous complex128 CUDA tensor of shape "
                             f"{(self.steps,) + self.shape} on {self.device}")

    @property
    def shifts(self) -> list:
        out = []
        for j in range(self.steps):
            re, im = ctypes.c_double(), ctypes.c_double()
            _check(load_library().paradiag_shift(self._h, j, ctypes.byref(re), ctypes.byref(im)))
            out.append(complex(re.value, im.value))
        return out

    def transform(self, x, y=None, inverse=False):
        torch = _torch()
        self._vec(x, "x")
        if y is None:
            y = torch.empty_like(x)
        self._vec(y, "y")
        _check(load_library().paradiag_transform(self._h, _ptr(x), _ptr(y), 1 if inverse else 0,
                                                 _stream(self.device)))
        return y

    def solve(self, r, u=None, want_info=True, raise_on_error=True):
        torch = _torch()
        self._vec(r, "r")
        if u is None:
            u = torch.empty_like(r)
        self._vec(u, "u")
        infos = (_SolveInfo * self.steps)()
        st = load_library().paradiag_solve(self._h, _ptr(r), _ptr(u),
                                           infos if want_info else None, _stream(self.device))
        d = [_info_dict(i) for i in infos] if want_info else None
        if raise_on_error and st != 0:
            _check(st, d)
        return u, d

    def tune(self, r) -> dict:
        self._vec(r, "r")
        t = _BatchTuning()
        _check(load_library().paradiag_tune(self._h, _ptr(r), ctypes.byref(t),
                                            _stream(self.device)))
        return _tuning_dict(t)

    @property
    def schedule(self) -> dict:
        b = ctypes.c_void_p()
        _check(load_library().paradiag_batch(self._h, ctypes.byref(b)))
        t = _BatchTuning()
        _check(load_library().batch_schedule(b, ctypes.byref(t)))
        return _tuning_dict(t)


def batch_create(problems, **kw) -> Batch:
    return Batch(problems, **kw)


def batch_solve(b: Batch, fs, zs=None, **kw):
    return b.solve(fs, zs, **kw)


def batch_destroy(b: Batch):
    b.close()


def _make_autograd():
    torch = _torch()

    class CSLSolve(torch.autograd.Function):
        """z = (K(a) + (alpha + i beta) I)^{-1} f with a hand-written adjoint.

        forward(f, a, alpha, beta, problem=None, opts=None): ``problem`` may be
        an existing Problem built from the same a, alpha, beta (reused);
        otherwise one is created.  backward returns dL/df, dL/da, dL/dalpha,
        dL/dbeta from one extra MINRES solve (minres_adjoint)."""

        @staticmethod
        def forward(ctx, f, a, alpha, beta, problem=None, opts=None):
            opts = dict(opts or {})
            p = problem
            if p is None:
                p = Problem(a.detach().contiguous(), float(alpha), float(beta),
                            pinv_fp32=opts.pop("pinv_fp32", False),
                            abar_rule=opts.pop("abar_rule", "mean"))
            else:
                opts.pop("pinv_fp32", None)
                opts.pop("abar_rule", None)
            z, info = minres_solve(p, f.detach().contiguous(), **opts)
            ctx.p = p
            ctx.opts = opts
            ctx.info = info
            ctx.save_for_backward(z)
            return z

        @staticmethod
        def backward(ctx, gz):
            (z,) = ctx.saved_tensors
            g, _ = minres_adjoint(ctx.p, z, gz.contiguous(), **ctx.opts)
            need = ctx.needs_input_grad
            return (g["f"] if need[0] else None, g["a"] if need[1] else None,
                    g["alpha"] if need[2] else None, g["beta"] if need[3] else None,
                    None, None)

    return CSLSolve


class _LazyAutograd:
    _cls = None

    def __getattr__(self, item):
        if _LazyAutograd._cls is None:
            _LazyAutograd._cls = _make_autograd()
        return getattr(_LazyAutograd._cls, item)


CSLSolve = _LazyAutograd()


def solve(f, a, alpha, beta, problem=None, **opts):
    """Differentiable solve (see CSLSolve)."""
    return CSLSolve.apply(f, a, alpha, beta, problem, opts)
