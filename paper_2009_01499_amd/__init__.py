"""Python face of the gfx950 two-level solver for isogeometric discretisations.

This module only marshals arguments to the C ABI of ``include/iga2l.h``
(``libiga2l.so``, built in-tree by :mod:`paper_2009_01499_amd.build`); every
step of the solver runs in the library's HIP kernels.  Device vectors are
contiguous ``torch.float64`` CUDA tensors; torch is used for device memory and
streams only.  If the library is missing, every entry point raises.
"""
from __future__ import annotations

import ctypes
import dataclasses
import os
from typing import Optional, Sequence

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libiga2l.so")
HEADER_PATH = os.path.join(os.path.dirname(_HERE), "include", "iga2l.h")

OK, EINVAL, ENOMEM, EDEVICE, ENOTCONV, ENUMERIC, EUNSUPPORTED = 0, -1, -2, -3, -4, -5, -6
LEX, COLOUR = 0, 1
COARSE_DIRECT, COARSE_VCYCLE = 0, 1
FP64, MIXED_FP32 = 0, 1

_ERRNAMES = {EINVAL: "EINVAL", ENOMEM: "ENOMEM", EDEVICE: "EDEVICE", ENOTCONV: "ENOTCONV",
             ENUMERIC: "ENUMERIC", EUNSUPPORTED: "EUNSUPPORTED"}


class IGA2LError(RuntimeError):
    def __init__(self, code: int, msg: str):
        super().__init__(f"{_ERRNAMES.get(code, code)}: {msg}")
        self.code = code


class CIgaOpts(ctypes.Structure):
    _fields_ = [("tol", ctypes.c_double), ("max_cycles", ctypes.c_int), ("ordering", ctypes.c_int),
                ("colour_period", ctypes.c_int), ("coarse", ctypes.c_int), ("nu1", ctypes.c_int),
                ("nu2", ctypes.c_int), ("precision", ctypes.c_int), ("fine_post_sweeps", ctypes.c_int),
                ("lumped", ctypes.c_int), ("aggressive", ctypes.c_int), ("plow", ctypes.c_int)]


class CIgaInfo(ctypes.Structure):
    _fields_ = [("iters", ctypes.c_int), ("status", ctypes.c_int), ("r0", ctypes.c_double),
                ("relres", ctypes.c_double), ("t_solve_ms", ctypes.c_double), ("t_setup_ms", ctypes.c_double),
                ("relres_history", ctypes.POINTER(ctypes.c_double)), ("history_cap", ctypes.c_int)]


@dataclasses.dataclass
class Opts:
    """Mirror of ``iga2l_opts`` (defaults as ``iga2l_default_opts``)."""
    tol: float = 1e-10
    max_cycles: int = 100
    ordering: int = COLOUR
    colour_period: int = 0
    coarse: int = COARSE_VCYCLE
    nu1: int = 1
    nu2: int = 1
    precision: int = FP64
    fine_post_sweeps: int = 0
    lumped: int = 1
    aggressive: int = 0
    plow: int = 1

    def c(self) -> CIgaOpts:
        return CIgaOpts(self.tol, self.max_cycles, self.ordering, self.colour_period, self.coarse,
                        self.nu1, self.nu2, self.precision, self.fine_post_sweeps, self.lumped, self.aggressive,
                        self.plow)


@dataclasses.dataclass
class Info:
    iters: int
    status: int
    r0: float
    relres: float
    t_solve_ms: float
    history: np.ndarray
    t_setup_ms: float = 0.0


_lib = None

_EXPORTS = {
    # name: (restype, argtypes)
    "iga2l_default_opts": (None, [ctypes.POINTER(CIgaOpts)]),
    "iga2l_last_error": (ctypes.c_char_p, []),
    "iga2l_assemble": (ctypes.c_int, [ctypes.c_int, ctypes.POINTER(ctypes.c_void_p), ctypes.POINTER(ctypes.c_int),
                                      ctypes.c_int, ctypes.c_void_p, ctypes.c_int, ctypes.POINTER(ctypes.c_void_p)]),
    "iga2l_assemble_annulus": (ctypes.c_int, [ctypes.c_int, ctypes.c_int, ctypes.c_double, ctypes.c_double,
                                              ctypes.c_int, ctypes.POINTER(ctypes.c_void_p)]),
    "iga2l_setup_blocks": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_int, ctypes.POINTER(CIgaOpts)]),
    "iga2l_sizes": (ctypes.c_int, [ctypes.c_void_p, ctypes.POINTER(ctypes.c_int64), ctypes.POINTER(ctypes.c_int64),
                                   ctypes.POINTER(ctypes.c_int64)]),
    "iga2l_residual": (ctypes.c_int, [ctypes.c_void_p] * 5),
    "iga2l_smooth": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p, ctypes.c_int,
                                    ctypes.POINTER(CIgaOpts), ctypes.c_void_p]),
    "iga2l_smooth_noalloc": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p, ctypes.c_int,
                                            ctypes.POINTER(CIgaOpts), ctypes.c_void_p]),
    "iga2l_time_colour": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_int, ctypes.c_int, ctypes.POINTER(CIgaOpts),
                                         ctypes.c_void_p, ctypes.POINTER(ctypes.c_double)]),
    "iga2l_restrict": (ctypes.c_int, [ctypes.c_void_p] * 4),
    "iga2l_prolong": (ctypes.c_int, [ctypes.c_void_p] * 4),
    "iga2l_coarse_solve": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p,
                                          ctypes.POINTER(CIgaOpts), ctypes.c_void_p]),
    "iga2l_solve": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p, ctypes.POINTER(CIgaOpts),
                                   ctypes.POINTER(CIgaInfo), ctypes.c_void_p]),
    "iga2l_solve_batch": (ctypes.c_int, [ctypes.POINTER(ctypes.c_void_p), ctypes.c_int,
                                         ctypes.POINTER(ctypes.c_void_p), ctypes.POINTER(ctypes.c_void_p),
                                         ctypes.POINTER(CIgaOpts), ctypes.POINTER(CIgaInfo), ctypes.c_void_p]),
    "iga2l_solve_backward": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p,
                                            ctypes.c_void_p, ctypes.POINTER(CIgaOpts), ctypes.POINTER(CIgaInfo),
                                            ctypes.c_void_p]),
    "iga2l_destroy": (None, [ctypes.c_void_p]),
}


def lib() -> ctypes.CDLL:
    """The loaded HIP library; raises if it has not been built."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise IGA2LError(EDEVICE, f"{LIB_PATH} is missing: build it with "
                                      "`python -m paper_2009_01499_amd.build` (there is no CPU fallback)")
        L = ctypes.CDLL(LIB_PATH)
        for name, (res, args) in _EXPORTS.items():
            f = getattr(L, name)
            f.restype = res
            f.argtypes = args
        _lib = L
    return _lib


def _check(code: int):
    if code != OK:
        raise IGA2LError(code, lib().iga2l_last_error().decode())


def _torch():
    import torch
    return torch


def _dev_ptr(t, n: Optional[int] = None, what: str = "vector") -> ctypes.c_void_p:
    torch = _torch()
    if not isinstance(t, torch.Tensor) or t.device.type != "cuda" or t.dtype != torch.float64 or not t.is_contiguous():
        raise TypeError(f"{what} must be a contiguous torch.float64 CUDA tensor")
    if n is not None and t.numel() != n:
        raise ValueError(f"{what} has {t.numel()} entries, expected {n}")
    return ctypes.c_void_p(t.data_ptr())


def _stream(stream=None) -> ctypes.c_void_p:
    torch = _torch()
    s = torch.cuda.current_stream() if stream is None else stream
    return ctypes.c_void_p(s.cuda_stream)


def open_uniform_knots(p: int, m: int) -> np.ndarray:
    """The open uniform knot vector of degree p on m elements (p+1 zeros, i/m, p+1 ones)."""
    return np.concatenate([np.zeros(p + 1), np.arange(1, m) / m, np.ones(p + 1)])


class Problem:
    """An assembled problem on one device (``iga2l_assemble``)."""

    def __init__(self, dim: int, p: int, m: int, kappa=None, device: int = 0, annulus=None):
        """annulus=(r_in, r_out): the quarter-annulus NURBS problem
        (``iga2l_assemble_annulus``; dim must be 2, no kappa)."""
        self.dim, self.p, self.m, self.device = dim, p, m, device
        if annulus is not None:
            if dim != 2 or kappa is not None:
                raise ValueError("the annulus problem is 2-D without a coefficient")
            h = ctypes.c_void_p()
            _check(lib().iga2l_assemble_annulus(p, m, float(annulus[0]), float(annulus[1]), device,
                                                ctypes.byref(h)))
            self._h = h
            nf, nc, ne = ctypes.c_int64(), ctypes.c_int64(), ctypes.c_int64()
            _check(lib().iga2l_sizes(self._h, ctypes.byref(nf), ctypes.byref(nc), ctypes.byref(ne)))
            self.n, self.nc, self.ne = nf.value, nc.value, ne.value
            return
        t = open_uniform_knots(p, m)
        self._knots = [np.ascontiguousarray(t, dtype=np.float64) for _ in range(dim)]
        kptrs = (ctypes.c_void_p * dim)(*[k.ctypes.data for k in self._knots])
        nk = (ctypes.c_int * dim)(*[len(k) for k in self._knots])
        kap = None
        if kappa is not None:
            self._kappa = np.ascontiguousarray(np.asarray(kappa, dtype=np.float64).ravel())
            kap = ctypes.c_void_p(self._kappa.ctypes.data)
        h = ctypes.c_void_p()
        _check(lib().iga2l_assemble(dim, ctypes.cast(kptrs, ctypes.POINTER(ctypes.c_void_p)), nk, p, kap, device,
                                    ctypes.byref(h)))
        self._h = h
        nf, nc, ne = ctypes.c_int64(), ctypes.c_int64(), ctypes.c_int64()
        _check(lib().iga2l_sizes(self._h, ctypes.byref(nf), ctypes.byref(nc), ctypes.byref(ne)))
        self.n, self.nc, self.ne = nf.value, nc.value, ne.value

    def close(self):
        if getattr(self, "_h", None) is not None and _lib is not None:
            _lib.iga2l_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    # ------------------------------------------------------------ set-up --
    def setup(self, block_width: int = 0, opts: Optional[Opts] = None):
        o = (opts or Opts()).c()
        _check(lib().iga2l_setup_blocks(self._h, block_width, ctypes.byref(o)))
        nc = ctypes.c_int64()
        _check(lib().iga2l_sizes(self._h, None, ctypes.byref(nc), None))
        self.nc = nc.value      # the coarse space follows the set-up's plow
        return self

    # --------------------------------------------------------- operations --
    def residual(self, u, b, r=None, stream=None):
        torch = _torch()
        if r is None:
            r = torch.empty_like(u)
        _check(lib().iga2l_residual(self._h, _dev_ptr(u, self.n, "u"), _dev_ptr(b, self.n, "b"),
                                    _dev_ptr(r, self.n, "r"), _stream(stream)))
        return r

    def smooth(self, u, b, nsweeps: int = 1, opts: Optional[Opts] = None, stream=None):
        o = (opts or Opts()).c()
        _check(lib().iga2l_smooth(self._h, _dev_ptr(u, self.n, "u"), _dev_ptr(b, self.n, "b"), nsweeps,
                                  ctypes.byref(o), _stream(stream)))
        return u

    def smooth_noalloc(self, u, b, nsweeps: int = 1, opts: Optional[Opts] = None, stream=None):
        """iga2l_smooth_noalloc: the coloured sweeps of smooth() without any
        device allocation (intermediate iterates in the library's fixed array)."""
        o = (opts or Opts()).c()
        _check(lib().iga2l_smooth_noalloc(self._h, _dev_ptr(u, self.n, "u"), _dev_ptr(b, self.n, "b"), nsweeps,
                                          ctypes.byref(o), _stream(stream)))
        return u

    def time_colour(self, precision: int = FP64, nsweeps: int = 20, opts: Optional[Opts] = None, stream=None) -> float:
        """Average ms per launch of the coloured Schwarz kernel (HIP events in the library)."""
        o = (opts or Opts()).c()
        ms = ctypes.c_double()
        _check(lib().iga2l_time_colour(self._h, precision, nsweeps, ctypes.byref(o), _stream(stream),
                                       ctypes.byref(ms)))
        return ms.value

    def restrict(self, r, dc=None, stream=None):
        torch = _torch()
        if dc is None:
            dc = torch.empty(self.nc, dtype=torch.float64, device=r.device)
        _check(lib().iga2l_restrict(self._h, _dev_ptr(r, self.n, "r"), _dev_ptr(dc, self.nc, "d_coarse"),
                                    _stream(stream)))
        return dc

    def prolong_add(self, ec, u, stream=None):
        _check(lib().iga2l_prolong(self._h, _dev_ptr(ec, self.nc, "e_coarse"), _dev_ptr(u, self.n, "u"),
                                   _stream(stream)))
        return u

    def coarse_solve(self, dc, ec=None, opts: Optional[Opts] = None, stream=None):
        torch = _torch()
        if ec is None:
            ec = torch.empty_like(dc)
        o = (opts or Opts()).c()
        _check(lib().iga2l_coarse_solve(self._h, _dev_ptr(dc, self.nc, "d_coarse"), _dev_ptr(ec, self.nc, "e_coarse"),
                                        ctypes.byref(o), _stream(stream)))
        return ec

    def solve(self, b, u=None, opts: Optional[Opts] = None, stream=None, raise_on_notconv: bool = True):
        """Two-level cycles from u (zero if None) to opts.tol; returns (u, Info)."""
        torch = _torch()
        o = opts or Opts()
        if u is None:
            u = torch.zeros_like(b)
        hist = np.zeros(max(o.max_cycles, 1))
        info = CIgaInfo()
        info.relres_history = hist.ctypes.data_as(ctypes.POINTER(ctypes.c_double))
        info.history_cap = len(hist)
        co = o.c()
        code = lib().iga2l_solve(self._h, _dev_ptr(b, self.n, "b"), _dev_ptr(u, self.n, "u"), ctypes.byref(co),
                                 ctypes.byref(info), _stream(stream))
        res = Info(info.iters, info.status, info.r0, info.relres, info.t_solve_ms, hist[:info.iters].copy(),
                   info.t_setup_ms)
        if code != OK and not (code == ENOTCONV and not raise_on_notconv):
            _check(code)
        return u, res

    def solve_backward(self, u, grad_u, opts: Optional[Opts] = None, stream=None):
        """(lambda, grad_kappa) for lambda = A^{-1} grad_u and dL/dkappa_e."""
        torch = _torch()
        lam = torch.empty_like(u)
        g = torch.empty(self.ne, dtype=torch.float64, device=u.device)
        info = CIgaInfo()
        co = (opts or Opts()).c()
        _check(lib().iga2l_solve_backward(self._h, _dev_ptr(u, self.n, "u"), _dev_ptr(grad_u, self.n, "grad_u"),
                                          _dev_ptr(lam, self.n, "lambda"), _dev_ptr(g, self.ne, "grad_kappa"),
                                          ctypes.byref(co), ctypes.byref(info), _stream(stream)))
        return lam, g


def solve_batch(problems: Sequence[Problem], bs, us, opts: Optional[Opts] = None, stream=None,
                raise_on_notconv: bool = True):
    """Solve independent problems b[k] -> u[k] (u[k] holds the start) in one
    call; returns a list of Info.  2-D batches with the coloured sweep and the
    V-cycle run with batched launches, other batches problem by problem."""
    n = len(problems)
    o = opts or Opts()
    hs = (ctypes.c_void_p * n)(*[p._h.value for p in problems])
    bp = (ctypes.c_void_p * n)(*[_dev_ptr(b, p.n, "b").value for b, p in zip(bs, problems)])
    up = (ctypes.c_void_p * n)(*[_dev_ptr(u, p.n, "u").value for u, p in zip(us, problems)])
    infos = (CIgaInfo * n)()
    hists = [np.zeros(max(o.max_cycles, 1)) for _ in range(n)]
    for i, h in zip(infos, hists):
        i.relres_history = h.ctypes.data_as(ctypes.POINTER(ctypes.c_double))
        i.history_cap = len(h)
    co = o.c()
    code = lib().iga2l_solve_batch(hs, n, bp, up, ctypes.byref(co), infos, _stream(stream))
    if code != OK and not (code == ENOTCONV and not raise_on_notconv):
        _check(code)
    return [Info(i.iters, i.status, i.r0, i.relres, i.t_solve_ms, h[:i.iters].copy(), i.t_setup_ms)
            for i, h in zip(infos, hists)]


def header_functions() -> list:
    """Names of the functions declared in include/iga2l.h."""
    import re
    txt = open(HEADER_PATH).read()
    txt = re.sub(r"/\*.*?\*/", "", txt, flags=re.S)
    return sorted(set(re.findall(r"\b(iga2l_[a-z_0-9]+)\s*\(", txt)))


def _autograd_function():
    torch = _torch()

    class IGASolve(torch.autograd.Function):
        """u = A(kappa)^{-1} b on the degree-p B-spline space of m^dim elements.

        forward(kappa, b, dim, p, m, opts_forward, opts_adjoint) assembles and
        solves with the two-level method; backward(grad_u) solves the adjoint
        system A lambda = grad_u with the same solver (A is symmetric) and
        evaluates dL/dkappa_e = -integral_e grad(lambda_h) . grad(u_h) in one
        element-wise kernel.  Returns (dL/dkappa, dL/db = lambda).
        """

        @staticmethod
        def forward(ctx, kappa, b, dim, p, m, opts_forward=None, opts_adjoint=None):
            kap = kappa.detach().to("cpu", torch.float64).contiguous().numpy()
            dev = b.device
            prob = Problem(dim, p, m, kappa=kap, device=dev.index or 0)
            of = opts_forward or Opts()
            oa = opts_adjoint or Opts(precision=FP64, tol=1e-12)
            prob.setup(0, of)
            if oa.precision != of.precision or oa.coarse != of.coarse:
                prob.setup(0, oa)
            u, _ = prob.solve(b.detach().contiguous(), None, of)
            ctx.prob, ctx.oa = prob, oa
            ctx.kappa_device, ctx.kappa_shape = kappa.device, kappa.shape
            ctx.save_for_backward(u)
            return u.clone()

        @staticmethod
        def backward(ctx, grad_u):
            (u,) = ctx.saved_tensors
            lam, g = ctx.prob.solve_backward(u, grad_u.detach().contiguous(), ctx.oa)
            gk = g.to(ctx.kappa_device).reshape(ctx.kappa_shape)
            return gk, lam, None, None, None, None, None

    return IGASolve


_IGASolve = None


def iga_solve(kappa, b, dim: int, p: int, m: int, opts_forward: Optional[Opts] = None,
              opts_adjoint: Optional[Opts] = None):
    """Differentiable solve u = A(kappa)^{-1} b (see the IGASolve Function)."""
    global _IGASolve
    if _IGASolve is None:
        _IGASolve = _autograd_function()
    return _IGASolve.apply(kappa, b, dim, p, m, opts_forward, opts_adjoint)
