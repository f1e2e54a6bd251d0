"""Plain FP64 CPU oracle for the two-level isogeometric solver.

TEST INFRASTRUCTURE ONLY: imported by ``tests/``, by ``__graft_entry__.smoke()``
and by the CPU-baseline leg of ``bench.py``.  The GPU library never imports,
links or calls anything here, and this package imports nothing from it.

The arithmetic lives in ``oracle.c`` (serial C, IEEE double); this module only
marshals numpy arrays through ctypes.  Every routine cites the part of the
paper (arXiv:2009.01499) it follows in ``oracle.c``.
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "oracle.c")
_LIB = os.path.join(_HERE, "liboracle.so")

LEX = 0
COLOUR = 1
DIRECT = 0
VCYCLE = 1


def build(force: bool = True) -> str:
    """Compile ``oracle.c`` into ``liboracle.so`` (plain -O2, no SIMD intrinsics)."""
    if force or not os.path.exists(_LIB):
        tmp = _LIB + ".tmp%d" % os.getpid()
        subprocess.check_call(["gcc", "-O2", "-std=c99", "-D_GNU_SOURCE", "-fPIC", "-shared",
                               "-o", tmp, _SRC, "-lm"])
        os.replace(tmp, _LIB)
    return _LIB


_lib = None


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB):
            build(force=True)
        L = ctypes.CDLL(_LIB)
        dp = ctypes.POINTER(ctypes.c_double)
        vp = ctypes.c_void_p
        i, l, d = ctypes.c_int, ctypes.c_long, ctypes.c_double
        sig = {
            "or_last_error": (ctypes.c_char_p, []),
            "or_knots": (i, [i, i, dp]),
            "or_bspline": (d, [dp, i, i, d]),
            "or_bspline_deriv": (d, [dp, i, i, d]),
            "or_gauss_legendre": (i, [i, dp, dp]),
            "or_assemble": (i, [i, i, i, dp, i, i, dp]),
            "or_assemble_mix": (i, [i, i, i, i, dp]),
            "or_load_manufactured": (i, [i, i, i, dp]),
            "or_l2_error_manufactured": (d, [i, i, i, dp]),
            "or_default_block_width": (i, [i]),
            "or_create": (vp, [i, i, i, dp, i, i, i, i, i]),
            "or_destroy": (None, [vp]),
            "or_n": (l, [vp]), "or_nc": (l, [vp]), "or_ne": (l, [vp]),
            "or_block_width": (i, [vp]), "or_nlevels": (i, [vp]),
            "or_get_A": (None, [vp, dp]), "or_get_Alow": (None, [vp, dp]),
            "or_get_Mlow": (None, [vp, dp]), "or_get_Mmix": (None, [vp, dp]),
            "or_get_Dlump": (None, [vp, dp]),
            "or_level_n": (l, [vp, i]), "or_get_level": (None, [vp, i, dp]),
            "or_apply_A": (None, [vp, dp, dp]),
            "or_residual": (None, [vp, dp, dp, dp]),
            "or_sweep": (i, [vp, dp, dp, i, i]),
            "or_restrict": (None, [vp, dp, dp]),
            "or_prolong_add": (None, [vp, dp, dp]),
            "or_coarse_direct": (i, [vp, dp, dp]),
            "or_coarse_vcycle": (i, [vp, dp, dp, i, i]),
            "or_cycle": (i, [vp, dp, dp, i, i, i, i, i, i, i, i]),
            "or_solve": (i, [vp, dp, dp, i, i, i, i, i, i, i, i, d, i, dp]),
            "or_setup_aggressive_direct": (i, [vp]),
            "or_coarse_aggressive": (i, [vp, dp, dp, i, i, i]),
            "or_direct_solve": (i, [vp, dp, dp]),
            "or_grad_kappa": (i, [vp, dp, dp, dp]),
            "or_element_apply": (i, [vp, l, dp, dp]),
            "or_annulus_weights": (i, [i, i, dp]),
            "or_load_annulus": (i, [i, i, d, d, dp]),
            "or_l2_error_annulus": (d, [i, i, d, d, dp]),
            "or_annulus_point": (None, [d, d, d, d, dp]),
            "or_assemble_annulus": (i, [i, i, i, d, d, i, dp]),
            "or_create_annulus": (vp, [i, i, i, i, i, i, d, d]),
        }
        for name, (res, args) in sig.items():
            f = getattr(L, name)
            f.restype = res
            f.argtypes = args
        _lib = L
    return _lib


def _p(a: np.ndarray):
    assert a.dtype == np.float64 and a.flags.c_contiguous
    return a.ctypes.data_as(ctypes.POINTER(ctypes.c_double))


def _err() -> str:
    return lib().or_last_error().decode()


# ---------------------------------------------------------------- basis --
def knots(p: int, m: int) -> np.ndarray:
    t = np.zeros(2 * p + m + 1)
    if lib().or_knots(p, m, _p(t)):
        raise ValueError(_err())
    return t


def bspline(t: np.ndarray, p: int, i: int, x: float) -> float:
    t = np.ascontiguousarray(t, dtype=np.float64)
    return lib().or_bspline(_p(t), p, i, x)


def bspline_deriv(t: np.ndarray, p: int, i: int, x: float) -> float:
    t = np.ascontiguousarray(t, dtype=np.float64)
    return lib().or_bspline_deriv(_p(t), p, i, x)


def gauss_legendre(q: int):
    x = np.zeros(q)
    w = np.zeros(q)
    if lib().or_gauss_legendre(q, _p(x), _p(w)):
        raise ValueError(_err())
    return x, w


# ------------------------------------------------------------- assembly --
def assemble(d: int, p: int, m: int, kappa=None, kind: str = "stiff", dirichlet: bool = True) -> np.ndarray:
    """Offset-stored stiffness/mass matrix, shape (n, (2p+1)^d)."""
    n1 = m + p - 2 if dirichlet else m + p
    out = np.zeros((n1 ** d, (2 * p + 1) ** d))
    kp = None
    if kappa is not None:
        kappa = np.ascontiguousarray(kappa, dtype=np.float64).ravel()
        kp = _p(kappa)
    if lib().or_assemble(d, p, m, kp, 0 if kind == "stiff" else 1, 1 if dirichlet else 0, _p(out)):
        raise ValueError(_err())
    return out


def assemble_mix(d: int, p: int, plow: int, m: int) -> np.ndarray:
    out = np.zeros(((m + plow - 2) ** d, (p + plow + 1) ** d))
    if lib().or_assemble_mix(d, p, plow, m, _p(out)):
        raise ValueError(_err())
    return out


def load_manufactured(d: int, p: int, m: int) -> np.ndarray:
    b = np.zeros((m + p - 2) ** d)
    lib().or_load_manufactured(d, p, m, _p(b))
    return b


def l2_error_manufactured(d: int, p: int, m: int, u: np.ndarray) -> float:
    u = np.ascontiguousarray(u, dtype=np.float64)
    return lib().or_l2_error_manufactured(d, p, m, _p(u))


def default_block_width(p: int) -> int:
    return lib().or_default_block_width(p)


def offsets_to_dense(S: np.ndarray, d: int, n1: int, q: int) -> np.ndarray:
    """Dense matrix of an offset-stored operator (test helper, tiny grids)."""
    n = n1 ** d
    w1 = 2 * q + 1
    D = np.zeros((n, n))
    for i in range(n):
        ix = [(i // n1 ** k) % n1 for k in range(d)]
        for w in range(w1 ** d):
            o = [(w // w1 ** k) % w1 - q for k in range(d)]
            jx = [ix[k] + o[k] for k in range(d)]
            if all(0 <= j < n1 for j in jx):
                D[i, sum(jx[k] * n1 ** k for k in range(d))] = S[i, w]
    return D


def mix_to_dense(S: np.ndarray, d: int, p: int, plow: int, m: int) -> np.ndarray:
    n1, n1c = m + p - 2, m + plow - 2
    wm = p + plow + 1
    D = np.zeros((n1c ** d, n1 ** d))
    for I in range(n1c ** d):
        IX = [(I // n1c ** k) % n1c for k in range(d)]
        for w in range(wm ** d):
            o = [(w // wm ** k) % wm - plow for k in range(d)]
            jx = [IX[k] + o[k] for k in range(d)]
            if all(0 <= j < n1 for j in jx):
                D[I, sum(jx[k] * n1 ** k for k in range(d))] = S[I, w]
    return D


# -------------------------------------------------------------- problem --
class Problem:
    """The oracle's problem object: operators, Schwarz blocks, coarse solvers."""

    def __init__(self, d: int, p: int, m: int, kappa=None, plow: int = 1, block_width: int = 0,
                 lumped: bool = True, coarse_direct: bool = True, vcycle: bool = False, annulus=None):
        """annulus=(r, R): the quarter-annulus NURBS problem of Section 5.2
        (d = 2, kappa unused) instead of the unit square."""
        self.d, self.p, self.m, self.plow = d, p, m, plow
        self._kappa = None
        kp = None
        if kappa is not None:
            self._kappa = np.ascontiguousarray(kappa, dtype=np.float64).ravel()
            kp = _p(self._kappa)
        if annulus is not None:
            if d != 2 or kappa is not None or vcycle:
                raise ValueError("the annulus problem is 2-D, with no coefficient and no V-cycle hierarchy")
            h = lib().or_create_annulus(p, m, plow, block_width, 1 if lumped else 0, 1 if coarse_direct else 0,
                                        float(annulus[0]), float(annulus[1]))
        else:
            h = lib().or_create(d, p, m, kp, plow, block_width, 1 if lumped else 0,
                                1 if coarse_direct else 0, 1 if vcycle else 0)
        if not h:
            raise ValueError(_err())
        self._h = ctypes.c_void_p(h)
        self.n = lib().or_n(self._h)
        self.nc = lib().or_nc(self._h)
        self.ne = lib().or_ne(self._h)
        self.block_width = lib().or_block_width(self._h)
        self.n1 = m + p - 2
        self.n1c = m + plow - 2

    def __del__(self):
        if getattr(self, "_h", None) is not None and _lib is not None:
            _lib.or_destroy(self._h)
            self._h = None

    # operators
    def A(self):
        out = np.zeros((self.n, (2 * self.p + 1) ** self.d))
        lib().or_get_A(self._h, _p(out))
        return out

    def Alow(self):
        out = np.zeros((self.nc, (2 * self.plow + 1) ** self.d))
        lib().or_get_Alow(self._h, _p(out))
        return out

    def Mlow(self):
        out = np.zeros((self.nc, (2 * self.plow + 1) ** self.d))
        lib().or_get_Mlow(self._h, _p(out))
        return out

    def Mmix(self):
        out = np.zeros((self.nc, (self.p + self.plow + 1) ** self.d))
        lib().or_get_Mmix(self._h, _p(out))
        return out

    def Dlump(self):
        out = np.zeros(self.nc)
        lib().or_get_Dlump(self._h, _p(out))
        return out

    def nlevels(self) -> int:
        return lib().or_nlevels(self._h)

    def level(self, l: int) -> np.ndarray:
        n = lib().or_level_n(self._h, l)
        out = np.zeros((n, 3 ** self.d))
        lib().or_get_level(self._h, l, _p(out))
        return out

    # operations
    def apply_A(self, x):
        x = np.ascontiguousarray(x, dtype=np.float64)
        y = np.zeros(self.n)
        lib().or_apply_A(self._h, _p(x), _p(y))
        return y

    def residual(self, u, b):
        u = np.ascontiguousarray(u, dtype=np.float64)
        b = np.ascontiguousarray(b, dtype=np.float64)
        r = np.zeros(self.n)
        lib().or_residual(self._h, _p(u), _p(b), _p(r))
        return r

    def sweep(self, u, b, ordering: int = COLOUR, s: int = 0):
        """Return the iterate after one Schwarz sweep (u is not modified)."""
        u = np.array(u, dtype=np.float64, copy=True)
        b = np.ascontiguousarray(b, dtype=np.float64)
        if lib().or_sweep(self._h, _p(u), _p(b), ordering, s or self.block_width):
            raise ValueError(_err())
        return u

    def restrict(self, d):
        d = np.ascontiguousarray(d, dtype=np.float64)
        dc = np.zeros(self.nc)
        lib().or_restrict(self._h, _p(d), _p(dc))
        return dc

    def prolong_add(self, ec, u):
        ec = np.ascontiguousarray(ec, dtype=np.float64)
        u = np.array(u, dtype=np.float64, copy=True)
        lib().or_prolong_add(self._h, _p(ec), _p(u))
        return u

    def coarse_direct(self, dc):
        dc = np.ascontiguousarray(dc, dtype=np.float64)
        ec = np.zeros(self.nc)
        if lib().or_coarse_direct(self._h, _p(dc), _p(ec)):
            raise ValueError(_err())
        return ec

    def coarse_vcycle(self, dc, nu1: int = 1, nu2: int = 1):
        dc = np.ascontiguousarray(dc, dtype=np.float64)
        ec = np.zeros(self.nc)
        if lib().or_coarse_vcycle(self._h, _p(dc), _p(ec), nu1, nu2):
            raise ValueError(_err())
        return ec

    def _aggressive_ready(self, coarse, aggressive):
        if aggressive and coarse == DIRECT and not getattr(self, "_agg_direct", False):
            if lib().or_setup_aggressive_direct(self._h):
                raise ValueError(_err())
            self._agg_direct = True

    def coarse_aggressive(self, dc, coarse=DIRECT, nu1=1, nu2=1):
        """Coarse correction of aggressive coarsening (degree 1 on 2h, Section 3.3)."""
        self._aggressive_ready(coarse, True)
        dc = np.ascontiguousarray(dc, dtype=np.float64)
        ec = np.zeros(self.nc)
        if lib().or_coarse_aggressive(self._h, _p(dc), _p(ec), coarse, nu1, nu2):
            raise ValueError(_err())
        return ec

    def cycle(self, u, b, ordering=COLOUR, s=0, nu1=1, nu2=0, coarse=DIRECT, cnu1=1, cnu2=1, aggressive=False):
        self._aggressive_ready(coarse, aggressive)
        u = np.array(u, dtype=np.float64, copy=True)
        b = np.ascontiguousarray(b, dtype=np.float64)
        if lib().or_cycle(self._h, _p(u), _p(b), ordering, s or self.block_width, nu1, nu2,
                          coarse, cnu1, cnu2, 1 if aggressive else 0):
            raise ValueError(_err())
        return u

    def solve(self, b, u0=None, ordering=COLOUR, s=0, nu1=1, nu2=0, coarse=DIRECT, cnu1=1, cnu2=1,
              tol=1e-10, max_cycles=100, aggressive=False):
        """Iterate cycles to ||r|| <= tol ||r0||; returns (u, cycles, residual history)."""
        self._aggressive_ready(coarse, aggressive)
        b = np.ascontiguousarray(b, dtype=np.float64)
        u = np.zeros(self.n) if u0 is None else np.array(u0, dtype=np.float64, copy=True)
        hist = np.zeros(max_cycles + 1)
        k = lib().or_solve(self._h, _p(b), _p(u), ordering, s or self.block_width, nu1, nu2,
                           coarse, cnu1, cnu2, 1 if aggressive else 0, tol, max_cycles, _p(hist))
        if k < 0:
            raise ValueError(_err())
        return u, k, hist[:k + 1].copy()

    def direct_solve(self, b):
        b = np.ascontiguousarray(b, dtype=np.float64)
        u = np.zeros(self.n)
        if lib().or_direct_solve(self._h, _p(b), _p(u)):
            raise ValueError(_err())
        return u

    def element_apply(self, e: int, u):
        """A_e u for element e (unit coefficient), full-length vector."""
        u = np.ascontiguousarray(u, dtype=np.float64)
        out = np.zeros(self.n)
        if lib().or_element_apply(self._h, e, _p(u), _p(out)):
            raise ValueError(_err())
        return out

    def grad_kappa(self, u, lam):
        u = np.ascontiguousarray(u, dtype=np.float64)
        lam = np.ascontiguousarray(lam, dtype=np.float64)
        g = np.zeros(self.ne)
        lib().or_grad_kappa(self._h, _p(u), _p(lam), _p(g))
        return g


# ------------------------------------------------------------- annulus --
ANNULUS = (0.3, 0.5)   # inner and outer radius of Section 5.2


def annulus_weights(q: int, m: int) -> np.ndarray:
    """Weights of the degree-q, m-element basis (all m+q functions) that
    reproduce the denominator of the rational quadratic quarter circle."""
    w = np.zeros(m + q)
    if lib().or_annulus_weights(q, m, _p(w)):
        raise ValueError(_err())
    return w


def load_annulus(p: int, m: int, radii=ANNULUS) -> np.ndarray:
    b = np.zeros((m + p - 2) ** 2)
    if lib().or_load_annulus(p, m, float(radii[0]), float(radii[1]), _p(b)):
        raise ValueError(_err())
    return b


def l2_error_annulus(p: int, m: int, u: np.ndarray, radii=ANNULUS) -> float:
    u = np.ascontiguousarray(u, dtype=np.float64)
    return lib().or_l2_error_annulus(p, m, float(radii[0]), float(radii[1]), _p(u))


def annulus_point(xi: float, eta: float, radii=ANNULUS) -> np.ndarray:
    out = np.zeros(2)
    lib().or_annulus_point(float(radii[0]), float(radii[1]), float(xi), float(eta), _p(out))
    return out


def assemble_annulus(p: int, plow: int, m: int, kind: str, radii=ANNULUS) -> np.ndarray:
    """kind: 'stiff', 'mass' (degree p, by offset of radius p) or 'mix'
    (rows degree plow, columns degree p, offsets [-plow, p])."""
    k = {"stiff": 0, "mass": 1, "mix": 2}[kind]
    if k == 2:
        out = np.zeros(((m + plow - 2) ** 2, (p + plow + 1) ** 2))
    else:
        out = np.zeros(((m + p - 2) ** 2, (2 * p + 1) ** 2))
    if lib().or_assemble_annulus(p, plow, m, float(radii[0]), float(radii[1]), k, _p(out)):
        raise ValueError(_err())
    return out
