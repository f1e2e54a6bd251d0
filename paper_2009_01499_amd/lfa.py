"""Local Fourier analysis (Section 4) of the two-level method for B-spline
discretisations of the 2-D Poisson problem: the convergence factors the paper
uses to choose the Schwarz block size per degree and to support the two
cheaper coarse levels.

  rho_2g(p, b)      two-grid factor: lexicographic multiplicative Schwarz sweep
                    with b x b blocks (Section 3.1.1), degree-1 coarse level on
                    the same grid, exact coarse solve (Section 4.1; Table 1)
  rho_3g(p, b)      three-grid factor: the degree-1 level approximated by one
                    V(nu1, nu2) red-black Gauss-Seidel two-grid cycle towards
                    2h (Section 4.1; Table 2)
  rho_2g_ag(p, b)   two-grid factor of aggressive coarsening: degree 1 on the
                    grid of size 2h (Section 3.3, Section 4.1; Table 3)

Everything is host arithmetic (numpy) on the infinite uniform grid of size h
(h cancels in 2-D).  The operators' stencils come from closed forms of the
centred cardinal B-spline B_n: the interior mass stencil h B_{2p+1}(k), the
interior stiffness stencil -(B_{2p-1}(k+1) - 2 B_{2p-1}(k) + B_{2p-1}(k-1))/h,
and the interior rows of the lumped restriction B_{p+2}(t) (t the offset from
a degree-1 node to a degree-p centre, in units of h).

Symbols.  Fourier modes exp(i theta x/h) are eigenfunctions of every operator
on one grid, so on the same grid the transfers give scalars.
  * Operator: A(theta) = sum_o a(o) exp(i theta.o).
  * Lexicographic block sweep: with the ansatz that block j's correction is
    d exp(i theta.j) (d a vector over the b^2 block points), block j sees the
    initial error plus the corrections of all blocks before it in the
    lexicographic order, which gives (A_B + L(theta)) d = -c(theta), with A_B
    the block matrix, c_o = A(theta) exp(i theta.o) and L(theta)_{oq} = the sum
    over preceding relative block positions k of a(k + q - o) exp(i theta.k);
    the sweep symbol is S(theta) = 1 + sum_q d_q exp(-i theta.q).
  * Degree transfers on one grid: R(theta) = R1(theta_x) R1(theta_y),
    R1(t) = sum over the lattice offsets of B_{p+2}(t) cos(theta t) (real, so
    the prolongation R^T has the same symbol).
  * h -> 2h between degree-1 spaces couples the four harmonics theta + pi a,
    a in {0,1}^2: the linear interpolation P0 contributes prod (1 + cos)/2 per
    harmonic, its transpose prod (1 + cos), the 2h operator is the Galerkin
    product; the red-black smoother couples theta with theta + (pi, pi).
The factors are the largest spectral radius of the symbol over the
frequencies: a cell-centred grid (theta = 0, where every coarse correction is
exact, is never a grid point) refined around its best points.
"""
from __future__ import annotations

import numpy as np

__all__ = ["cardinal_bspline", "stencils_1d", "operator_stencil_2d", "restriction_symbol_1d", "schwarz_lex_symbol",
           "two_grid_symbol", "three_grid_symbol", "aggressive_symbol", "rho_2g", "rho_3g", "rho_2g_ag",
           "block_width_for"]


def block_width_for(p: int) -> int:
    """The paper's block width per degree (Sections 4.2, 5.1)."""
    return 3 if p <= 4 else (5 if p <= 6 else 7)


def cardinal_bspline(n: int, x):
    """Centred cardinal B-spline of degree n (support [-(n+1)/2, (n+1)/2]) by the
    recursion B_n(x) = ((n+1)/2 + x) B_{n-1}(x + 1/2) + ((n+1)/2 - x) B_{n-1}(x - 1/2),
    divided by n, from the unit box B_0 (1/2 at its two ends, the mean of the
    one-sided values; B_n is continuous for n >= 1).  Stable for every degree,
    unlike the alternating truncated-power sum."""
    x = np.asarray(x, dtype=np.float64)
    if n == 0:
        ax = np.abs(x)
        return np.where(ax < 0.5, 1.0, np.where(ax == 0.5, 0.5, 0.0))
    c = (n + 1) / 2.0
    return ((c + x) * cardinal_bspline(n - 1, x + 0.5) + (c - x) * cardinal_bspline(n - 1, x - 0.5)) / n


def stencils_1d(p: int):
    """Interior rows (offsets -p..p) of the 1-D degree-p stiffness and mass
    matrices with h = 1: (K, M)."""
    k = np.arange(-p, p + 1, dtype=np.float64)
    M = cardinal_bspline(2 * p + 1, k)
    if p == 1:
        K = np.array([-1.0, 2.0, -1.0])
    else:
        K = -(cardinal_bspline(2 * p - 1, k + 1) - 2 * cardinal_bspline(2 * p - 1, k) +
              cardinal_bspline(2 * p - 1, k - 1))
    return K, M


def operator_stencil_2d(p: int) -> np.ndarray:
    """a[oy + p, ox + p] of the 2-D stiffness K (x) M + M (x) K (h cancels)."""
    K, M = stencils_1d(p)
    return np.outer(M, K) + np.outer(K, M)


def _symbol(stencil: np.ndarray, th: np.ndarray) -> np.ndarray:
    """sum_o a(o) exp(i theta.o) for theta of shape (..., 2)."""
    q = (stencil.shape[0] - 1) // 2
    o = np.arange(-q, q + 1)
    ex = np.exp(1j * th[..., 0, None] * o)       # (..., W)
    ey = np.exp(1j * th[..., 1, None] * o)
    return np.einsum("...y,yx,...x->...", ey, stencil, ex)


def restriction_symbol_1d(p: int, theta, lumped: bool = True):
    """Symbol of one direction of I_p^1 on the same grid: interior rows of
    D^{-1} M_p^1 are B_{p+2}(t) at the offsets t between a degree-1 node and
    the degree-p centres (integers for odd p, half-integers for even p).
    lumped=False: (M_1^1)^{-1} M_p^1, i.e. divided by the mass symbol
    (2 + cos theta)/3 of the degree-1 space."""
    theta = np.asarray(theta, dtype=np.float64)
    half = (p + 2) / 2.0
    shift = 0.0 if p % 2 == 1 else 0.5
    t = np.arange(-np.ceil(half) - 1, np.ceil(half) + 2) + shift
    t = t[np.abs(t) < half]
    r = np.sum(cardinal_bspline(p + 2, t) * np.cos(theta[..., None] * t), axis=-1)
    if not lumped:
        r = r / ((2.0 + np.cos(theta)) / 3.0)
    return r


def _lex_preceding(radius: int):
    """Relative block positions k with k <_lex 0 (y, then x) and |k|_inf <= radius."""
    ks = [(kx, ky) for ky in range(-radius, 1) for kx in range(-radius, radius + 1) if ky < 0 or kx < 0]
    return np.array(ks, dtype=np.int64)


def schwarz_lex_symbol(p: int, b: int, th: np.ndarray, chunk: int = 2048) -> np.ndarray:
    """Symbol S(theta) of one lexicographic multiplicative Schwarz sweep with
    b x b blocks around every grid point (Section 3.1.1), theta: (..., 2)."""
    a = operator_stencil_2d(p)
    hb = (b - 1) // 2
    offs = np.array([(qx, qy) for qy in range(-hb, hb + 1) for qx in range(-hb, hb + 1)], dtype=np.int64)
    nb = len(offs)

    def aval(d):            # a(d) for an array of offsets d (..., 2), zero outside [-p, p]^2
        inside = (np.abs(d[..., 0]) <= p) & (np.abs(d[..., 1]) <= p)
        dx = np.clip(d[..., 0] + p, 0, 2 * p)
        dy = np.clip(d[..., 1] + p, 0, 2 * p)
        return np.where(inside, a[dy, dx], 0.0)

    AB = aval(offs[None, :, :] - offs[:, None, :])             # [o][q] = a(q - o)
    ks = _lex_preceding(p + 2 * hb)
    G = aval(ks[:, None, None, :] + offs[None, None, :, :] - offs[None, :, None, :])   # [k][o][q]
    shp = th.shape[:-1]
    flat = th.reshape(-1, 2)
    out = np.empty(len(flat), dtype=np.complex128)
    for s in range(0, len(flat), chunk):
        t = flat[s:s + chunk]
        ph = np.exp(1j * (t @ ks.T))                           # (c, K)
        L = np.einsum("ck,koq->coq", ph, G)
        Ahat = _symbol(a, t)                                   # (c,)
        c = Ahat[:, None] * np.exp(1j * (t @ offs.T))          # (c, nb)
        d = -np.linalg.solve(AB[None] + L, c[..., None])[..., 0]
        out[s:s + chunk] = 1.0 + np.sum(d * np.exp(-1j * (t @ offs.T)), axis=-1)
    return out.reshape(shp)


def _grid(n: int, lo: float, hi: float) -> np.ndarray:
    """n x n frequencies in (lo, hi]^2 (cell centres), shape (n, n, 2)."""
    g = lo + (np.arange(n) + 0.5) * (hi - lo) / n
    return np.stack(np.meshgrid(g, g, indexing="xy"), axis=-1)


def _sup(fun, lo: float, hi: float, n: int, refine: int = 3, keep: int = 4) -> float:
    """max of fun over (lo, hi]^2: an n x n grid, then `refine` rounds of a
    9 x 9 grid of a quarter of the previous spacing around each of the `keep`
    best points (the supremum is attained in the interior of a cell)."""
    pts = _grid(n, lo, hi).reshape(-1, 2)
    vals = fun(pts)
    best = float(np.max(vals))
    step = (hi - lo) / n
    for _ in range(refine):
        centres = pts[np.argsort(vals)[-keep:]]
        off = (np.arange(9) - 4) * (step / 4.0)
        loc = np.stack(np.meshgrid(off, off, indexing="xy"), axis=-1).reshape(-1, 2)
        pts = (centres[:, None, :] + loc[None, :, :]).reshape(-1, 2)
        pts = np.clip(pts, lo + 1e-9, hi)
        # theta = 0 is excluded (every coarse correction is exact there; near it
        # the symbols lose their digits to cancellation)
        pts = pts[np.max(np.abs(pts), axis=1) > 1e-3]
        vals = fun(pts)
        best = max(best, float(np.max(vals)))
        step /= 4.0
    return best


def two_grid_symbol(p: int, b: int, th: np.ndarray, lumped: bool = True) -> np.ndarray:
    """T(theta) = (1 - R(theta)^2 A_p(theta) / A_1(theta)) S(theta) (exact
    degree-1 coarse solve on the same grid)."""
    S = schwarz_lex_symbol(p, b, th)
    Ap = _symbol(operator_stencil_2d(p), th).real
    A1 = _symbol(operator_stencil_2d(1), th).real
    R = restriction_symbol_1d(p, th[..., 0], lumped) * restriction_symbol_1d(p, th[..., 1], lumped)
    return (1.0 - R * R * Ap / A1) * S


def rho_2g(p: int, b: int = 0, n: int = 48, lumped: bool = True) -> float:
    """Two-grid factor (Table 1): sup |T(theta)| over theta in (-pi, pi]^2."""
    b = b or block_width_for(p)
    return _sup(lambda th: np.abs(two_grid_symbol(p, b, th, lumped)), -np.pi, np.pi, n)


def _harmonics(th00: np.ndarray) -> np.ndarray:
    """The four 2h-harmonics theta + pi (ax, ay), shape (..., 4, 2)."""
    alpha = np.array([(0, 0), (1, 0), (0, 1), (1, 1)], dtype=np.float64) * np.pi
    return th00[..., None, :] + alpha


def _two_grid_q1(th4: np.ndarray, nu1: int, nu2: int) -> np.ndarray:
    """4x4 symbol of the degree-1 two-grid cycle h -> 2h with nu1 / nu2 red-black
    Gauss-Seidel steps (red first), linear interpolation P0, restriction P0^T,
    Galerkin 2h operator (the degree-1 operator on 2h)."""
    a1 = operator_stencil_2d(1)
    A1 = _symbol(a1, th4).real                                  # (..., 4)
    pw = np.prod((1.0 + np.cos(th4)) / 2.0, axis=-1)            # P0 per harmonic
    rw = np.prod(1.0 + np.cos(th4), axis=-1)                    # P0^T per harmonic
    A2h = np.sum(rw * A1 * pw, axis=-1)
    eye = np.eye(4)
    K = eye - pw[..., :, None] * (rw * A1)[..., None, :] / A2h[..., None, None]
    J = np.zeros((4, 4))
    for i, j in ((0, 3), (3, 0), (1, 2), (2, 1)):                # theta <-> theta + (pi, pi)
        J[i, j] = 1.0
    D = A1 / a1[1, 1]
    red = eye - 0.5 * (eye + J) * D[..., None, :]
    black = eye - 0.5 * (eye - J) * D[..., None, :]
    S1 = black @ red
    M = K
    for _ in range(nu1):
        M = M @ S1
    for _ in range(nu2):
        M = S1 @ M
    return M


def three_grid_symbol(p: int, b: int, th00: np.ndarray, nu1: int = 1, nu2: int = 1,
                      lumped: bool = True) -> np.ndarray:
    """4x4 symbol [I - P (I - M2) A_1^{-1} R A_p] S on the 2h-harmonics of th00."""
    th4 = _harmonics(th00)
    S = schwarz_lex_symbol(p, b, th4)
    Ap = _symbol(operator_stencil_2d(p), th4).real
    A1 = _symbol(operator_stencil_2d(1), th4).real
    R = restriction_symbol_1d(p, th4[..., 0], lumped) * restriction_symbol_1d(p, th4[..., 1], lumped)
    M2 = _two_grid_q1(th4, nu1, nu2)
    eye = np.eye(4)
    C = eye - R[..., :, None] * (eye - M2) * (R * Ap / A1)[..., None, :]
    return C * S[..., None, :]


def aggressive_symbol(p: int, b: int, th00: np.ndarray, lumped: bool = True) -> np.ndarray:
    """4x4 symbol [I - P A_2h^{-1} R A_p] S of aggressive coarsening: R = P0^T
    I_p^1, P = I_1^p P0, A_2h the Galerkin (= rediscretised) degree-1 operator."""
    th4 = _harmonics(th00)
    S = schwarz_lex_symbol(p, b, th4)
    Ap = _symbol(operator_stencil_2d(p), th4).real
    A1 = _symbol(operator_stencil_2d(1), th4).real
    R = restriction_symbol_1d(p, th4[..., 0], lumped) * restriction_symbol_1d(p, th4[..., 1], lumped)
    pw = np.prod((1.0 + np.cos(th4)) / 2.0, axis=-1)
    rw = np.prod(1.0 + np.cos(th4), axis=-1)
    A2h = np.sum(rw * A1 * pw, axis=-1)
    u = R * pw
    w = rw * R * Ap
    return (np.eye(4) - u[..., :, None] * w[..., None, :] / A2h[..., None, None]) * S[..., None, :]


def _spectral_radius(M: np.ndarray) -> np.ndarray:
    return np.max(np.abs(np.linalg.eigvals(M)), axis=-1)


def rho_3g(p: int, b: int = 0, nu1: int = 1, nu2: int = 1, n: int = 24, lumped: bool = True) -> float:
    """Three-grid factor (Table 2): sup over theta in (-pi/2, pi/2]^2 of the
    spectral radius of the 4x4 three-grid symbol."""
    b = b or block_width_for(p)
    return _sup(lambda th: _spectral_radius(three_grid_symbol(p, b, th, nu1, nu2, lumped)),
                -np.pi / 2, np.pi / 2, n)


def rho_2g_ag(p: int, b: int = 0, n: int = 24, lumped: bool = True) -> float:
    """Two-grid factor of aggressive coarsening (Table 3)."""
    b = b or block_width_for(p)
    return _sup(lambda th: _spectral_radius(aggressive_symbol(p, b, th, lumped)), -np.pi / 2, np.pi / 2, n)
