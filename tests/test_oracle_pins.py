"""Pins of the CPU oracle against facts fixed by the paper and by mathematics.

None of these tests re-types the oracle's own formulas: each compares it with a
library routine, a closed form, an invariant, a brute-force dense computation or
a number printed in the paper (arXiv:2009.01499).
"""
import math
from fractions import Fraction

import numpy as np
import pytest
import scipy.interpolate
import scipy.linalg

import oracle as O
import synth


def setup_module(module):
    O.build(force=False)


# ------------------------------------------------------------------ basis --
def test_gauss_legendre_matches_numpy():
    for q in range(1, 12):
        x, w = O.gauss_legendre(q)
        xr, wr = np.polynomial.legendre.leggauss(q)
        assert np.allclose(x, xr, atol=1e-15, rtol=0)
        assert np.allclose(w, wr, atol=1e-14, rtol=0)


@pytest.mark.parametrize("p", [1, 2, 3, 5, 8])
def test_bspline_matches_scipy_and_partition_of_unity(p):
    """Cox-de Boor values (Section 2.1) against scipy's B-spline evaluation."""
    m = 7
    t = O.knots(p, m)
    assert len(t) == 2 * p + m + 1
    assert np.all(t[:p + 1] == 0) and np.all(t[-p - 1:] == 1)
    xs = np.linspace(0.0, 1.0, 53, endpoint=False) + 0.003
    nb = m + p
    for x in xs:
        vals = np.array([O.bspline(t, p, i, x) for i in range(nb)])
        ders = np.array([O.bspline_deriv(t, p, i, x) for i in range(nb)])
        ref = np.array([scipy.interpolate.BSpline(t, np.eye(nb)[i], p)(x) for i in range(nb)])
        dref = np.array([scipy.interpolate.BSpline(t, np.eye(nb)[i], p).derivative()(x) for i in range(nb)])
        assert np.allclose(vals, ref, atol=1e-14)
        assert np.allclose(ders, dref, atol=1e-11 * m)
        assert abs(vals.sum() - 1.0) < 1e-14           # partition of unity
        assert abs(ders.sum()) < 1e-10 * m             # derivative of a constant


def test_dimension_of_dirichlet_space():
    """dim S_h^p = p + m - 2 (Section 2.1)."""
    for p in (1, 2, 3, 4, 7):
        for m in (3, 8, 13):
            A = O.assemble(1, p, m)
            assert A.shape[0] == p + m - 2


# ------------------------------------------------------ assembly closed forms --
def cardinal_bspline(n: int, x: Fraction) -> Fraction:
    """Centred cardinal B-spline of degree n (support [-(n+1)/2, (n+1)/2]),
    (1/n!) sum_j (-1)^j C(n+1,j) (x + (n+1)/2 - j)_+^n, in exact arithmetic."""
    s = Fraction(0)
    for j in range(n + 2):
        y = x + Fraction(n + 1, 2) - j
        if y > 0:
            s += (-1) ** j * math.comb(n + 1, j) * y ** n
    return s / math.factorial(n)


@pytest.mark.parametrize("p", [1, 2, 3, 4, 5])
def test_interior_1d_stencils_closed_form(p):
    """Away from the boundary the 1-D mass row is h B_{2p+1}(k) and the stiffness
    row is -(1/h)[B_{2p-1}(k+1) - 2 B_{2p-1}(k) + B_{2p-1}(k-1)], k=-p..p
    (convolutions of centred cardinal B-splines)."""
    m = 6 * p + 6
    h = 1.0 / m
    K = O.assemble(1, p, m, kind="stiff")
    M = O.assemble(1, p, m, kind="mass")
    row = m // 2
    for k in range(-p, p + 1):
        mref = h * float(cardinal_bspline(2 * p + 1, Fraction(k)))
        if p >= 1:
            b = lambda x: cardinal_bspline(2 * p - 1, Fraction(x)) if 2 * p - 1 >= 0 else 0
            kref = -(1.0 / h) * float(b(k + 1) - 2 * b(k) + b(k - 1))
        assert abs(M[row, k + p] - mref) < 1e-15
        assert abs(K[row, k + p] - kref) < 1e-12 * m


def test_explicit_rational_stencils():
    """p=1: K=(1/h)[-1,2,-1], M=(h/6)[1,4,1]; p=2: K h=[-1/6,-1/3,1,-1/3,-1/6],
    M/h=[1/120,13/60,11/20,13/60,1/120]; p=3: centre K h = 2/3, M/h = 151/315."""
    m = 20
    h = 1.0 / m
    K1 = O.assemble(1, 1, m, kind="stiff")
    M1 = O.assemble(1, 1, m, kind="mass")
    assert np.allclose(K1[9] * h, [-1, 2, -1], atol=1e-13)
    assert np.allclose(M1[9] / h, [1 / 6, 4 / 6, 1 / 6], atol=1e-14)
    K2 = O.assemble(1, 2, m, kind="stiff")
    M2 = O.assemble(1, 2, m, kind="mass")
    assert np.allclose(K2[9] * h, [-1 / 6, -1 / 3, 1, -1 / 3, -1 / 6], atol=1e-13)
    assert np.allclose(M2[9] / h, [1 / 120, 13 / 60, 11 / 20, 13 / 60, 1 / 120], atol=1e-14)
    K3 = O.assemble(1, 3, m, kind="stiff")
    M3 = O.assemble(1, 3, m, kind="mass")
    assert abs(K3[9, 3] * h - 2 / 3) < 1e-13
    assert abs(M3[9, 3] / h - 151 / 315) < 1e-14
    # 2-D Q1 stencil: 8/3 at the centre, -1/3 for all eight neighbours
    A = O.assemble(2, 1, 8)
    c = 3 * 7 + 3
    assert np.allclose(A[c], [-1 / 3] * 4 + [8 / 3] + [-1 / 3] * 4, atol=1e-14)


@pytest.mark.parametrize("d,p", [(1, 3), (2, 2), (2, 3), (3, 2)])
def test_neumann_row_sums_and_mass_total(d, p):
    """Without Dirichlet reduction the stiffness annihilates constants (row sums
    0) and the mass entries sum to the domain measure 1."""
    m = 4
    K = O.assemble(d, p, m, kind="stiff", dirichlet=False)
    M = O.assemble(d, p, m, kind="mass", dirichlet=False)
    assert np.abs(K.sum(axis=1)).max() < 1e-12
    assert abs(M.sum() - 1.0) < 1e-13


@pytest.mark.parametrize("p", [1, 2, 3])
def test_tensor_structure_2d_3d(p):
    """Brute-force 2-D/3-D quadrature equals the Kronecker forms K(x)M + M(x)K
    (and the three-term 3-D analogue) built from 1-D assembly."""
    m = 4
    n1 = m + p - 2
    K = O.offsets_to_dense(O.assemble(1, p, m, kind="stiff"), 1, n1, p)
    M = O.offsets_to_dense(O.assemble(1, p, m, kind="mass"), 1, n1, p)
    A2 = O.offsets_to_dense(O.assemble(2, p, m), 2, n1, p)
    # x fastest: index = ix + n1*iy  ->  kron(Y-factor, X-factor)
    assert np.allclose(A2, np.kron(M, K) + np.kron(K, M), atol=1e-13)
    A3 = O.offsets_to_dense(O.assemble(3, p, m), 3, n1, p)
    ref3 = np.kron(np.kron(M, M), K) + np.kron(np.kron(M, K), M) + np.kron(np.kron(K, M), M)
    assert np.allclose(A3, ref3, atol=1e-13)


def test_stiffness_spd_and_kappa_linearity():
    d, p, m = 2, 3, 5
    n1 = m + p - 2
    A = O.offsets_to_dense(O.assemble(d, p, m), d, n1, p)
    assert np.allclose(A, A.T, atol=1e-14)
    assert np.linalg.eigvalsh(A).min() > 0
    kap = synth.kappa_grf(d, m, 1.0, 0.2, seed=3)
    Ak = O.offsets_to_dense(O.assemble(d, p, m, kappa=kap), d, n1, p)
    # A(kappa) = sum_e kappa_e A(e_e): assemble with one unit element at a time
    acc = np.zeros_like(Ak)
    for e in range(m ** d):
        ke = np.zeros(m ** d)
        ke[e] = 1.0
        acc += kap[e] * O.offsets_to_dense(O.assemble(d, p, m, kappa=ke), d, n1, p)
    assert np.allclose(acc, Ak, atol=1e-12)
    assert np.linalg.eigvalsh(Ak).min() > 0


@pytest.mark.parametrize("p", [2, 3, 4])
def test_manufactured_l2_convergence_order(p):
    """Manufactured problem of Section 5.1: ||u - u_h||_L2 = O(h^{p+1})."""
    errs = []
    ms = (6, 12, 24)
    for m in ms:
        P = O.Problem(2, p, m)
        b = O.load_manufactured(2, p, m)
        u = P.direct_solve(b)
        errs.append(O.l2_error_manufactured(2, p, m, u))
    rates = [math.log(errs[i] / errs[i + 1], 2) for i in range(len(ms) - 1)]
    assert abs(rates[-1] - (p + 1)) < 0.3, (errs, rates)


# ------------------------------------------------------- Schwarz smoother --
def _dense_problem(d, p, m, bw, kappa=None):
    P = O.Problem(d, p, m, block_width=bw, kappa=kappa)
    A = O.offsets_to_dense(P.A(), d, P.n1, p)
    return P, A


def _block_members(d, n1, bw, j):
    hb = (bw - 1) // 2
    jx = [(j // n1 ** k) % n1 for k in range(d)]
    mem = []
    for w in range(bw ** d):
        o = [(w // bw ** k) % bw - hb for k in range(d)]
        kx = [jx[k] + o[k] for k in range(d)]
        if all(0 <= v < n1 for v in kx):
            mem.append(sum(kx[k] * n1 ** k for k in range(d)))
    return mem


def test_sweep_lex_equals_product_formula():
    """Lexicographic sweep = the product of (I - V_j^T (A^{B_j})^{-1} V_j A)
    over the blocks (Section 3.1.1), built densely."""
    d, p, m, bw = 2, 3, 4, 3
    P, A = _dense_problem(d, p, m, bw)
    n = P.n
    b = synth.rhs_normal(d, p, m, seed=5)
    u0 = synth.initial_guess(d, p, m, seed=6)
    u = u0.copy()
    for j in range(n):          # block j applied j-th
        V = np.eye(n)[_block_members(d, P.n1, bw, j)]
        AB = V @ A @ V.T
        u = u + V.T @ np.linalg.solve(AB, V @ (b - A @ u))
    assert np.allclose(P.sweep(u0, b, ordering=O.LEX), u, atol=1e-12, rtol=0)
    # iteration-matrix form: e' = prod (I - V^T AB^{-1} V A) e
    E = np.eye(n)
    for j in range(n):
        V = np.eye(n)[_block_members(d, P.n1, bw, j)]
        E = (np.eye(n) - V.T @ np.linalg.solve(V @ A @ V.T, V @ A)) @ E
    us = np.linalg.solve(A, b)
    assert np.allclose(P.sweep(u0, b, ordering=O.LEX) - us, E @ (u0 - us), atol=1e-10)


def test_sweep_point_block_is_gauss_seidel():
    """Block width 1 reduces the lexicographic sweep to point Gauss-Seidel:
    u' = u + (D+L)^{-1}(b - A u)."""
    d, p, m = 2, 2, 5
    P, A = _dense_problem(d, p, m, 1)
    b = synth.rhs_normal(d, p, m, seed=1)
    u0 = synth.initial_guess(d, p, m, seed=2)
    ref = u0 + scipy.linalg.solve_triangular(np.tril(A), b - A @ u0, lower=True)
    assert np.allclose(P.sweep(u0, b, ordering=O.LEX), ref, atol=1e-12)


def test_sweep_with_global_block_is_exact_solve():
    """If every block covers the whole grid, the first local solve is the exact
    solution and the sweep returns A^{-1} b."""
    d, p, m = 2, 3, 3
    n1 = m + p - 2
    bw = 2 * n1 + 1
    P, A = _dense_problem(d, p, m, bw)
    b = synth.rhs_normal(d, p, m, seed=1)
    u0 = synth.initial_guess(d, p, m, seed=2)
    assert np.allclose(P.sweep(u0, b, ordering=O.LEX), np.linalg.solve(A, b), atol=1e-12)


@pytest.mark.parametrize("extra", [0, 3])
def test_coloured_sweep_definition(extra):
    """Coloured ordering with period s: classes c = sum (j_k mod s) s^k in order;
    inside a class every correction is computed from the class-start iterate.
    Brute-force dense version of that statement."""
    d, p, m, bw = 2, 3, 7, 3
    s = bw + extra
    P, A = _dense_problem(d, p, m, bw)
    n, n1 = P.n, P.n1
    b = synth.rhs_normal(d, p, m, seed=8)
    u0 = synth.initial_guess(d, p, m, seed=9)
    u = u0.copy()
    for c in range(s ** d):
        cls = [j for j in range(n) if sum(((j // n1 ** k) % n1 % s) * s ** k for k in range(d)) == c]
        r = b - A @ u
        du = np.zeros(n)
        for j in cls:
            V = np.eye(n)[_block_members(d, n1, bw, j)]
            du += V.T @ np.linalg.solve(V @ A @ V.T, V @ r)
        u = u + du
    assert np.allclose(P.sweep(u0, b, ordering=O.COLOUR, s=s), u, atol=1e-12)


def test_coloured_sweep_with_decoupled_classes_is_sequential():
    """With s = b + p the blocks of a class do not interact, so the coloured
    sweep equals the sequential multiplicative sweep in colour-major order."""
    d, p, m, bw = 2, 2, 9, 3
    s = bw + p
    P, A = _dense_problem(d, p, m, bw)
    n, n1 = P.n, P.n1
    b = synth.rhs_normal(d, p, m, seed=3)
    u0 = synth.initial_guess(d, p, m, seed=4)
    order = sorted(range(n), key=lambda j: (sum(((j // n1 ** k) % n1 % s) * s ** k for k in range(d)), -j))
    u = u0.copy()
    for j in order:           # reversed order inside a class on purpose
        V = np.eye(n)[_block_members(d, n1, bw, j)]
        u = u + V.T @ np.linalg.solve(V @ A @ V.T, V @ (b - A @ u))
    assert np.allclose(P.sweep(u0, b, ordering=O.COLOUR, s=s), u, atol=1e-12)


# -------------------------------------------------------------- transfers --
@pytest.mark.parametrize("p", [2, 3, 4, 5])
def test_restriction_closed_form_and_adjoint(p):
    """R = D^{-1} M_p^{plow} with lumped D: interior rows of the 1-D factor are
    samples B_{p+2}((x_i - c_j)/h) of the cardinal B-spline (hat * B_p), row
    sums are 1 away from the boundary; the lumped first/last entries are 5h/6;
    the prolongation is exactly the transpose (Section 3.1.2)."""
    m = 4 * p + 8
    h = 1.0 / m
    P1 = O.Problem(1, p, m)
    D = P1.Dlump()
    assert abs(D[0] - 5 * h / 6) < 1e-15 and abs(D[-1] - 5 * h / 6) < 1e-15
    assert np.allclose(D[1:-1], h, atol=1e-15)
    nc, n = P1.nc, P1.n
    R = np.stack([P1.restrict(np.eye(n)[j]) for j in range(n)], axis=1)
    Pm = np.stack([P1.prolong_add(np.eye(nc)[I], np.zeros(n)) for I in range(nc)], axis=1)
    assert np.allclose(Pm, R.T, rtol=1e-15, atol=1e-17)
    for I in range(p + 1, nc - p - 1):          # rows touching uniform functions only
        xI = (I + 1) * h
        for j in range(n):
            cj = (j + 1 - p + (p + 1) / 2.0) * h  # centre of the support of full function j+1
            ref = float(cardinal_bspline(p + 2, Fraction((xI - cj) / h).limit_denominator(1000)))
            assert abs(R[I, j] - ref) < 1e-14
        assert abs(R[I].sum() - 1.0) < 1e-14
    # 2-D restriction is the Kronecker product of 1-D ones
    P2 = O.Problem(2, p, 6)
    P1s = O.Problem(1, p, 6)
    R1 = np.stack([P1s.restrict(np.eye(P1s.n)[j]) for j in range(P1s.n)], axis=1)
    R2 = np.stack([P2.restrict(np.eye(P2.n)[j]) for j in range(P2.n)], axis=1)
    assert np.allclose(R2, np.kron(R1, R1), atol=1e-15)


@pytest.mark.parametrize("p", [2, 3, 4, 5, 6])
def test_mixed_mass_polynomial_reproduction(p):
    """Every row of M_p^1, the rows next to the boundary included, through an
    identity that holds for any polynomial g of degree <= p vanishing at 0 and
    1: g lies in the degree-p spline space, its B-spline coefficients at the
    two ends are g(0) = g(1) = 0 (open knot vector), so with c the interior
    coefficients, sum_j (M_p^1)_{Ij} c_j = integral of phi_I^1 g (Section
    3.1.2, definition of M_p^{p_low}).  The coefficients come from scipy's
    spline interpolation at the Greville abscissae, the integrals from Gauss
    rules on the two elements of each hat; 1-D and the 2-D tensor case."""
    from scipy.interpolate import make_interp_spline
    m = 9
    h = 1.0 / m
    t = np.r_[np.zeros(p + 1), np.arange(1, m) / m, np.ones(p + 1)]
    tau = np.array([t[i + 1:i + p + 1].mean() for i in range(m + p)])
    xg, wg = np.polynomial.legendre.leggauss(p + 3)

    def hat_integral(g, I):        # interior hat I, centred at node (I+1) h
        xc = (I + 1) * h
        tot = 0.0
        for a, bnd in ((xc - h, xc), (xc, xc + h)):
            x = 0.5 * (bnd - a) * xg + 0.5 * (a + bnd)
            tot += 0.5 * (bnd - a) * np.sum(wg * g(x) * (1.0 - np.abs(x - xc) / h))
        return tot

    M1 = O.mix_to_dense(O.assemble_mix(1, p, 1, m), 1, p, 1, m)
    M2 = O.mix_to_dense(O.assemble_mix(2, p, 1, m), 2, p, 1, m)
    for k in range(p - 1):
        def g(x, k=k):
            return x * (1.0 - x) * (x - 0.3) ** k
        c = make_interp_spline(tau, g(tau), k=p, t=t).c
        assert abs(c[0]) < 1e-13 and abs(c[-1]) < 1e-13
        ci = c[1:-1]
        want = np.array([hat_integral(g, I) for I in range(m - 1)])
        assert np.allclose(M1 @ ci, want, rtol=0, atol=1e-14 * np.abs(want).max()), (p, k)
        assert np.allclose(M2 @ np.outer(ci, ci).ravel(), np.outer(want, want).ravel(), rtol=0,
                           atol=1e-14 * np.abs(want).max() ** 2), (p, k)


@pytest.mark.parametrize("p", [2, 3, 5])
def test_mixed_mass_degree2_polynomial_reproduction(p):
    """Every row of M_p^2 (the degree-2 coarse space of Section 5): for a
    polynomial g of degree <= p vanishing at 0 and 1, M_p^2 c = (phi_I^2, g)
    with c its interior degree-p B-spline coefficients; the degree-2 basis
    functions and the integrals come from scipy's B-spline elements and Gauss
    rules on every element."""
    from scipy.interpolate import BSpline, make_interp_spline
    m = 8
    t = np.r_[np.zeros(p + 1), np.arange(1, m) / m, np.ones(p + 1)]
    tau = np.array([t[i + 1:i + p + 1].mean() for i in range(m + p)])
    t2 = np.r_[np.zeros(3), np.arange(1, m) / m, np.ones(3)]
    xg, wg = np.polynomial.legendre.leggauss(p + 4)
    M2 = O.mix_to_dense(O.assemble_mix(1, p, 2, m), 1, p, 2, m)
    assert M2.shape == (m, m + p - 2)
    for k in range(p - 1):
        def g(x, k=k):
            return x * (1.0 - x) * (x - 0.3) ** k
        c = make_interp_spline(tau, g(tau), k=p, t=t).c[1:-1]
        want = np.zeros(m)
        for I in range(m):                       # interior degree-2 function I = full index I + 1
            phi = BSpline.basis_element(t2[I + 1:I + 5], extrapolate=False)
            for e in range(m):
                a, b = e / m, (e + 1) / m
                x = 0.5 * (b - a) * xg + 0.5 * (a + b)
                want[I] += 0.5 * (b - a) * np.sum(wg * np.nan_to_num(phi(x)) * g(x))
        assert np.allclose(M2 @ c, want, rtol=0, atol=1e-14 * np.abs(want).max()), (p, k)


@pytest.mark.parametrize("lumped", [True, False])
def test_degree2_coarse_cycle_dense(lumped):
    """The two-level cycle with the degree-2 coarse space (plow = 2, exact
    coarse solve): after the sweep, u1 = u_s + R^T A_2^{-1} R (b - A u_s) with
    R = D^{-1} M_p^2 (lumped: row sums of the degree-2 mass matrix) or
    M_2^{-1} M_p^2, built densely from the oracle's assembled matrices."""
    d, p, m = 2, 3, 6
    P = O.Problem(d, p, m, plow=2, lumped=lumped)
    A = O.offsets_to_dense(P.A(), d, P.n1, p)
    A2 = O.offsets_to_dense(P.Alow(), d, P.n1c, 2)
    M2 = O.offsets_to_dense(P.Mlow(), d, P.n1c, 2)
    Mmix = O.mix_to_dense(P.Mmix(), d, p, 2, m)
    assert np.allclose(P.Dlump(), M2.sum(axis=1), atol=1e-15)
    R = Mmix / P.Dlump()[:, None] if lumped else np.linalg.solve(M2, Mmix)
    b = synth.rhs_normal(d, p, m, seed=41)
    u0 = synth.initial_guess(d, p, m, seed=42)
    us = P.sweep(u0, b, ordering=O.COLOUR)
    ref = us + R.T @ np.linalg.solve(A2, R @ (b - A @ us))
    got = P.cycle(u0, b, ordering=O.COLOUR, coarse=O.DIRECT)
    assert np.allclose(got, ref, rtol=0, atol=1e-12 * np.abs(ref).max())


def test_seven_by_seven_sweep_sensitivity():
    """The 7x7-block sweep (p = 7) of the oracle against the same sweep carried
    out in extended precision (numpy longdouble, Gaussian elimination) on the
    oracle's operator: agreement to 1e-13.  The same exact sweep on an equally
    valid FP64 assembly of A (Kronecker products of the oracle's 1-D matrices,
    within ~1e-15 of the quadrature-assembled entries) differs by more than
    1e-12: blocks with condition numbers ~1e4 amplify last-bit differences of
    the operator, which sets the GPU parity bar for 7x7 blocks (5e-11)."""
    d, p, m = 2, 7, 14
    P = O.Problem(d, p, m)
    bw, n1, n = P.block_width, P.n1, P.n
    A = O.offsets_to_dense(P.A(), d, n1, p)
    K1 = O.offsets_to_dense(O.assemble(1, p, m, kind="stiff"), 1, n1, p)
    M1 = O.offsets_to_dense(O.assemble(1, p, m, kind="mass"), 1, n1, p)
    Ak = np.kron(M1, K1) + np.kron(K1, M1)
    assert np.max(np.abs(A - Ak)) <= 5e-15 * np.max(np.abs(A))
    u0 = synth.initial_guess(d, p, m, seed=1)
    b = synth.rhs_normal(d, p, m, seed=0)
    members = [_block_members(d, n1, bw, j) for j in range(n)]

    def ge_solve(Mx, r):
        Mx, r = Mx.copy(), r.copy()
        k = len(r)
        for i in range(k):
            f = Mx[i + 1:, i] / Mx[i, i]
            Mx[i + 1:, i:] -= np.outer(f, Mx[i, i:])
            r[i + 1:] -= f * r[i]
        x = np.zeros_like(r)
        for i in range(k - 1, -1, -1):
            x[i] = (r[i] - Mx[i, i + 1:] @ x[i + 1:]) / Mx[i, i]
        return x

    def exact_sweep(Aop):
        Al = Aop.astype(np.longdouble)
        u, bl = u0.astype(np.longdouble), b.astype(np.longdouble)
        for c in range(bw * bw):
            r = bl - Al @ u
            du = np.zeros_like(u)
            for j in range(n):
                if (j % n1) % bw + bw * ((j // n1) % bw) == c:
                    I = members[j]
                    du[I] += ge_solve(Al[np.ix_(I, I)], r[I])
            u = u + du
        return u

    ext = exact_sweep(A)
    ext_k = exact_sweep(Ak)
    nrm = float(np.linalg.norm(ext))
    e_orc = float(np.linalg.norm(P.sweep(u0, b, ordering=O.COLOUR, s=bw) - ext)) / nrm
    e_asm = float(np.linalg.norm(ext_k - ext)) / nrm
    print(f"oracle vs exact sweep {e_orc:.2e}; exact sweeps on two FP64 assemblies {e_asm:.2e}")
    assert e_orc < 1e-13
    assert 1e-12 < e_asm < 5e-11


def test_exact_mass_inverse_variant():
    """lumped=0 applies (M_{plow}^{plow})^{-1} exactly."""
    d, p, m = 2, 3, 5
    P = O.Problem(d, p, m, lumped=False)
    Mlow = O.offsets_to_dense(P.Mlow(), d, P.n1c, 1)
    Mmix = O.mix_to_dense(P.Mmix(), d, p, 1, m)
    x = synth.rhs_normal(d, p, m, seed=2)
    assert np.allclose(P.restrict(x), np.linalg.solve(Mlow, Mmix @ x), atol=1e-12)


# ---------------------------------------------------------------- coarse --
def test_coarse_direct_matches_dst_closed_form():
    """A_1 = (S (x) S) diag(mu) (S (x) S) with the DST-I matrix
    S_ik = sqrt(2/m) sin(ik pi/m): mu_kl = lK_k lM_l + lM_k lK_l,
    lK = (2/h)(1 - cos t), lM = (h/3)(2 + cos t), t = k pi / m."""
    m = 12
    P = O.Problem(2, 3, m)
    h = 1.0 / m
    k = np.arange(1, m)
    S = np.sqrt(2.0 / m) * np.sin(np.outer(k, k) * np.pi / m)
    th = k * np.pi / m
    lK = (2 / h) * (1 - np.cos(th))
    lM = (h / 3) * (2 + np.cos(th))
    mu = np.outer(lK, lM) + np.outer(lM, lK)        # [ky, kx]
    dc = synth.rhs_normal(2, 1, m, seed=4)
    Dm = dc.reshape(m - 1, m - 1)                   # [iy, ix]
    E = S @ ((S @ Dm @ S) / mu) @ S
    assert np.allclose(P.coarse_direct(dc), E.ravel(), atol=1e-12 * np.abs(E).max())


def test_galerkin_equals_rediscretisation_and_vcycle_rate():
    """P^T A_h P with bilinear P reproduces the Q1 rediscretisation on 2h
    (kappa = 1), and V(1,1) with red-black smoothing contracts like a
    multigrid cycle (factor below 0.3)."""
    m = 64
    P = O.Problem(2, 3, m, vcycle=True)
    assert P.nlevels() == 3                          # 63^2, 31^2, 15^2 (<= 512 unknowns, exact)
    for l in range(1, P.nlevels()):
        ref = O.assemble(2, 1, m >> l)
        assert np.allclose(P.level(l), ref, atol=1e-14)
    A1 = O.offsets_to_dense(P.Alow(), 2, P.n1c, 1)
    rhs = synth.rhs_normal(2, 1, m, seed=1)
    x = np.zeros(P.nc)
    res = [np.linalg.norm(rhs)]
    for _ in range(8):
        x = x + P.coarse_vcycle(rhs - A1 @ x, 1, 1)
        res.append(np.linalg.norm(rhs - A1 @ x))
    rate = (res[-1] / res[2]) ** (1 / 6)
    assert rate < 0.3, res


def _interp_1d(nf):
    """Dense linear-interpolation factor from the odd-indexed fine interior
    nodes (coarse node I = fine node 2I+1) to all nf fine interior nodes."""
    nc = nf // 2
    Pm = np.zeros((nf, nc))
    for I in range(nc):
        Pm[2 * I + 1, I] = 1.0
        Pm[2 * I, I] = 0.5
        if 2 * I + 2 < nf:
            Pm[2 * I + 2, I] = 0.5
    return Pm


@pytest.mark.parametrize("kappa_seed,m", [(None, 64), (5, 64), (5, 63), (None, 50)])
def test_vcycle_matches_dense_brute_force(kappa_seed, m):
    """Dense re-implementation of the V(nu1,nu2) definition (red then black
    points updated simultaneously from the half-step start, linear P onto the
    odd-indexed nodes, Galerkin P^T A P, exact solve on the first level with at
    most 512 unknowns) agrees with the oracle, also for odd m."""
    d = 2
    kap = None if kappa_seed is None else synth.kappa_grf(d, m, 1.0, 0.2, seed=kappa_seed)
    P = O.Problem(d, 2, m, kappa=kap, vcycle=True)
    A0 = O.offsets_to_dense(O.assemble(d, 1, m, kappa=kap), d, m - 1, 1)
    levels = [A0]
    Ps = []
    nn = m - 1
    while nn ** d > 512:
        P1 = _interp_1d(nn)
        Pk = np.kron(P1, P1)
        Ps.append(Pk)
        levels.append(Pk.T @ levels[-1] @ Pk)
        nn //= 2

    def red_black(A, e, f, n1):
        par = np.array([(i % n1 + i // n1) % 2 for i in range(n1 * n1)])
        for colour in (0, 1):
            r = f - A @ e
            e = e + np.where(par == colour, r / np.diag(A), 0.0)
        return e

    def vc(l, f, nu1, nu2):
        A = levels[l]
        if l == len(levels) - 1:
            return np.linalg.solve(A, f)
        n1 = int(round(np.sqrt(A.shape[0])))
        e = np.zeros_like(f)
        for _ in range(nu1):
            e = red_black(A, e, f, n1)
        ec = vc(l + 1, Ps[l].T @ (f - A @ e), nu1, nu2)
        e = e + Ps[l] @ ec
        for _ in range(nu2):
            e = red_black(A, e, f, n1)
        return e

    f = synth.rhs_normal(d, 1, m, seed=3)
    for nu in ((1, 1), (2, 2), (1, 0)):
        assert np.allclose(P.coarse_vcycle(f, *nu), vc(0, f, *nu), atol=1e-12)


def test_vcycle_3d_galerkin():
    m = 16
    P = O.Problem(3, 2, m, vcycle=True, coarse_direct=False)
    for l in range(1, P.nlevels()):
        assert np.allclose(P.level(l), O.assemble(3, 1, m >> l), atol=1e-14)


# ---------------------------------------------------------- two-level cycle --
def test_cycle_error_propagation_matrix():
    """One cycle maps the error by T = (I - P A_c^{-1} R A) S (Section 4.1),
    with S the Schwarz error propagation and P = R^T."""
    d, p, m = 2, 3, 4
    P, A = _dense_problem(d, p, m, 3)
    n, nc = P.n, P.nc
    Ac = O.offsets_to_dense(P.Alow(), d, P.n1c, 1)
    Mmix = O.mix_to_dense(P.Mmix(), d, p, 1, m)
    D = P.Dlump()
    R = Mmix / D[:, None]
    S = np.eye(n)
    for j in range(n):
        V = np.eye(n)[_block_members(d, P.n1, 3, j)]
        S = (np.eye(n) - V.T @ np.linalg.solve(V @ A @ V.T, V @ A)) @ S
    T = (np.eye(n) - R.T @ np.linalg.solve(Ac, R @ A)) @ S
    b = synth.rhs_normal(d, p, m, seed=11)
    u0 = synth.initial_guess(d, p, m, seed=12)
    us = np.linalg.solve(A, b)
    u1 = P.cycle(u0, b, ordering=O.LEX, coarse=O.DIRECT)
    assert np.allclose(u1 - us, T @ (u0 - us), atol=1e-10)


def _golden(name):
    rows = []
    with open(__file__.replace("test_oracle_pins.py", "golden/" + name)) as f:
        for line in f:
            if line.strip() and not line.startswith("#"):
                rows.append([float(v) for v in line.split()])
    return rows


@pytest.mark.slow
@pytest.mark.parametrize("p,m", [(2, 128), (3, 64), (4, 64), (5, 96), (6, 64), (7, 64), (8, 64)])
def test_table1_convergence_factors(p, m):
    """Table 1 (rho_h, exact coarse solve, p_low=1, same h, zero RHS, random
    initial guess): measured here as the geometric-mean residual reduction over
    cycles 10..K of the lexicographic two-level method; agreement within 8%
    (the paper's grid size is not stated; at p = 6..8 the rate measured on
    64x64 is 5-6 % below the paper's and rises with m)."""
    ref = {int(r[0]): (int(r[1]), r[2]) for r in _golden("table1_rho_h.txt")}
    bw, rho_paper = ref[p]
    P = O.Problem(2, p, m, block_width=bw)
    K = 30 if p <= 4 else (25 if p <= 6 else 20)
    u0 = synth.initial_guess(2, p, m, seed=1)
    _, k, hist = P.solve(np.zeros(P.n), u0=u0, ordering=O.LEX, tol=0.0, max_cycles=K)
    est = (hist[K] / hist[10]) ** (1.0 / (K - 10))
    assert abs(est / rho_paper - 1) < 0.08, (est, rho_paper)


def test_vcycle_coarse_matches_exact_coarse_rate():
    """Tables 1-2: approximating the coarse solve by one V(1,1) cycle leaves the
    convergence factor essentially unchanged for p >= 3."""
    p, m = 3, 64
    P = O.Problem(2, p, m, vcycle=True)
    u0 = synth.initial_guess(2, p, m, seed=1)
    z = np.zeros(P.n)
    _, _, h1 = P.solve(z, u0=u0, ordering=O.LEX, coarse=O.DIRECT, tol=0.0, max_cycles=30)
    _, _, h2 = P.solve(z, u0=u0, ordering=O.LEX, coarse=O.VCYCLE, tol=0.0, max_cycles=30)
    r1 = (h1[30] / h1[10]) ** (1 / 20)
    r2 = (h2[30] / h2[10]) ** (1 / 20)
    assert abs(r2 / r1 - 1) < 0.05
    ref = {int(r[0]): r[2] for r in _golden("table2_rho_3g.txt")}
    assert abs(r2 / ref[3] - 1) < 0.08


def test_coloured_iteration_counts_in_paper_band():
    """The configuration of Table 4 (coloured Schwarz sweep, aggressive
    coarsening to degree 1 on 2h with one V(1,1) red-black cycle, random
    initial guess, 1e-8 reduction) reaches the tolerance in a number of cycles
    comparable to the paper's (context band, not an exact target: the paper's
    colouring is not reproducible, Section 3.1.1); the same method without
    aggressive coarsening needs about as many (Section 3.3)."""
    table = _golden("table4_iterations.txt")
    it_paper = {2: table[0][1], 3: table[0][2], 4: table[0][3], 5: table[0][4]}
    for p in (2, 3, 4, 5):
        m = 64
        P = O.Problem(2, p, m, vcycle=True, coarse_direct=False)
        u0 = synth.initial_guess(2, p, m, seed=7)
        _, k, _ = P.solve(np.zeros(P.n), u0=u0, ordering=O.COLOUR, coarse=O.VCYCLE, cnu1=1, cnu2=1,
                          tol=1e-8, max_cycles=60, aggressive=True)
        _, k_same, _ = P.solve(np.zeros(P.n), u0=u0, ordering=O.COLOUR, coarse=O.VCYCLE, cnu1=1, cnu2=1,
                               tol=1e-8, max_cycles=60)
        assert it_paper[p] - 3 <= k <= 3 * it_paper[p], (p, k)
        assert abs(k - k_same) <= 1, (p, k, k_same)


def _interp_1d(n1f):
    """Linear interpolation from the odd-indexed interior nodes (coarse node I
    at fine index 2I+1) of a 1-D grid of n1f interior nodes, zero boundary."""
    n1c = n1f // 2
    P0 = np.zeros((n1f, n1c))
    for I in range(n1c):
        P0[2 * I + 1, I] = 1.0
        P0[2 * I, I] = 0.5
        if 2 * I + 2 < n1f:
            P0[2 * I + 2, I] = 0.5
    return P0


@pytest.mark.parametrize("d,p,m", [(2, 3, 24), (3, 2, 10)])
def test_aggressive_coarse_correction_dense(d, p, m):
    """Aggressive coarsening (Section 3.3), dense statement: after the sweep,
    u1 = u_s + P_p P_0 A_2h^{-1} P_0^T R (b - A u_s), where R, P_p = R^T are the
    degree transfers on h (Section 3.1.2), P_0 the linear interpolation from
    the 2h grid and A_2h = P_0^T A_1 P_0, which for kappa = 1 equals the degree-1
    operator assembled directly on m/2 elements.  With a hierarchy of two
    levels the V-cycle variant solves the 2h level exactly, so it gives the
    same iterate."""
    P = O.Problem(d, p, m, vcycle=True, coarse_direct=False)
    assert P.nlevels() == 2
    A = O.offsets_to_dense(P.A(), d, P.n1, p)
    A1 = O.offsets_to_dense(P.Alow(), d, P.n1c, 1)
    Mmix = O.mix_to_dense(P.Mmix(), d, p, 1, m)
    R = Mmix / P.Dlump()[:, None]
    P1 = _interp_1d(P.n1c)
    P0 = P1
    for _ in range(d - 1):
        P0 = np.kron(P0, P1)
    A2h = P0.T @ A1 @ P0
    A2h_direct = O.offsets_to_dense(O.assemble(d, 1, m // 2), d, m // 2 - 1, 1)
    assert np.allclose(A2h, A2h_direct, atol=1e-13 * np.abs(A2h).max())
    b = synth.rhs_normal(d, p, m, seed=31)
    u0 = synth.initial_guess(d, p, m, seed=32)
    us = P.sweep(u0, b, ordering=O.COLOUR)
    ref = us + R.T @ (P0 @ np.linalg.solve(A2h, P0.T @ (R @ (b - A @ us))))
    got = P.cycle(u0, b, ordering=O.COLOUR, coarse=O.DIRECT, aggressive=True)
    assert np.allclose(got, ref, rtol=0, atol=1e-12 * np.abs(ref).max())
    got_v = P.cycle(u0, b, ordering=O.COLOUR, coarse=O.VCYCLE, cnu1=2, cnu2=1, aggressive=True)
    assert np.allclose(got_v, ref, rtol=0, atol=1e-12 * np.abs(ref).max())


@pytest.mark.slow
def test_table3_aggressive_rates():
    """Table 3 (rho_2g^ag: degree 1 on 2h, exact coarse solve): the measured
    rate of the lexicographic method with aggressive coarsening on 64x64
    elements is within 8 % of the LFA prediction for p = 3, 4, 5.  At p = 2 the
    measured rate stays below the prediction and rises with m (0.09, 0.14,
    0.14 on 64, 128, 256 elements): the infinite-grid analysis is pessimistic
    there; checked as a band at m = 128.  One V(1,1) cycle on the 2h level
    gives the same rate as the exact 2h solve (p = 3)."""
    ref = {int(r[0]): (int(r[1]), r[2]) for r in _golden("table3_rho_ag.txt")}
    for p, m, lo, hi in [(3, 64, 0.92, 1.08), (4, 64, 0.92, 1.08), (5, 64, 0.92, 1.08), (2, 128, 0.7, 1.0)]:
        bw, rho_lfa = ref[p]
        P = O.Problem(2, p, m, block_width=bw, vcycle=True, coarse_direct=False)
        K = 30 if p <= 4 else 25
        u0 = synth.initial_guess(2, p, m, seed=1)
        _, _, hist = P.solve(np.zeros(P.n), u0=u0, ordering=O.LEX, coarse=O.DIRECT, aggressive=True, tol=0.0,
                             max_cycles=K)
        est = (hist[K] / hist[10]) ** (1.0 / (K - 10))
        assert lo < est / rho_lfa < hi, (p, est, rho_lfa)
        if p == 3:
            _, _, hv = P.solve(np.zeros(P.n), u0=u0, ordering=O.LEX, coarse=O.VCYCLE, aggressive=True, tol=0.0,
                               max_cycles=K)
            est_v = (hv[K] / hv[10]) ** (1.0 / (K - 10))
            assert abs(est_v / est - 1) < 0.02, (est_v, est)


def test_solution_matches_direct_solve():
    """The fixed point of the cycle is A^{-1} b: after reaching tol the error
    is within the bound cond(A) * tol (generous constant)."""
    p, m = 3, 32
    P = O.Problem(2, p, m)
    b = synth.rhs_normal(2, p, m, seed=0)
    u, k, hist = P.solve(b, ordering=O.COLOUR, coarse=O.DIRECT, tol=1e-10)
    assert hist[-1] <= 1e-10 * hist[0]
    us = P.direct_solve(b)
    A = O.offsets_to_dense(P.A(), 2, P.n1, p)
    assert np.allclose(A @ us, b, atol=1e-10)
    assert np.linalg.norm(u - us) / np.linalg.norm(us) < 1e-10 * 1e4


# ---------------------------------------------------------------- adjoint --
def test_gradient_identities_and_finite_differences():
    """For L = 0.5||u - u_obs||^2 with A(kappa) u = b:
    (i) Euler identity sum_e kappa_e g_e = -lambda^T A u (A linear in kappa);
    (ii) central finite differences of L in kappa_e."""
    d, p, m = 2, 3, 5
    kap = synth.kappa_grf(d, m, 0.5, 0.3, seed=1)
    kap_obs = synth.kappa_grf(d, m, 0.5, 0.3, seed=2)
    b = synth.rhs_normal(d, p, m, seed=0)
    P = O.Problem(d, p, m, kappa=kap)
    u = P.direct_solve(b)
    u_obs = O.Problem(d, p, m, kappa=kap_obs).direct_solve(b)
    lam = P.direct_solve(u - u_obs)
    g = P.grad_kappa(u, lam)
    assert abs(np.dot(kap, g) + lam @ P.apply_A(u)) < 1e-12 * abs(lam @ P.apply_A(u))

    def loss(kv):
        uu = O.Problem(d, p, m, kappa=kv).direct_solve(b)
        return 0.5 * np.sum((uu - u_obs) ** 2)

    for e in (0, 7, 13, 24):
        eps = 1e-5 * kap[e]
        kp, km = kap.copy(), kap.copy()
        kp[e] += eps
        km[e] -= eps
        fd = (loss(kp) - loss(km)) / (2 * eps)
        assert abs(fd - g[e]) <= 1e-6 * abs(g).max(), (e, fd, g[e])


def test_kappa_element_order_is_x_fastest():
    """kappa[e] with e = ex + m*ey: raising the coefficient of the element in the
    top-left corner (ex=0, ey=m-1) changes only rows whose support touches it."""
    d, p, m = 2, 2, 6
    n1 = m + p - 2
    A1 = O.assemble(d, p, m)
    kap = np.ones(m * m)
    kap[0 + m * (m - 1)] = 1000.0
    Ak = O.assemble(d, p, m, kappa=kap)
    changed = np.abs(Ak - A1).max(axis=1) > 1e-9
    top_left = 0 + n1 * (n1 - 1)
    bottom_right = (n1 - 1) + 0
    assert changed[top_left] and not changed[bottom_right]
    # DOF (ix, iy) is supported on elements ex in [ix+1-p, ix+1]: only ix <= p-1 rows change
    for i in np.nonzero(changed)[0]:
        ix, iy = i % n1, i // n1
        assert ix <= p - 1 and iy >= n1 - p


def test_element_operator_sums_to_assembled_operator():
    """sum_e kappa_e A_e u = A(kappa) u, and g_e = -lambda^T A_e u agrees with
    the gradient routine (two independent element loops)."""
    d, p, m = 2, 3, 5
    kap = synth.kappa_grf(d, m, 1.0, 0.3, seed=4)
    P = O.Problem(d, p, m, kappa=kap)
    u = synth.initial_guess(d, p, m, seed=1)
    lam = synth.initial_guess(d, p, m, seed=2)
    acc = np.zeros(P.n)
    g = np.zeros(P.ne)
    for e in range(P.ne):
        Aeu = P.element_apply(e, u)
        acc += kap[e] * Aeu
        g[e] = -lam @ Aeu
    assert np.allclose(acc, P.apply_A(u), atol=1e-12)
    assert np.allclose(g, P.grad_kappa(u, lam), atol=1e-12)


# ------------------------------------------------------------- annulus --
def test_annulus_map_is_the_rational_quadratic_arc():
    """Sections 2.2 and 5.2: the oracle's map F(xi, eta) = rho(eta) (c, s)(xi)
    is the quadratic NURBS curve with control points (1,0), (1,1), (0,1) and
    weights 1, sqrt(2)/2, 1 (evaluated here with scipy's B-splines as
    sum w_i P_i N_i / sum w_i N_i), scaled to the radius rho = r + (R-r) eta;
    every image point lies on that circle."""
    from scipy.interpolate import BSpline
    t = [0.0, 0.0, 0.0, 1.0, 1.0, 1.0]
    w = np.array([1.0, np.sqrt(2.0) / 2.0, 1.0])
    cp = np.array([[1.0, 0.0], [1.0, 1.0], [0.0, 1.0]])
    num, den = BSpline(t, w[:, None] * cp, 2), BSpline(t, w, 2)
    r, R = O.ANNULUS
    for xi in np.linspace(0.0, 1.0, 11):
        for eta in (0.0, 0.3, 1.0):
            rho = r + (R - r) * eta
            got = O.annulus_point(xi, eta)
            assert np.allclose(got, rho * num(xi) / den(xi), rtol=0, atol=1e-15)
            assert abs(np.hypot(*got) - rho) < 1e-15


@pytest.mark.parametrize("q,m", [(2, 1), (2, 5), (3, 4), (5, 7), (8, 6)])
def test_annulus_weights_reproduce_the_denominator(q, m):
    """The weight net of the degree-q refinement (Section 2.2): the spline
    with the oracle's weights as coefficients equals the arc's quadratic
    denominator (1-xi)^2 + sqrt(2) xi (1-xi) + xi^2; one quadratic element
    gives back the defining weights."""
    from scipy.interpolate import BSpline
    w = O.annulus_weights(q, m)
    xs = np.linspace(0.0, 1.0, 37)
    ref = (1 - xs) ** 2 + np.sqrt(2.0) * xs * (1 - xs) + xs ** 2
    assert np.max(np.abs(BSpline(O.knots(q, m), w, q)(xs) - ref)) < 1e-13
    if (q, m) == (2, 1):
        assert np.allclose(w, [1.0, np.sqrt(2.0) / 2.0, 1.0], rtol=0, atol=1e-14)


@pytest.mark.parametrize("p", [2, 3])
def test_annulus_discrete_solution_converges(p):
    """Section 5.2: the NURBS Galerkin solution of the manufactured problem
    (exact solution sin(pi x) sin(pi y)(x^2+y^2-r^2)(x^2+y^2-R^2)) converges in
    L2 at order p+1 under refinement (pins the map and its Jacobian, the
    rational basis and its gradients, the quadrature and the load vector)."""
    errs = []
    for m in (4, 8, 16):
        P = O.Problem(2, p, m, plow=2, annulus=O.ANNULUS)
        u = P.direct_solve(O.load_annulus(p, m))
        errs.append(O.l2_error_annulus(p, m, u))
    rates = [np.log2(errs[i] / errs[i + 1]) for i in range(2)]
    assert min(rates) > p + 1 - 0.3, (errs, rates)


def test_annulus_mixed_form_with_equal_degrees_is_the_mass():
    """With p_low = p the mixed mass M_p^{p_low} of Section 3.1.2 is the mass
    matrix of the space, symmetric (entry (i, i+o) equals entry (i+o, i))."""
    p, m = 3, 6
    Mm = O.assemble_annulus(p, p, m, "mix")
    M = O.assemble_annulus(p, p, m, "mass")
    assert np.allclose(Mm, M, rtol=0, atol=1e-15 * np.abs(M).max())
    D = O.offsets_to_dense(M, 2, m + p - 2, p)
    assert np.allclose(D, D.T, rtol=0, atol=1e-15 * np.abs(D).max())
    assert np.linalg.eigvalsh(D).min() > 0


def test_table5_iteration_counts_in_paper_band():
    """Table 5 (quarter annulus, NURBS, p_low = 2, direct coarse solve, initial
    residual reduced by 1e-8; manufactured right-hand side, zero initial
    guess): iteration counts of the coloured two-level method on 32 x 32
    elements for p = 3..6 lie in the context band used for Table 4 (the
    paper's colouring and initial data are not stated exactly).  The colour
    period is b + p, so that blocks of one colour do not couple (Section
    3.1.1); with period b the method does not reach the tolerance on the
    annulus for p >= 6 (measured: no convergence in 60 cycles)."""
    table = {int(r[0]): r[1:] for r in _golden("table5_annulus_iterations.txt")}
    m = 32
    for k, p in enumerate((3, 4, 5, 6)):
        it_ds = table[m][2 * k]
        P = O.Problem(2, p, m, plow=2, annulus=O.ANNULUS)
        b = O.load_annulus(p, m)
        _, cyc, _ = P.solve(b, ordering=O.COLOUR, s=P.block_width + p, coarse=O.DIRECT, tol=1e-8, max_cycles=60)
        assert it_ds - 3 <= cyc <= 3 * it_ds, (p, cyc, it_ds)


def test_annulus_seven_by_seven_sweep_sensitivity():
    """The 7x7-block bar of the annulus (p = 8, m = 10, colour period b+p).
    The operator assembled as the library does it, tensor sums of weighted
    1-D forms (built here from the oracle's knots, B-splines, weights and
    Gauss rule), agrees with the oracle's 2-D quadrature to 2e-14 of its
    largest entry, the gap of two equally valid FP64 assemblies.  Block
    condition numbers reach ~1e5 on the annulus, and the same sweep computed
    on the two operators differs by ~6e-11 (more than 1e-11, less than
    2e-10): the GPU parity bar for 7x7 blocks on the annulus is 2e-10."""
    d, p, m = 2, 8, 10
    r, R = O.ANNULUS
    n1 = m + p - 2
    t, w = O.knots(p, m), O.annulus_weights(p, m)
    gx, gw = O.gauss_legendre(p + 3)

    def arc(x):
        a, r2 = 1 - x, np.sqrt(2.0)
        nx, ny = a * a + r2 * x * a, r2 * x * a + x * x
        W = nx + x * x
        dnx, dny = -2 * a + r2 * (1 - 2 * x), r2 * (1 - 2 * x) + 2 * x
        dW = dnx + 2 * x
        return W, dW, np.hypot((dnx * W - nx * dW) / W ** 2, (dny * W - ny * dW) / W ** 2)

    def forms(axis):
        K, M = np.zeros((n1, n1)), np.zeros((n1, n1))
        for e in range(m):
            for k in range(len(gx)):
                x, wq = (e + 0.5 * (gx[k] + 1)) / m, 0.5 * gw[k] / m
                v = np.array([O.bspline(t, p, e + a, x) for a in range(p + 1)])
                dv = np.array([O.bspline_deriv(t, p, e + a, x) for a in range(p + 1)])
                if axis == 0:   # angular: phi = w_i N_i / W, weights 1/speed and speed
                    W, dW, sp = arc(x)
                    om = w[e:e + p + 1]
                    dv, v = om * (dv * W - v * dW) / W ** 2, om * v / W
                    wk, wm = 1 / sp, sp
                else:           # radial: rho/(R-r) and (R-r)/rho
                    rho = r + (R - r) * x
                    wk, wm = rho / (R - r), (R - r) / rho
                for a in range(p + 1):
                    for c in range(p + 1):
                        i, j = e + a - 1, e + c - 1
                        if 0 <= i < n1 and 0 <= j < n1:
                            K[i, j] += wq * wk * dv[a] * dv[c]
                            M[i, j] += wq * wm * v[a] * v[c]
        return K, M

    Kx, Mx = forms(0)
    Ky, My = forms(1)
    Ak = np.kron(My, Kx) + np.kron(Ky, Mx)
    P = O.Problem(d, p, m, plow=2, annulus=O.ANNULUS)
    A = O.offsets_to_dense(P.A(), d, n1, p)
    assert np.max(np.abs(A - Ak)) <= 2e-14 * np.max(np.abs(A))
    bw, n = P.block_width, P.n
    s = bw + p
    members = [_block_members(d, n1, bw, j) for j in range(n)]
    u0 = synth.initial_guess(d, p, m, seed=1)
    b = synth.rhs_normal(d, p, m, seed=0)

    def sweep(Aop):
        u = u0.copy()
        for cy in range(s):
            for cx in range(s):
                res = b - Aop @ u
                du = np.zeros_like(u)
                for j in range(n):
                    if (j % n1) % s == cx and (j // n1) % s == cy:
                        idx = members[j]
                        du[idx] += np.linalg.solve(Aop[np.ix_(idx, idx)], res[idx])
                u = u + du
        return u

    ref = P.sweep(u0, b, ordering=O.COLOUR, s=s)
    on_A = sweep(A)
    assert np.linalg.norm(on_A - ref) <= 1e-12 * np.linalg.norm(ref)
    gap = np.linalg.norm(sweep(Ak) - on_A) / np.linalg.norm(on_A)
    assert 1e-11 < gap < 2e-10, gap
