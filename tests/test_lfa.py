"""Local Fourier analysis (Section 4) of the two-level method: the calculator
of paper_2009_01499_amd.lfa against the factors the paper prints (Tables 1-3),
against textbook special cases, and against rates measured with the oracle.

The LFA reproduces Table 1 (two-grid, exact coarse solve) to four digits
wherever the refined frequency search agrees with the paper's sampling
(16 of 21 entries tested here), and Tables 2-3 wherever the smoother
limits the rate.  Where the coarse level limits it (p = 2, and 25-point
blocks at p = 3 with aggressive coarsening) the paper's three-grid and
aggressive factors are 2-14 % above this calculator's, and the rates the
oracle measures follow the calculator (p = 2 aggressive on 256^2: measured
0.143, LFA 0.149, paper 0.172): the paper's h <-> 2h transfers cannot be
recovered exactly from its text; the test keeps those entries as a band.
"""
import numpy as np
import pytest

import oracle as O
import synth
from paper_2009_01499_amd import lfa


def _table():
    rows = []
    with open(__file__.replace("test_lfa.py", "golden/lfa_tables.txt")) as f:
        for line in f:
            if line.strip() and not line.startswith("#"):
                v = line.split()
                rows.append((int(v[0]), int(v[1]), float(v[2]), float(v[3]), float(v[4])))
    return rows


def test_cardinal_bspline_stencils():
    """Closed forms used by the analysis: p = 1 gives (h/6)[1,4,1] and
    (1/h)[-1,2,-1]; p = 2 mass (h/120)[1,26,66,26,1]; stiffness rows sum to 0,
    mass rows to 1 (h = 1)."""
    K1, M1 = lfa.stencils_1d(1)
    assert np.allclose(M1, [1 / 6, 4 / 6, 1 / 6]) and np.allclose(K1, [-1, 2, -1])
    K2, M2 = lfa.stencils_1d(2)
    assert np.allclose(M2, np.array([1, 26, 66, 26, 1]) / 120)
    assert np.allclose(K2, [-1 / 6, -1 / 3, 1, -1 / 3, -1 / 6])
    for p in range(1, 9):
        K, M = lfa.stencils_1d(p)
        assert abs(K.sum()) < 1e-13 and abs(M.sum() - 1) < 1e-13
        r = lfa.restriction_symbol_1d(p, np.array([0.0]))
        assert abs(r[0] - 1) < 1e-13                  # interior rows of D^{-1} M_p^1 sum to 1


def test_point_block_is_gauss_seidel_symbol():
    """b = 1: the lexicographic block sweep is point Gauss-Seidel, whose symbol
    is -U(theta) / (a_0 + L(theta)) (L: the stencil entries before the point in
    the lexicographic order, U: those after it)."""
    p = 3
    a = lfa.operator_stencil_2d(p)
    rng = np.random.default_rng(0)
    th = rng.uniform(-np.pi, np.pi, (50, 2))
    Lh = np.zeros(50, complex)
    Uh = np.zeros(50, complex)
    for oy in range(-p, p + 1):
        for ox in range(-p, p + 1):
            if oy == 0 and ox == 0:
                continue
            e = a[oy + p, ox + p] * np.exp(1j * (th[:, 0] * ox + th[:, 1] * oy))
            if oy < 0 or (oy == 0 and ox < 0):
                Lh += e
            else:
                Uh += e
    ref = -Uh / (a[p, p] + Lh)
    assert np.allclose(lfa.schwarz_lex_symbol(p, 1, th), ref, atol=1e-12)


def test_block_covering_everything_kills_error():
    """Blocks much wider than the operator make the Schwarz sweep nearly an exact
    solve for smooth errors, and any sweep leaves theta = pi (the highest
    frequency) strongly damped: |S| < 1 everywhere away from theta = 0."""
    th = lfa._grid(16, -np.pi, np.pi).reshape(-1, 2)
    for p, b in ((2, 3), (3, 5)):
        s = np.abs(lfa.schwarz_lex_symbol(p, b, th))
        assert np.all(s < 1.0)


@pytest.mark.slow
def test_table1_two_grid_factors():
    """Table 1 (rho_2g): within 0.3 % where the paper's sampling finds the same
    supremum (all 3x3 entries, 5x5 for p <= 5, 7x7 at p = 5), within 2.5 % at
    p = 6 with 5x5 blocks (the refined search finds 0.4575 against 0.4549; at
    p = 6 with 7x7 blocks, not tested for time, 0.1948 against 0.1909)."""
    for p, b, r2, _, _ in _table():
        if (b == 7 and p != 5) or (b == 5 and p > 6):
            continue
        v = lfa.rho_2g(p, b, n=48 if b == 3 else 32)
        tol = 0.025 if (p, b) == (6, 5) else 0.003
        assert abs(v / r2 - 1) < tol, (p, b, v, r2)


@pytest.mark.slow
def test_tables2_3_where_the_smoother_limits():
    """Tables 2 and 3 where the coarse level does not limit the rate (tested:
    3x3 blocks at p = 3, 4, 6, 8; 5x5 blocks at p >= 4 agree as well, not
    tested for time): the three-grid and aggressive factors equal the two-grid
    one, and the paper's values are within 0.6 % below (up to 3 % below for
    7x7 blocks)."""
    for p, b, r2, r3, ra in _table():
        if (p, b) not in ((3, 3), (4, 3), (6, 3), (8, 3)):
            continue
        v3, va = lfa.rho_3g(p, b), lfa.rho_2g_ag(p, b)
        assert 0.0 <= v3 / r3 - 1 < 0.006, (p, b, v3, r3)
        assert 0.0 <= va / ra - 1 < 0.006, (p, b, va, ra)


@pytest.mark.slow
def test_coarse_limited_entries_band_and_oracle():
    """Where the coarse level limits the rate (p = 2): the three-grid factor is
    within 3 % of Table 2 and the aggressive one 10-15 % below Table 3, and the
    oracle's measured rate of aggressive coarsening (lexicographic sweep,
    exact 2h solve, random initial guess, 256^2) is within 6 % of this
    calculator's factor."""
    rows = {(p, b): (r3, ra) for p, b, _, r3, ra in _table()}
    v3, va = lfa.rho_3g(2, 3), lfa.rho_2g_ag(2, 3)
    r3, ra = rows[(2, 3)]
    assert abs(v3 / r3 - 1) < 0.03
    assert 0.85 < va / ra < 0.9
    p, m, K = 2, 256, 30
    P = O.Problem(2, p, m, vcycle=True, coarse_direct=False)
    u0 = synth.initial_guess(2, p, m, seed=1)
    _, _, hist = P.solve(np.zeros(P.n), u0=u0, ordering=O.LEX, coarse=O.DIRECT, aggressive=True, tol=0.0,
                         max_cycles=K)
    measured = (hist[K] / hist[10]) ** (1.0 / (K - 10))
    assert abs(measured / va - 1) < 0.06, (measured, va)


def test_two_grid_factor_matches_oracle_rate():
    """The LFA two-grid factor against the oracle's measured rate of the same
    method (lexicographic sweep, exact degree-1 coarse solve, p = 3, 64^2,
    random initial guess): within 8 % (finite grid vs infinite grid)."""
    p, m, K = 3, 64, 30
    P = O.Problem(2, p, m)
    u0 = synth.initial_guess(2, p, m, seed=1)
    _, _, hist = P.solve(np.zeros(P.n), u0=u0, ordering=O.LEX, tol=0.0, max_cycles=K)
    measured = (hist[K] / hist[10]) ** (1.0 / (K - 10))
    v = lfa.rho_2g(p, 3)
    assert abs(measured / v - 1) < 0.08, (measured, v)
