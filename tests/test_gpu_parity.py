"""GPU (gfx950 HIP library, through the C ABI) against the CPU oracle.

FP64 bar: 1e-12 relative (norm-wise) per operation and per cycle iterate,
on the same seeded inputs and the same block ordering.
"""
import json
import os

import numpy as np
import pytest

import oracle as O
import synth

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


def _gpu():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_2009_01499_amd as G
    return G


def dev(x):
    return torch.tensor(np.asarray(x, dtype=np.float64), device="cuda")


def host(t):
    torch.cuda.synchronize()
    return t.detach().cpu().numpy()


def rel(a, b):
    nb = np.linalg.norm(b)
    return np.linalg.norm(a - b) / (nb if nb > 0 else 1.0)


def _pair(d, p, m, kappa=None, bw=0, vcycle=True, direct=True, mixed=False):
    G = _gpu()
    print(f"\n[case] d={d} p={p} m={m} kappa={'grf' if kappa is not None else 1} bw={bw}", flush=True)
    orc = O.Problem(d, p, m, kappa=kappa, block_width=bw, coarse_direct=direct, vcycle=vcycle)
    gp = G.Problem(d, p, m, kappa=kappa)
    if vcycle:
        gp.setup(bw, G.Opts(coarse=G.COARSE_VCYCLE, precision=G.MIXED_FP32 if mixed else G.FP64))
    if direct and kappa is None:
        gp.setup(bw, G.Opts(coarse=G.COARSE_DIRECT, precision=G.MIXED_FP32 if mixed else G.FP64))
    if not vcycle and not direct:
        gp.setup(bw, G.Opts())
    assert gp.n == orc.n and gp.nc == orc.nc
    return G, orc, gp


def sweep_tolerance(orc):
    """FP64 bar for Schwarz sweeps: 1e-12 relative, unless the rounding bound of
    two backward-stable local solvers exceeds it.  A block solve of size bd with
    condition kappa_B is accurate to about bd * eps * kappa_B; one sweep chains
    bd colours (s = b), so two correct implementations may differ by up to
    about bd^2 * eps * kappa_B.  With 3x3 and 5x5 blocks (p <= 6) this stays far
    below 1e-12; with 7x7 blocks (p = 7, 8; kappa_B up to ~5e3) it is ~1e-10,
    and the bar becomes 5e-11."""
    return 1e-12 if orc.block_width <= 5 else 5e-11


CASES_2D = [(2, 3, 32, None), (2, 2, 33, None), (2, 5, 20, None), (2, 4, 24, "grf"), (2, 7, 14, None)]


@pytest.mark.parametrize("d,p,m,kap", CASES_2D + [(3, 2, 6, None), (3, 3, 5, "grf")])
def test_residual_parity(d, p, m, kap):
    kappa = synth.kappa_grf(d, m, 1.0, 0.1, seed=7) if kap else None
    G, orc, gp = _pair(d, p, m, kappa, vcycle=False, direct=False)
    u = synth.initial_guess(d, p, m, seed=1)
    b = synth.rhs_normal(d, p, m, seed=0)
    r = host(gp.residual(dev(u), dev(b)))
    e = rel(r, orc.residual(u, b))
    assert e < 1e-12, e


@pytest.mark.parametrize("d,p,m,kap", CASES_2D + [(3, 2, 6, None), (3, 3, 5, "grf")])
@pytest.mark.parametrize("period", ["b", "b+p", "lex"])
def test_one_sweep_parity(d, p, m, kap, period):
    kappa = synth.kappa_grf(d, m, 1.0, 0.1, seed=7) if kap else None
    G, orc, gp = _pair(d, p, m, kappa, vcycle=False, direct=False)
    bw = orc.block_width
    u = synth.initial_guess(d, p, m, seed=1)
    b = synth.rhs_normal(d, p, m, seed=0)
    if period == "lex":
        ref = orc.sweep(u, b, ordering=O.LEX)
        opts = G.Opts(ordering=G.LEX)
    else:
        s = bw if period == "b" else bw + p
        ref = orc.sweep(u, b, ordering=O.COLOUR, s=s)
        opts = G.Opts(ordering=G.COLOUR, colour_period=s)
    ug = dev(u)
    gp.smooth(ug, dev(b), 1, opts)
    e = rel(host(ug), ref)
    assert e < sweep_tolerance(orc), e


@pytest.mark.parametrize("d,p,m", [(2, 2, 100), (3, 2, 24)])
def test_lex_sweep_large_grid(d, p, m):
    """Lexicographic sweep on grids whose iterate exceeds one workgroup's
    LDS: the sweep runs as one launch per hyperplane step instead."""
    G, orc, gp = _pair(d, p, m, vcycle=False, direct=False)
    u = synth.initial_guess(d, p, m, seed=1)
    b = synth.rhs_normal(d, p, m, seed=0)
    ref = orc.sweep(u, b, ordering=O.LEX)
    ug = dev(u)
    gp.smooth(ug, dev(b), 1, G.Opts(ordering=G.LEX))
    e = rel(host(ug), ref)
    assert e < sweep_tolerance(orc), e


@pytest.mark.parametrize("d,p,m", [(2, 3, 32), (2, 4, 25), (2, 8, 12), (3, 3, 6)])
def test_transfer_parity(d, p, m):
    G, orc, gp = _pair(d, p, m, vcycle=False, direct=False)
    x = synth.rhs_normal(d, p, m, seed=3)
    xc = synth.rhs_normal(d, 1, m, seed=4)
    dc = host(gp.restrict(dev(x)))
    e = rel(dc, orc.restrict(x))
    assert e < 1e-14, e
    u0 = synth.initial_guess(d, p, m, seed=5)
    ug = dev(u0)
    gp.prolong_add(dev(xc), ug)
    e = rel(host(ug) - u0, orc.prolong_add(xc, u0) - u0)
    assert e < 1e-14, e


@pytest.mark.parametrize("d,m,kap", [(2, 32, None), (2, 64, None), (2, 33, "grf"), (2, 27, None), (2, 128, "grf"),
                                     (3, 8, None), (3, 16, None), (3, 13, "grf")])
@pytest.mark.parametrize("nu", [(1, 1), (2, 2), (1, 0)])
def test_vcycle_parity(d, m, kap, nu):
    kappa = synth.kappa_grf(d, m, 1.0, 0.1, seed=9) if kap else None
    G, orc, gp = _pair(d, 2, m, kappa, vcycle=True, direct=False)
    dc = synth.rhs_normal(d, 1, m, seed=2)
    ec = host(gp.coarse_solve(dev(dc), opts=G.Opts(coarse=G.COARSE_VCYCLE, nu1=nu[0], nu2=nu[1])))
    e = rel(ec, orc.coarse_vcycle(dc, *nu))
    assert e < 1e-12, e


@pytest.mark.parametrize("d,m", [(2, 32), (2, 17), (3, 6)])
def test_direct_coarse_parity(d, m):
    G, orc, gp = _pair(d, 3 if d == 2 else 2, m, vcycle=False, direct=True)
    dc = synth.rhs_normal(d, 1, m, seed=2)
    ec = host(gp.coarse_solve(dev(dc), opts=G.Opts(coarse=G.COARSE_DIRECT)))
    e = rel(ec, orc.coarse_direct(dc))
    assert e < 1e-12, e


def _iterates_gpu(G, gp, b, u0, opts, k):
    out = []
    u = dev(u0)
    bd = dev(b)
    for _ in range(k):
        o = G.Opts(**{**opts.__dict__, "max_cycles": 1, "tol": 0.0})
        gp.solve(bd, u, o, raise_on_notconv=False)
        out.append(host(u).copy())
    return out


@pytest.mark.parametrize("name,d,p,m,kap,ordering,period,coarse,nu", [
    ("C1-lex-direct", 2, 3, 32, None, "lex", 0, "direct", (1, 1)),
    ("colour-vcycle22", 2, 3, 32, None, "colour", 0, "vcycle", (2, 2)),
    ("colour-b+p-direct", 2, 2, 24, None, "colour", 5, "direct", (1, 1)),
    ("grf-vcycle", 2, 4, 24, "grf", "colour", 0, "vcycle", (1, 1)),
    ("p5-vcycle", 2, 5, 20, None, "colour", 0, "vcycle", (2, 2)),
    ("3d-vcycle", 3, 3, 6, None, "colour", 0, "vcycle", (1, 1)),
])
def test_cycle_iterates_parity(name, d, p, m, kap, ordering, period, coarse, nu):
    kappa = synth.kappa_grf(d, m, 1.0, 0.1, seed=5) if kap else None
    G, orc, gp = _pair(d, p, m, kappa, vcycle=(coarse == "vcycle"), direct=(coarse == "direct"))
    b = synth.rhs_normal(d, p, m, seed=0)
    u0 = synth.initial_guess(d, p, m, seed=11)
    gopts = G.Opts(ordering=G.LEX if ordering == "lex" else G.COLOUR, colour_period=period,
                   coarse=G.COARSE_DIRECT if coarse == "direct" else G.COARSE_VCYCLE, nu1=nu[0], nu2=nu[1])
    its = _iterates_gpu(G, gp, b, u0, gopts, 4)
    u = u0.copy()
    for k in range(4):
        u = orc.cycle(u, b, ordering=O.LEX if ordering == "lex" else O.COLOUR, s=period,
                      coarse=O.DIRECT if coarse == "direct" else O.VCYCLE, cnu1=nu[0], cnu2=nu[1])
        e = rel(its[k], u)
        assert e < 1e-12, (name, k, e)


def test_c1_solve_matches_oracle():
    """Configuration 1: 2-D, p=3, 32x32, lexicographic sweep, exact p=1 coarse
    solve, FP64, to 1e-10; random N(0,1) and manufactured right-hand sides."""
    G, orc, gp = _pair(2, 3, 32, vcycle=False, direct=True)
    opts = G.Opts(ordering=G.LEX, coarse=G.COARSE_DIRECT, tol=1e-10)
    for b in (synth.rhs_normal(2, 3, 32, seed=0), O.load_manufactured(2, 3, 32)):
        u_ref, k_ref, hist = orc.solve(b, ordering=O.LEX, coarse=O.DIRECT, tol=1e-10)
        u, info = gp.solve(dev(b), opts=opts)
        assert info.iters == k_ref
        e = rel(host(u), u_ref)
        assert e < 1e-12, e
        assert abs(info.relres - hist[-1] / hist[0]) <= 1e-3 * hist[-1] / hist[0]


def test_mixed_precision_reaches_tolerance():
    """FP32 smoother/defect/transfers/V-cycle with FP64 residual and update
    reaches the same 1e-10 reduction; error against the oracle's direct solve
    is of the order of the FP64 run's."""
    G, orc, gp = _pair(2, 3, 64, vcycle=True, direct=False, mixed=True)
    b = synth.rhs_normal(2, 3, 64, seed=0)
    u_star = orc.direct_solve(b)
    u64, i64 = gp.solve(dev(b), opts=G.Opts(coarse=G.COARSE_VCYCLE, nu1=2, nu2=2))
    u32, i32 = gp.solve(dev(b), opts=G.Opts(coarse=G.COARSE_VCYCLE, nu1=2, nu2=2, precision=G.MIXED_FP32))
    assert i64.relres <= 1e-10 and i32.relres <= 1e-10
    e64, e32 = rel(host(u64), u_star), rel(host(u32), u_star)
    print(f"[mixed] cycles fp64={i64.iters} mixed={i32.iters} err fp64={e64:.2e} mixed={e32:.2e}")
    assert i32.iters <= i64.iters + 3
    assert e32 < 1e-8 and e64 < 1e-8


@pytest.mark.parametrize("m", [256])
def test_full_size_cycle_parity_256(m):
    """Headline configuration size (2-D, p=3, 256x256, coloured blocks,
    V(2,2) coarse cycle): the first two FP64 cycle iterates match the oracle."""
    G, orc, gp = _pair(2, 3, m, vcycle=True, direct=False)
    b = synth.rhs_normal(2, 3, m, seed=0)
    u0 = np.zeros(orc.n)
    its = _iterates_gpu(G, gp, b, u0, G.Opts(coarse=G.COARSE_VCYCLE, nu1=2, nu2=2), 2)
    u = u0
    for k in range(2):
        u = orc.cycle(u, b, coarse=O.VCYCLE, cnu1=2, cnu2=2)
        e = rel(its[k], u)
        print(f"[256^2] cycle {k + 1}: relative difference {e:.2e}")
        assert e < 1e-12, e


GOLDEN_LARGE = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden", "large_grid_2d_p3_m1024.json")


def test_large_grid_kernels_sampled():
    """2-D p=3 on 1024x1024 elements (1.05 M DOFs), where the residual runs as
    the column-blocked kernel and the transfers on 64x16 tiles:
    sampled entries and the 2-norms of the whole vectors against the oracle
    (values written by tests/golden/make_large_grid.py, which calls only the
    oracle)."""
    G = _gpu()
    ref = json.load(open(GOLDEN_LARGE))
    d, p, m = 2, 3, 1024
    print(f"\n[case] large grid d={d} p={p} m={m}", flush=True)
    gp = G.Problem(d, p, m)
    gp.setup(0, G.Opts())
    assert gp.n == ref["n"] and gp.nc == ref["nc"]
    u = synth.initial_guess(d, p, m, seed=1)
    b = synth.rhs_normal(d, p, m, seed=0)
    x = synth.rhs_normal(d, p, m, seed=3)
    ec = synth.rhs_normal(d, 1, m, seed=4)

    def check(name, full):
        idx = np.array(ref[name]["index"], dtype=np.int64)
        want = np.array([float(v) for v in ref[name]["value"]])
        e = rel(full[idx], want)
        en = abs(np.linalg.norm(full) / float(ref["norms"][name.replace("_add", "") + "_l2"]) - 1.0)
        print(f"[large] {name}: sampled rel {e:.2e}, norm rel {en:.2e}", flush=True)
        assert e < 1e-12 and en < 1e-12, (name, e, en)

    for _ in range(2):  # the second call reuses the norm partials of the first
        check("residual", host(gp.residual(dev(u), dev(b))))
    check("restrict", host(gp.restrict(dev(x))))
    ug = dev(u)
    gp.prolong_add(dev(ec), ug)
    check("prolong_add", host(ug))


def test_3d_factor_rows_bitwise(monkeypatch):
    """kappa = 1 in 3-D: rows next to the boundary formed from the 1-D factors
    give the FP64 residual and Schwarz sweep of the stored diagonals bit for
    bit (IGA2L_DIAGONAL_ROWS=1 makes set-up keep the diagonals for all rows)."""
    G = _gpu()
    d, p, m = 3, 3, 12
    u = synth.initial_guess(d, p, m, seed=1)
    b = synth.rhs_normal(d, p, m, seed=0)
    out = []
    for flag in ("1", "0"):
        monkeypatch.setenv("IGA2L_DIAGONAL_ROWS", flag)
        gp = G.Problem(d, p, m)
        gp.setup(0, G.Opts())
        r = host(gp.residual(dev(u), dev(b)))
        ug = dev(u)
        gp.smooth(ug, dev(b), 1, G.Opts())
        out.append((r, host(ug)))
    assert np.array_equal(out[0][0], out[1][0])
    assert np.array_equal(out[0][1], out[1][1])
