"""iga2l_smooth_noalloc (the allocation-free coloured sweep) against
iga2l_smooth through the C ABI: two calls in a row, the second on a smaller
problem, each bit for bit equal to the allocating entry point; sizes beyond
the fixed array and the lexicographic ordering are rejected."""
import numpy as np
import pytest

import synth

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


def _gpu():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_2009_01499_amd as G
    return G


def _dev(x):
    return torch.tensor(np.asarray(x, dtype=np.float64), device="cuda")


def test_noalloc_smooth_matches_smooth():
    G = _gpu()
    cases = [(2, 3, 48, 0, 2), (2, 3, 20, 5, 1), (3, 3, 12, 0, 1)]   # second call smaller than the first
    for d, p, m, extra, nsweeps in cases:
        print(f"\n[case] noalloc d={d} p={p} m={m} s=b+{extra} sweeps={nsweeps}", flush=True)
        gp = G.Problem(d, p, m)
        gp.setup(0, G.Opts())
        bw = 3
        opts = G.Opts(ordering=G.COLOUR, colour_period=bw + extra if extra else 0)
        u0 = synth.initial_guess(d, p, m, seed=21)
        b = _dev(synth.rhs_normal(d, p, m, seed=22))
        ref = _dev(u0)
        gp.smooth(ref, b, nsweeps, opts)
        got = _dev(u0)
        gp.smooth_noalloc(got, b, nsweeps, opts)
        torch.cuda.synchronize()
        assert torch.equal(got, ref), (d, p, m, float((got - ref).abs().max()))
        gp.close()


def test_noalloc_smooth_rejects():
    G = _gpu()
    gp = G.Problem(2, 3, 8)
    gp.setup(0, G.Opts())
    u = _dev(np.zeros(gp.n))
    b = _dev(np.ones(gp.n))
    with pytest.raises(G.IGA2LError) as ei:
        gp.smooth_noalloc(u, b, 1, G.Opts(ordering=G.LEX))
    assert ei.value.code == G.EUNSUPPORTED
    gp.close()
    big = G.Problem(2, 3, 1448)          # 1449^2 = 2 099 601 > IGA2L_NOALLOC_MAX_FINE fine DOFs
    u = torch.zeros(big.n, dtype=torch.float64, device="cuda")
    with pytest.raises(G.IGA2LError) as ei:
        big.smooth_noalloc(u, u.clone(), 1, G.Opts())
    assert ei.value.code == G.EINVAL and "IGA2L_NOALLOC_MAX_FINE" in str(ei.value)
    big.close()
