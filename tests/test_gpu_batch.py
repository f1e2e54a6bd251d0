"""Batched solve of independent problems of uneven size, degree and
coefficient field (configuration 4 recipe, fewer problems): every batched
result equals the single-problem solve bitwise, reaches the tolerance, and
matches the oracle's direct solution within the bound the tolerance allows."""
import numpy as np
import pytest

import oracle as O
import synth

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")


def _G():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_2009_01499_amd as G
    return G


def _problems(G, specs, opts):
    probs, bs = [], []
    for sp in specs:
        kap = synth.kappa_grf(2, sp["m"], 1.0, 0.1, seed=sp["kappa_seed"])
        pr = G.Problem(2, sp["p"], sp["m"], kappa=kap).setup(3, opts)
        probs.append(pr)
        bs.append(torch.tensor(synth.rhs_normal(2, sp["p"], sp["m"], seed=sp["rhs_seed"]), device="cuda"))
    return probs, bs


@pytest.mark.parametrize("precision", ["fp64", "mixed"])
def test_batch_equals_single_solves(precision):
    G = _G()
    specs = synth.batch_specs(12, seed=4)
    print("\n[case] batch of", [(s["m"], s["p"]) for s in specs], precision, flush=True)
    opts = G.Opts(coarse=G.COARSE_VCYCLE, nu1=2, nu2=2, tol=1e-10,
                  precision=G.FP64 if precision == "fp64" else G.MIXED_FP32)
    probs, bs = _problems(G, specs, opts)
    us = [torch.zeros_like(b) for b in bs]
    infos = G.solve_batch(probs, bs, us, opts)
    for k, (pr, b) in enumerate(zip(probs, bs)):
        assert infos[k].relres <= 1e-10, (k, infos[k])
        u1, i1 = pr.solve(b, None, opts)
        assert i1.iters == infos[k].iters
        assert torch.equal(u1, us[k]), k
    for k in (0, 5):
        sp = specs[k]
        kap = synth.kappa_grf(2, sp["m"], 1.0, 0.1, seed=sp["kappa_seed"])
        ref = O.Problem(2, sp["p"], sp["m"], kappa=kap).direct_solve(bs[k].cpu().numpy())
        err = np.linalg.norm(us[k].cpu().numpy() - ref) / np.linalg.norm(ref)
        print(f"[batch] problem {k} (m={sp['m']}, p={sp['p']}): error vs oracle direct solve {err:.2e}")
        assert err < 1e-7
