"""Differentiable solve on the GPU: adjoint gradients against the oracle's
adjoint gradient and against central finite differences (configuration 5:
2-D, p=4, 256x256 elements, kappa = exp(GRF sigma=0.5, l=0.05), loss
L = 0.5 ||u - u_obs||^2, forward in mixed precision)."""
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


def test_adjoint_gradient_matches_oracle_small():
    G = _G()
    d, p, m = 2, 3, 12
    print(f"\n[case] adjoint small d={d} p={p} m={m}", flush=True)
    kap = synth.kappa_grf(d, m, 0.5, 0.2, seed=1)
    kap_obs = synth.kappa_grf(d, m, 0.5, 0.2, seed=2)
    b = synth.rhs_normal(d, p, m, seed=0)
    orc = O.Problem(d, p, m, kappa=kap)
    u_ref = orc.direct_solve(b)
    u_obs = O.Problem(d, p, m, kappa=kap_obs).direct_solve(b)
    lam_ref = orc.direct_solve(u_ref - u_obs)
    g_ref = orc.grad_kappa(u_ref, lam_ref)

    kt = torch.tensor(kap, dtype=torch.float64, requires_grad=True)
    bt = torch.tensor(b, device="cuda")
    fwd = G.Opts(tol=1e-13, max_cycles=200)
    adj = G.Opts(tol=1e-13, max_cycles=200)
    u = G.iga_solve(kt, bt, d, p, m, fwd, adj)
    loss = 0.5 * torch.sum((u - torch.tensor(u_obs, device="cuda")) ** 2)
    loss.backward()
    g = kt.grad.numpy()
    e = np.linalg.norm(g - g_ref) / np.linalg.norm(g_ref)
    print(f"[adjoint] |g - g_oracle| / |g_oracle| = {e:.2e}")
    assert e < 1e-9, e
    assert abs(np.dot(kap, g) + (u_ref - u_obs) @ u_ref) < 1e-8 * abs((u_ref - u_obs) @ u_ref)


@pytest.mark.timeout(600)
def test_c5_gradient_vs_central_differences():
    """Configuration 5.  Central differences in the cancellation-free form: with
    eps = eta * kappa_e, (A +- eps A_e) delta_pm = -+ eps A_e u gives
    L_pm - L = delta_pm . (u - u_obs) + 0.5 ||delta_pm||^2; Richardson
    extrapolation over eta = 1e-3 and 5e-4 removes the O(eta^2) term.  50
    elements drawn from seed 3; agreement to 1e-6 relative."""
    G = _G()
    d, p, m = 2, 4, 256
    kap = synth.kappa_grf(d, m, 0.5, 0.05, seed=1)
    kap_obs = synth.kappa_grf(d, m, 0.5, 0.05, seed=2)
    b = synth.rhs_normal(d, p, m, seed=0)
    bt = torch.tensor(b, device="cuda")
    mixed = G.Opts(precision=G.MIXED_FP32, tol=1e-12, max_cycles=300)
    tight = G.Opts(precision=G.FP64, tol=1e-13, max_cycles=300)
    print("\n[case] C5 d=2 p=4 m=256 GRF(0.5, 0.05)", flush=True)
    obs = G.Problem(d, p, m, kappa=kap_obs).setup(0, tight)
    u_obs, _ = obs.solve(bt, None, tight)
    kt = torch.tensor(kap, dtype=torch.float64, requires_grad=True)
    u = G.iga_solve(kt, bt, d, p, m, mixed, tight)
    loss = 0.5 * torch.sum((u - u_obs) ** 2)
    loss.backward()
    g = kt.grad.numpy()
    un = u.detach().cpu().numpy()
    res = un - u_obs.cpu().numpy()
    orc = O.Problem(d, p, m, kappa=kap, coarse_direct=False)   # for A_e u only
    elems = np.random.default_rng(3).choice(m * m, size=50, replace=False)
    worst = 0.0
    for idx, e in enumerate(elems):
        Aeu = orc.element_apply(int(e), un)
        est = []
        for eta in (1e-3, 5e-4):
            eps = eta * kap[e]
            dl = []
            for sgn in (+1, -1):
                kk = kap.copy()
                kk[e] += sgn * eps
                pr = G.Problem(d, p, m, kappa=kk).setup(0, tight)
                delta, _ = pr.solve(torch.tensor(-sgn * eps * Aeu, device="cuda"), None, tight)
                dn = delta.cpu().numpy()
                dl.append(dn @ res + 0.5 * dn @ dn)
                pr.close()
            est.append((dl[0] - dl[1]) / (2 * eps))
        fd = (4 * est[1] - est[0]) / 3
        rel = abs(fd - g[e]) / max(abs(g[e]), 1e-300)
        worst = max(worst, rel)
        if idx % 10 == 0:
            print(f"[fd] element {e}: adjoint {g[e]:.12e} fd {fd:.12e} rel {rel:.2e}", flush=True)
    print(f"[fd] worst relative difference over 50 elements: {worst:.2e}")
    assert worst < 1e-6
