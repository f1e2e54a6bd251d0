"""Measurements of the other configurations, printed by ``bench.py --suite``
as one JSON line each (the headline line of bench.py stays the first line).

  C1  2-D p=3, 32x32, lexicographic Schwarz, exact p=1 coarse solve, FP64
  C2  2-D 256x256, p = 2..5, coloured Schwarz, V(2,2) coarse, FP64 and mixed
  C3  3-D p=3, 64x64x64, coloured 3x3x3 Schwarz, V(2,2) coarse, FP64 and mixed
  C4  256 independent 2-D problems, m in 32..128, p in 2..4, kappa = exp(GRF)
  C5  2-D p=4 256x256 GRF kappa: forward mixed solve + adjoint gradient
Every step is a complete solve to a 1e-10 residual reduction from u = 0 with
inputs resident on the GPU; times are host wall clock around synchronised
calls.
"""
from __future__ import annotations

import time

import synth


def _timed(torch, fn, steps):
    fn()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    out = None
    for _ in range(steps):
        out = fn()
    torch.cuda.synchronize()
    return (time.perf_counter() - t0) / steps, out


def _solve_line(torch, G, name, d, p, m, opts_list, steps, kappa=None, block_width=0):
    prob = G.Problem(d, p, m, kappa=kappa, device=0)
    t0 = time.perf_counter()
    for o in opts_list.values():
        prob.setup(block_width, o)
    torch.cuda.synchronize()
    t_setup = time.perf_counter() - t0
    b = torch.tensor(synth.rhs_normal(d, p, m, seed=0), device="cuda")
    u = torch.zeros_like(b)
    line = {"config": name, "dim": d, "p": p, "m": m, "n_fine": prob.n, "setup_s": t_setup}

    for label, o in opts_list.items():
        def one():
            u.zero_()
            return prob.solve(b, u, o)[1]
        t, info = _timed(torch, one, steps)
        line[label] = {"time_to_tol_ms": 1e3 * t, "cycles": info.iters, "relres": info.relres,
                       "fine_dof_per_s_per_cycle": prob.n * info.iters / t}
    prob.close()
    return line


def run(torch, G, steps=5, only=None):
    """One record per configuration; only: names of the configurations to run (all if None)."""
    lines = []
    v22 = dict(coarse=G.COARSE_VCYCLE, nu1=2, nu2=2, tol=1e-10)

    def want(name):
        return only is None or name in only

    # C1
    if want("C1"):
        lines.append(_solve_line(torch, G, "C1", 2, 3, 32,
                                 {"fp64_lex_direct": G.Opts(ordering=G.LEX, coarse=G.COARSE_DIRECT, tol=1e-10)},
                                 steps))
    # C2 sweep over p
    for p in ((2, 3, 4, 5) if want("C2") else ()):
        lines.append(_solve_line(torch, G, "C2", 2, p, 256,
                                 {"fp64": G.Opts(**v22), "mixed": G.Opts(precision=G.MIXED_FP32, **v22)}, steps))
    # C3
    if want("C3"):
        lines.append(_solve_line(torch, G, "C3", 3, 3, 64,
                                 {"fp64": G.Opts(**v22), "mixed": G.Opts(precision=G.MIXED_FP32, **v22)},
                                 max(2, steps // 2)))
    if want("C4"):
        lines.append(_c4(torch, G, v22))
    if want("C5"):
        lines.append(_c5(torch, G))
    return lines


def _c4(torch, G, v22):
    specs = synth.batch_specs(256, seed=4)
    t0 = time.perf_counter()
    probs, bs = [], []
    mixed = G.Opts(precision=G.MIXED_FP32, **v22)
    fp64 = G.Opts(**v22)
    for sp in specs:
        kap = synth.kappa_grf(2, sp["m"], 1.0, 0.1, seed=sp["kappa_seed"])
        pr = G.Problem(2, sp["p"], sp["m"], kappa=kap, device=0)
        pr.setup(3, mixed)
        probs.append(pr)
        bs.append(torch.tensor(synth.rhs_normal(2, sp["p"], sp["m"], seed=sp["rhs_seed"]), device="cuda"))
    torch.cuda.synchronize()
    t_setup = time.perf_counter() - t0
    us = [torch.zeros_like(b) for b in bs]

    def batch(o):
        for u in us:
            u.zero_()
        return G.solve_batch(probs, bs, us, o)

    t_mixed, infos = _timed(torch, lambda: batch(mixed), 3)
    t_fp64, infos64 = _timed(torch, lambda: batch(fp64), 3)

    def one_by_one():
        for pr, b, u in zip(probs, bs, us):
            u.zero_()
            pr.solve(b, u, mixed)

    t_seq, _ = _timed(torch, one_by_one, 1)
    ndof = sum(p.n for p in probs)
    cyc = sum(p.n * i.iters for p, i in zip(probs, infos))
    rec = {"config": "C4", "problems": len(probs), "total_fine_dofs": ndof, "setup_s": t_setup,
           "mixed": {"time_to_tol_ms": 1e3 * t_mixed, "max_cycles": max(i.iters for i in infos),
                     "worst_relres": max(i.relres for i in infos), "fine_dof_cycles_per_s": cyc / t_mixed},
           "fp64": {"time_to_tol_ms": 1e3 * t_fp64, "max_cycles": max(i.iters for i in infos64),
                    "worst_relres": max(i.relres for i in infos64)},
           "mixed_one_problem_at_a_time_ms": 1e3 * t_seq}
    for pr in probs:
        pr.close()
    return rec


def _c5(torch, G):
    d, p, m = 2, 4, 256
    kap = synth.kappa_grf(d, m, 0.5, 0.05, seed=1)
    kap_obs = synth.kappa_grf(d, m, 0.5, 0.05, seed=2)
    b = torch.tensor(synth.rhs_normal(d, p, m, seed=0), device="cuda")
    tight = G.Opts(tol=1e-12, max_cycles=300)
    fwd = G.Opts(precision=G.MIXED_FP32, tol=1e-10, coarse=G.COARSE_VCYCLE, nu1=2, nu2=2)
    obs = G.Problem(d, p, m, kappa=kap_obs, device=0).setup(0, tight)
    u_obs, _ = obs.solve(b, None, tight)
    kt = torch.tensor(kap, dtype=torch.float64, requires_grad=True)

    def fb():
        kt.grad = None
        u = G.iga_solve(kt, b, d, p, m, fwd, tight)
        loss = 0.5 * torch.sum((u - u_obs) ** 2)
        loss.backward()
        return loss

    t, _ = _timed(torch, fb, 2)
    rec = {"config": "C5", "dim": d, "p": p, "m": m, "forward_backward_ms_incl_assembly": 1e3 * t,
           "note": "assembly + set-up of A(kappa), mixed forward solve, FP64 adjoint solve to 1e-12, "
                   "dL/dkappa kernel"}
    obs.close()
    return rec
