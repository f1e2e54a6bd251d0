"""Measurements of the other configurations, printed by ``bench.py --suite``
as one JSON line each (the headline line of bench.py stays the first line).

  C1  2-D p=3, 32x32, lexicographic Schwarz, exact p=1 coarse solve, FP64
  C2  2-D 256x256, p = 2..5, coloured Schwarz, V(2,2) coarse, FP64 and mixed
  C3  3-D p=3, 64x64x64, coloured 3x3x3 Schwarz, V(2,2) coarse, FP64 and mixed
  C4  256 independent 2-D problems, m in 32..128, p in 2..4, kappa = exp(GRF)
  C5  2-D p=4 256x256 GRF kappa: forward mixed solve + adjoint gradient
  AGG 2-D 256x256, p = 2..5, the paper's timed configuration: aggressive
      coarsening (degree 1 on 2h) with one V(1,1) cycle there
  LARGE 2-D p=3 at 2048^2 and 4096^2 (4.2 M and 16.8 M DOFs), V(2,2) coarse, FP64
      and mixed: the bandwidth regime (streamed kernels) on the whole solve
  ANN quarter annulus (NURBS, Section 5.2), 32^2 .. 256^2, p = 3..8, degree-2
      coarse space solved exactly, coloured Schwarz with period b+2 (the
      shortest period that converges like non-interacting colours on the
      annulus), to a 1e-8 reduction (Table 5's stopping rule), FP64 and mixed
Each line states the error of the GPU solution against the oracle's (C3:
against sampled values of a stored oracle solution; C4: four sampled problems).
Every step is a complete solve to a 1e-10 residual reduction from u = 0 with
inputs resident on the GPU; times are host wall clock around synchronised
calls.
"""
from __future__ import annotations

import json
import os
import time

import numpy as np

import synth

GOLDEN_C3 = os.path.join(os.path.dirname(os.path.abspath(__file__)), "tests", "golden", "c3_solution_3d_p3_m64.json")


def _timed(torch, fn, steps):
    fn()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    out = None
    for _ in range(steps):
        out = fn()
    torch.cuda.synchronize()
    return (time.perf_counter() - t0) / steps, out


def _error_vs(u_ref, u):
    return float(np.linalg.norm(u - u_ref) / np.linalg.norm(u_ref))


def _solve_line(torch, G, name, d, p, m, opts_list, steps, kappa=None, block_width=0, oracle_ref=None):
    """oracle_ref(b_np, solutions) -> dict of errors against the oracle (or None)."""
    prob = G.Problem(d, p, m, kappa=kappa, device=0)
    t0 = time.perf_counter()
    for o in opts_list.values():
        prob.setup(block_width, o)
    torch.cuda.synchronize()
    t_setup = time.perf_counter() - t0
    b_np = synth.rhs_normal(d, p, m, seed=0)
    b = torch.tensor(b_np, device="cuda")
    u = torch.zeros_like(b)
    line = {"config": name, "dim": d, "p": p, "m": m, "n_fine": prob.n, "setup_s": t_setup}
    sols = {}
    for label, o in opts_list.items():
        def one():
            u.zero_()
            return prob.solve(b, u, o)[1]
        t, info = _timed(torch, one, steps)
        line[label] = {"time_to_tol_ms": 1e3 * t, "cycles": info.iters, "relres": info.relres,
                       "fine_dof_per_s_per_cycle": prob.n * info.iters / t}
        sols[label] = u.cpu().numpy().copy()
    prob.close()
    if oracle_ref is not None:
        line["error_vs_oracle"] = oracle_ref(b_np, sols)
    return line


def _oracle_c2(d, p, m, nu, aggressive=False):
    """Errors of every solution against the oracle's converged solution of the
    same FP64 solve (CPU-oracle leg)."""
    def ref(b_np, sols):
        from bench import oracle_solution
        u_orc, k = oracle_solution(d, p, m, b_np, nu=nu, aggressive=aggressive)
        out = {label: _error_vs(u_orc, v) for label, v in sols.items()}
        out["oracle_cycles"] = k
        return out
    return ref


def _oracle_c3(b_np, sols):
    """C3: the oracle's solution at 3000 sampled DOFs and its 2-norm, written by
    tests/golden/make_c3_solution.py (the oracle's set-up at 64^3 takes ~20 min)."""
    if not os.path.exists(GOLDEN_C3):
        return None
    ref = json.load(open(GOLDEN_C3))
    idx = np.array(ref["sample"]["index"], dtype=np.int64)
    want = np.array([float(v) for v in ref["sample"]["value"]])
    out = {"oracle_cycles": ref["cycles"], "sample": "3000 seeded DOFs + 2-norm of u"}
    for label, v in sols.items():
        out[label] = {"sampled_rel": _error_vs(want, v[idx]),
                      "norm_rel": abs(float(np.linalg.norm(v)) / float(ref["u_l2"]) - 1.0)}
    return out


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
                                 {"fp64": G.Opts(**v22), "mixed": G.Opts(precision=G.MIXED_FP32, **v22)}, steps,
                                 oracle_ref=_oracle_c2(2, p, 256, (2, 2))))
    # C3
    if want("C3"):
        lines.append(_solve_line(torch, G, "C3", 3, 3, 64,
                                 {"fp64": G.Opts(**v22), "mixed": G.Opts(precision=G.MIXED_FP32, **v22)},
                                 max(2, steps // 2), oracle_ref=_oracle_c3))
    # the paper's own configuration (Section 5.1): aggressive coarsening to degree 1
    # on 2h with one V(1,1) cycle there, coloured sweep
    if want("AGG"):
        v11a = dict(coarse=G.COARSE_VCYCLE, nu1=1, nu2=1, tol=1e-10, aggressive=1)
        for p in (2, 3, 4, 5):
            line = _solve_line(torch, G, "C2-aggressive", 2, p, 256,
                               {"fp64": G.Opts(**v11a), "mixed": G.Opts(precision=G.MIXED_FP32, **v11a)}, steps,
                               oracle_ref=_oracle_c2(2, p, 256, (1, 1), aggressive=True))
            line["paper_table4_iterations_1e-8_context"] = {2: 6, 3: 6, 4: 7, 5: 5}[p]
            lines.append(line)
    if want("LARGE"):
        for m in (2048, 4096):
            line = _solve_line(torch, G, "LARGE", 2, 3, m,
                               {"fp64": G.Opts(**v22), "mixed": G.Opts(precision=G.MIXED_FP32, **v22)},
                               max(2, steps // 4),
                               oracle_ref=lambda b_np, sols: {"mixed_vs_fp64": _error_vs(sols["fp64"], sols["mixed"])})
            # no oracle solution at this size (its set-up alone takes minutes): the
            # mixed solution against the FP64 one instead
            line["difference"] = line.pop("error_vs_oracle")
            lines.append(line)
    if want("ANN"):
        lines.extend(_annulus(torch, G, steps))
    if want("C4"):
        lines.append(_c4(torch, G, v22))
    if want("C5"):
        lines.append(_c5(torch, G))
    return lines


ANNULUS_RADII = (0.3, 0.5)
TABLE5_DS = {32: {3: 5, 4: 8, 5: 4, 6: 6, 7: 3, 8: 4}, 64: {3: 5, 4: 8, 5: 4, 6: 6, 7: 4, 8: 5},
             128: {3: 6, 4: 7, 5: 4, 6: 6, 7: 4, 8: 5}, 256: {3: 6, 4: 8, 5: 4, 6: 6, 7: 4, 8: 5}}


def _annulus(torch, G, steps):
    """Quarter annulus: one line per grid, every degree; the right-hand side is
    seeded N(0,1) (Table 5 uses a manufactured load: its counts are context).
    At 32^2 and p <= 5 the FP64 solution is compared with the oracle's."""
    out = []
    for m in (32, 64, 128, 256):
        line = {"config": "ANN", "grid": f"{m}x{m}", "radii": ANNULUS_RADII, "plow": 2, "coarse": "exact (FDM)",
                "colour_period": "b+2"}
        for p in (3, 4, 5, 6, 7, 8):
            bw = 3 if p <= 4 else (5 if p <= 6 else 7)
            o64 = G.Opts(coarse=G.COARSE_DIRECT, plow=2, colour_period=bw + 2, tol=1e-8, max_cycles=100)
            o32 = G.Opts(coarse=G.COARSE_DIRECT, plow=2, colour_period=bw + 2, tol=1e-8, max_cycles=100,
                         precision=G.MIXED_FP32)
            t0 = time.perf_counter()
            prob = G.Problem(2, p, m, annulus=ANNULUS_RADII, device=0)
            prob.setup(0, o64)
            prob.setup(0, o32)
            torch.cuda.synchronize()
            t_setup = time.perf_counter() - t0
            b_np = synth.rhs_normal(2, p, m, seed=0)
            b = torch.tensor(b_np, device="cuda")
            u = torch.zeros_like(b)
            rec = {"n_fine": prob.n, "setup_s": t_setup, "paper_table5_DS_iterations_context": TABLE5_DS[m][p]}
            for label, o in (("fp64", o64), ("mixed", o32)):
                def one():
                    u.zero_()
                    return prob.solve(b, u, o)[1]
                t, info = _timed(torch, one, steps)
                rec[label] = {"time_to_tol_ms": 1e3 * t, "cycles": info.iters, "relres": info.relres}
                if label == "fp64":
                    u64 = u.cpu().numpy().copy()
            if m == 32 and p <= 5:
                import oracle as O
                orc = O.Problem(2, p, m, plow=2, annulus=ANNULUS_RADII)
                uo, ko, _ = orc.solve(b_np, ordering=O.COLOUR, s=bw + 2, coarse=O.DIRECT, tol=1e-8, max_cycles=100)
                rec["error_vs_oracle_fp64"] = _error_vs(uo, u64)
                rec["oracle_cycles"] = ko
            line[f"p{p}"] = rec
            prob.close()
        out.append(line)
    return out


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
    # the same with the kernels of every cycle launched directly instead of the
    # captured graph being replayed (numerics identical)
    os.environ["IGA2L_BATCH_GRAPH"] = "0"
    t_mixed_eager, _ = _timed(torch, lambda: batch(mixed), 3)
    del os.environ["IGA2L_BATCH_GRAPH"]

    def one_by_one():
        for pr, b, u in zip(probs, bs, us):
            u.zero_()
            pr.solve(b, u, mixed)

    t_seq, _ = _timed(torch, one_by_one, 1)
    # error against the oracle on four sampled problems (mixed batch solution)
    batch(mixed)
    torch.cuda.synchronize()
    err = {}
    from bench import oracle_solution
    for k in (0, 85, 170, 255):
        sp = specs[k]
        kap = synth.kappa_grf(2, sp["m"], 1.0, 0.1, seed=sp["kappa_seed"])
        u_orc, _ = oracle_solution(2, sp["p"], sp["m"], synth.rhs_normal(2, sp["p"], sp["m"], seed=sp["rhs_seed"]),
                                   kappa=kap, nu=(2, 2))
        err[f"problem {k} (m={sp['m']}, p={sp['p']})"] = _error_vs(u_orc, us[k].cpu().numpy())
    ndof = sum(p.n for p in probs)
    cyc = sum(p.n * i.iters for p, i in zip(probs, infos))
    rec = {"config": "C4", "problems": len(probs), "total_fine_dofs": ndof, "setup_s": t_setup,
           "mixed": {"time_to_tol_ms": 1e3 * t_mixed, "max_cycles": max(i.iters for i in infos),
                     "worst_relres": max(i.relres for i in infos), "fine_dof_cycles_per_s": cyc / t_mixed},
           "fp64": {"time_to_tol_ms": 1e3 * t_fp64, "max_cycles": max(i.iters for i in infos64),
                    "worst_relres": max(i.relres for i in infos64)},
           "mixed_without_graph_ms": 1e3 * t_mixed_eager,
           "mixed_one_problem_at_a_time_ms": 1e3 * t_seq, "error_vs_oracle_mixed_sampled": err}
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
    # forward solution against the oracle's converged solution (CPU-oracle leg)
    from bench import oracle_solution
    u_fwd = G.iga_solve(kt.detach(), b, d, p, m, fwd, tight).cpu().numpy()
    u_orc, _ = oracle_solution(d, p, m, b.cpu().numpy(), kappa=kap, nu=(2, 2))
    err_fwd = _error_vs(u_orc, u_fwd)
    rec = {"config": "C5", "dim": d, "p": p, "m": m, "forward_backward_ms_incl_assembly": 1e3 * t,
           "error_vs_oracle_forward_mixed": err_fwd,
           "note": "assembly + set-up of A(kappa), mixed forward solve, FP64 adjoint solve to 1e-12, "
                   "dL/dkappa kernel"}
    obs.close()
    return rec
