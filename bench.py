"""Benchmark of the two-level isogeometric solver on one MI355X.

Workload (headline): 2-D Poisson on the unit square, tensor B-splines of
degree p=3 with maximal smoothness on 256x256 elements (66049 fine DOFs),
homogeneous Dirichlet, load vector b ~ N(0,1) (seed 0).  Two-level method:
one coloured overlapping multiplicative Schwarz sweep with 3x3 blocks, lumped
L2 restriction to p=1 on the same knots, one V(2,2) red-black Gauss-Seidel
cycle on the coarse level, prolongation by the transpose.  A step is one full
solve from u=0 to a 1e-10 residual reduction; the inputs are resident on the
GPU before the timed region.

value   = fine DOF/s per two-level cycle of the mixed-precision solver
          (FP32 smoother/defect/transfers/V-cycle, FP64 residual and update):
          n_fine * cycles / solve time.
Also reported: time-to-1e-10 for mixed and FP64, their ratio, the error of
both against the CPU oracle's converged solution, the roofline of the
dominant kernel (HIP-event timed inside this script) and the CPU oracle on a
bounded sample of the same workload.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0       # MI355X HBM3E, published
FP64_PEAK_TFS = 78.6        # MI355X FP64 vector, published
FP32_PEAK_TFS = 157.3       # MI355X FP32 vector, published (packed FP32 instructions)
# FP32 without packed instructions (the library is compiled without them): one
# FMA per lane per cycle, 256 CUs x 4 SIMDs x 16 lanes x 2 flops x 2.4 GHz
FP32_NONPACKED_TFS = 78.6


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--m", type=int, default=256)
    ap.add_argument("--p", type=int, default=3)
    ap.add_argument("--no-cpu-baseline", action="store_true", help="skip the CPU oracle leg (profiling runs)")
    ap.add_argument("--no-roofline", action="store_true")
    ap.add_argument("--large-m", type=int, default=4096, help="mesh of the bandwidth-regime roofline leg (0: skip)")
    ap.add_argument("--suite", action="store_true",
                    help="after the headline line, print one JSON line per other configuration")
    ap.add_argument("--only-large", action="store_true",
                    help="run only the bandwidth-regime roofline leg (for hardware-counter profiles)")
    ap.add_argument("--only-config", default="",
                    help="comma-separated configurations of the suite (C1..C5) to run alone (for profiles)")
    return ap.parse_args()


def cpu_baseline(d, p, m, b, nu, cycles_gpu):
    """The CPU oracle (plain serial C, -O2, 1 thread) on a bounded sample of the
    same workload: set-up, then the same coloured cycles from u=0, stopped
    after ~15 s of cycles.  Returns (record, converged oracle solution or None)."""
    import oracle as O
    t0 = time.perf_counter()
    orc = O.Problem(d, p, m, vcycle=True, coarse_direct=False)
    t_setup = time.perf_counter() - t0
    u = np.zeros(orc.n)
    r0 = np.linalg.norm(orc.residual(u, b))
    ncyc, t_cyc, rel = 0, 0.0, 1.0
    while rel > 1e-10 and t_cyc < 15.0 and ncyc < 60:
        t1 = time.perf_counter()
        u = orc.cycle(u, b, coarse=O.VCYCLE, cnu1=nu[0], cnu2=nu[1])
        t_cyc += time.perf_counter() - t1
        ncyc += 1
        rel = np.linalg.norm(orc.residual(u, b)) / r0
    rec = {"value": orc.n * ncyc / t_cyc, "unit": "fine DOF/s per two-level cycle", "cores": 1, "kind": "oracle",
           "sample": f"{ncyc} FP64 cycles of the same 2-D p={p} {m}x{m} coloured/V(2,2) solve from u=0 "
                     f"(relres {rel:.1e}); set-up {t_setup:.1f}s excluded",
           "seconds_per_cycle": t_cyc / ncyc, "host_cpu": _cpu_model(), "nproc": os.cpu_count()}
    return rec, (u if rel <= 1e-10 else None)


def oracle_solution(d, p, m, b, kappa=None, nu=(2, 2), tol=1e-10, max_cycles=200, aggressive=False):
    """CPU-oracle leg of the suite lines: the oracle's converged solution of the
    same coloured two-level solve (FP64, V(nu) coarse, from u=0; with
    aggressive coarsening the V-cycle runs from the 2h level), against which
    the GPU result's error is stated."""
    import oracle as O
    orc = O.Problem(d, p, m, kappa=kappa, vcycle=True, coarse_direct=False)
    u, k, _ = orc.solve(b, coarse=O.VCYCLE, cnu1=nu[0], cnu2=nu[1], tol=tol, max_cycles=max_cycles,
                        aggressive=aggressive)
    return u, k


def _cpu_model():
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def roofline_large(torch, G, m, p=3):
    """Kernels of the path in the bandwidth regime: 2-D p=3 on m x m elements
    (m=4096: 16.8 M DOFs, every vector 134 MB, above the 256 MB Infinity Cache
    together).  Algorithmic bytes per launch (kappa = 1, interior stencil in
    registers): residual 24 B/DOF (u, b read, r written); restriction 8 B per
    fine DOF read + 8 B per coarse DOF written; prolongation 16 B per fine DOF
    (u read and written) + 8 B per coarse DOF; one Schwarz colour 24 B/DOF
    (iterate read and written, right-hand side read; 12 B/DOF in FP32).  Averages over many
    launches, HIP events on the stream the library launches on."""
    prob = G.Problem(2, p, m, device=0)
    prob.setup(0, G.Opts(coarse=G.COARSE_DIRECT, precision=G.MIXED_FP32))
    n, nc = prob.n, prob.nc
    gen = torch.Generator(device="cuda").manual_seed(0)
    u = torch.rand(n, dtype=torch.float64, device="cuda", generator=gen)
    b = torch.rand(n, dtype=torch.float64, device="cuda", generator=gen)
    r = torch.empty_like(u)
    dc = torch.rand(nc, dtype=torch.float64, device="cuda", generator=gen)
    ec = torch.empty_like(dc)
    out = {"workload": f"2D p={p} {m}x{m} ({n} fine DOFs, {nc} coarse), kappa=1, FP64"}
    t = event_time(torch, lambda: prob.residual(u, b, r), 20)
    out["k_residual"] = _rl(24.0 * n, t)
    t = event_time(torch, lambda: prob.restrict(r, ec), 20)
    out["k_restrict"] = _rl(8.0 * n + 8.0 * nc, t)
    t = event_time(torch, lambda: prob.prolong_add(dc, u), 20)
    out["k_prolong_add"] = _rl(16.0 * n + 8.0 * nc, t)
    # one Schwarz colour (the streamed kernel at this size), timed by HIP
    # events inside the library on its launch stream: FP64, and FP32 as in the
    # correction cycle of the mixed solve (12 B/DOF)
    out["k_colour"] = _rl(24.0 * n, prob.time_colour(G.FP64, 5))
    out["k_colour_fp32"] = _rl(12.0 * n, prob.time_colour(G.MIXED_FP32, 5))
    # a plain device copy of one vector: calibrates byte counters (FETCH_SIZE /
    # WRITE_SIZE of this kernel against its known 8n bytes each way)
    v = torch.empty_like(u)
    t = event_time(torch, lambda: v.copy_(u), 20)
    out["copy_reference"] = _rl(16.0 * n, t)
    del v
    prob.close()
    del u, b, r, dc, ec
    torch.cuda.empty_cache()
    return out


TRAFFIC_FILE = os.path.join(ROOT, "profiles", "k_colour_2d_p3_m256_fp32_traffic.json")
KERNEL_SOURCE = os.path.join(ROOT, "paper_2009_01499_amd", "csrc", "kernels_fine.hip")


def measured_traffic():
    """HBM bytes per launch of the dominant kernel from the committed counter
    runs (FETCH_SIZE + WRITE_SIZE, calibrated against a plain copy), or None
    when the kernel source has changed since they were taken."""
    import hashlib
    try:
        rec = json.load(open(TRAFFIC_FILE))
        digest = hashlib.sha256(open(KERNEL_SOURCE, "rb").read()).hexdigest()
    except (OSError, ValueError):
        return None
    if rec.get("kernel_source_sha256") != digest:
        return None
    return rec.get("bytes_per_launch")


def _rl(bytes_per_launch, ms):
    gbs = bytes_per_launch / (ms * 1e-3) / 1e9
    return {"achieved": gbs, "peak": HBM_PEAK_GBS, "unit": "GB/s", "frac": gbs / HBM_PEAK_GBS,
            "avg_launch_us": ms * 1e3, "algorithmic_bytes_per_launch": bytes_per_launch}


def event_time(torch, fn, reps):
    """Average duration (ms) of fn() over reps calls, with HIP events on the
    current stream (the stream the library launches on)."""
    s, e = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    fn()
    torch.cuda.synchronize()
    s.record()
    for _ in range(reps):
        fn()
    e.record()
    torch.cuda.synchronize()
    return s.elapsed_time(e) / reps


def main():
    args = parse()
    if args.gpus != 1:
        print(f"bench.py runs on one GPU only (asked for --gpus {args.gpus}): sharding the path over "
              "several GPUs is not built.", file=sys.stderr)
        sys.exit(2)
    import torch

    import paper_2009_01499_amd as G
    import synth

    if args.only_large:
        print(json.dumps({"roofline_large": roofline_large(torch, G, args.large_m)}), flush=True)
        return
    if args.only_config:
        import bench_suite
        for line in bench_suite.run(torch, G, steps=max(3, args.steps // 2), only=set(args.only_config.split(","))):
            print(json.dumps(line), flush=True)
        return
    d, p, m = 2, args.p, args.m
    nu = (2, 2)
    b_np = synth.rhs_normal(d, p, m, seed=0)
    dev = torch.device("cuda:0")
    b = torch.tensor(b_np, device=dev)
    t0 = time.perf_counter()
    prob = G.Problem(d, p, m, device=0)
    prob.setup(0, G.Opts(coarse=G.COARSE_VCYCLE, precision=G.MIXED_FP32))
    torch.cuda.synchronize()
    t_setup = time.perf_counter() - t0
    n = prob.n
    o_mixed = G.Opts(coarse=G.COARSE_VCYCLE, nu1=nu[0], nu2=nu[1], precision=G.MIXED_FP32, tol=1e-10)
    o_fp64 = G.Opts(coarse=G.COARSE_VCYCLE, nu1=nu[0], nu2=nu[1], precision=G.FP64, tol=1e-10)
    u = torch.zeros_like(b)

    def solve(opts):
        u.zero_()
        _, info = prob.solve(b, u, opts)
        return info

    for _ in range(args.warmup):
        solve(o_mixed)
        solve(o_fp64)
    # ---- timed region: K mixed-precision solves
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    cycles = 0
    for _ in range(args.steps):
        cycles += solve(o_mixed).iters
    torch.cuda.synchronize()
    t_mixed = time.perf_counter() - t0
    u_mixed = u.cpu().numpy().copy()
    # ---- the same for FP64 (comparison)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    cycles64 = 0
    for _ in range(args.steps):
        cycles64 += solve(o_fp64).iters
    torch.cuda.synchronize()
    t_fp64 = time.perf_counter() - t0
    u_fp64 = u.cpu().numpy().copy()

    ms_step = 1e3 * t_mixed / args.steps
    value = n * cycles / t_mixed
    out = {
        "metric": "fine DOF/s per two-level cycle (mixed precision), with time-to-1e-10 vs FP64",
        "value": value, "unit": "fine DOF/s per cycle",
        "n_gpus": 1, "steps": args.steps, "warmup": args.warmup, "ms_per_step": ms_step,
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": "f32+f64", "data": "synthetic",
        "config": {"workload": f"2D Poisson p={p} {m}x{m} elements ({n} DOFs), coloured 3x3 Schwarz, "
                               f"p=1 coarse V({nu[0]},{nu[1]}) RB-GS, tol 1e-10, b~N(0,1) seed 0",
                   "dim": d, "p": p, "m": m, "n_fine": n, "block_width": 3, "ordering": "colour s=b"},
        "time_to_tol_ms": {"mixed": ms_step, "fp64": 1e3 * t_fp64 / args.steps},
        "cycles": {"mixed": cycles / args.steps, "fp64": cycles64 / args.steps},
        "fp64_value": n * cycles64 / t_fp64,
        "speedup_mixed_vs_fp64": t_fp64 / t_mixed,
        "setup_s": t_setup,
    }
    # ---- roofline of the dominant kernel, HIP-event timed
    if not args.no_roofline:
        # The timed mixed solve spends most of its time in the FP32 Schwarz colour
        # kernel (9 launches per cycle).  Its work per launch: one block per DOF,
        # n/b^d blocks per colour, each 2 b^d (2p+1)^d flops for the block
        # residual and 2 b^{2d} for the shared inverse: n (2(2p+1)^d + 2 b^d)
        # flops, bound by FP32 arithmetic (no dense contraction in 2-D).
        # Timed by the library with HIP events on the stream it launches on.
        bw = 3
        flops = float(n) * (2 * (2 * p + 1) ** d + 2 * bw ** d)
        ms32 = prob.time_colour(G.MIXED_FP32, 50)
        ms64 = prob.time_colour(G.FP64, 50)
        ach32 = flops / (ms32 * 1e-3) / 1e12
        ach64 = flops / (ms64 * 1e-3) / 1e12
        out["roofline"] = {"kernel": f"k_colour<2,{p},3,float,true> (one colour of the FP32 Schwarz sweep)",
                           "bound": "alu", "achieved": ach32, "peak": FP32_PEAK_TFS, "unit": "TFLOP/s",
                           "frac": ach32 / FP32_PEAK_TFS, "traffic": measured_traffic(),
                           "frac_nonpacked_fp32_peak": ach32 / FP32_NONPACKED_TFS,
                           "avg_launch_us": ms32 * 1e3, "algorithmic_flops_per_launch": flops,
                           "bytes_view": {"algorithmic_bytes_per_sweep": 12.0 * n,
                                          "GB_per_s_per_sweep": 12.0 * n / (9 * ms32 * 1e-3) / 1e9},
                           "note": "latency-bound at 66049 DOFs (0.26 MB per FP32 vector); see roofline_large"}
        out["roofline_fp64_colour"] = {"kernel": f"k_colour<2,{p},3,double,true>", "bound": "alu",
                                       "achieved": ach64, "peak": FP64_PEAK_TFS, "unit": "TFLOP/s",
                                       "frac": ach64 / FP64_PEAK_TFS, "avg_launch_us": ms64 * 1e3,
                                       "algorithmic_flops_per_launch": flops}
        uu = torch.zeros_like(b)
        r = torch.empty_like(b)
        ms_res = event_time(torch, lambda: prob.residual(uu, b, r), 100)
        ach_res = 24.0 * n / (ms_res * 1e-3) / 1e9
        out["roofline_residual"] = {"kernel": "k_residual<2,3,double,true>", "achieved": ach_res, "unit": "GB/s",
                                    "frac": ach_res / HBM_PEAK_GBS, "avg_launch_us": ms_res * 1e3,
                                    "algorithmic_bytes_per_launch": 24.0 * n}
        # a plain copy of known size: calibrates FETCH_SIZE / WRITE_SIZE in counter runs
        cal = torch.empty(1 << 23, dtype=torch.float64, device="cuda")
        cal2 = torch.empty_like(cal)
        for _ in range(3):
            cal2.copy_(cal)
        torch.cuda.synchronize()
        del cal, cal2
        if args.large_m:
            out["roofline_large"] = roofline_large(torch, G, args.large_m)
    # ---- CPU oracle leg
    if not args.no_cpu_baseline:
        rec, u_orc = cpu_baseline(d, p, m, b_np, nu, out["cycles"]["mixed"])
        out["cpu_baseline"] = rec
        if u_orc is not None:
            nrm = np.linalg.norm(u_orc)
            out["error_vs_oracle"] = {"mixed": float(np.linalg.norm(u_mixed - u_orc) / nrm),
                                      "fp64": float(np.linalg.norm(u_fp64 - u_orc) / nrm)}
    print(json.dumps(out), flush=True)
    if args.suite:
        import bench_suite
        for line in bench_suite.run(torch, G, steps=max(3, args.steps // 2)):
            print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
