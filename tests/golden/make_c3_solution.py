"""Writes c3_solution_3d_p3_m64.json: the oracle's solution of the 3-D p = 3
Poisson problem on 64 x 64 x 64 elements (274 625 fine DOFs) by the coloured
two-level method (3x3x3 blocks, colour period 3, lumped restriction to p = 1,
one V(2,2) red-black Gauss-Seidel cycle on the coarse level) from u = 0 to a
1e-10 residual reduction, b = synth.rhs_normal(3, 3, 64, seed=0): the cycle
count, the residual history, the 2-norm of the solution and its values at
3000 seeded random positions.  The benchmark's suite reads it to state the
error of the GPU solution against the oracle (the oracle's set-up at this size
takes about 20 minutes on one core).

Run from the repository root:  python tests/golden/make_c3_solution.py
"""
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
sys.path.insert(0, ROOT)
import oracle as O  # noqa: E402
import synth  # noqa: E402

D, P, M = 3, 3, 64


def main():
    t0 = time.time()
    orc = O.Problem(D, P, M, vcycle=True, coarse_direct=False)
    print(f"oracle set-up {time.time() - t0:.1f} s", flush=True)
    b = synth.rhs_normal(D, P, M, seed=0)
    u, k, hist = orc.solve(b, ordering=O.COLOUR, s=3, coarse=O.VCYCLE, cnu1=2, cnu2=2, tol=1e-10)
    print(f"oracle solve: {k} cycles, {time.time() - t0:.1f} s", flush=True)
    idx = np.sort(np.random.default_rng(17).choice(orc.n, 3000, replace=False))
    out = {
        "what": "oracle solution, 3-D p=3 m=64, coloured 3x3x3 Schwarz (s=3), V(2,2) coarse, tol 1e-10, u0=0",
        "inputs": {"b": "synth.rhs_normal(3, 3, 64, seed=0)"},
        "n": orc.n, "cycles": k, "relres_history": [repr(float(h / hist[0])) for h in hist[1:]],
        "u_l2": repr(float(np.linalg.norm(u))),
        "sample": {"index": idx.tolist(), "value": [repr(float(v)) for v in u[idx]]},
    }
    path = os.path.join(os.path.dirname(os.path.abspath(__file__)), "c3_solution_3d_p3_m64.json")
    with open(path, "w") as f:
        json.dump(out, f, separators=(",", ":"))
    print("wrote", path, os.path.getsize(path), "bytes")


if __name__ == "__main__":
    main()
