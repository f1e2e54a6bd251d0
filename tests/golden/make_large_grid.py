"""Writes large_grid_2d_p3_m1024.json: oracle values of the fine residual
r = b - A u, the restriction d_c = R x and the prolongation update
u + P e_c (lumped L2 transfer to p = 1 on the same knots) for the 2-D p = 3
problem on 1024 x 1024 elements (1 050 625 fine DOFs), at sampled positions.

Inputs are the seeded synthetic vectors of `synth` (u: initial_guess seed 1,
b: rhs_normal seed 0, x: rhs_normal seed 3, e_c: rhs_normal at p = 1
seed 4).  Samples: 1500
uniform random positions plus every 4th point of the two outermost grid lines
on each side (where rows differ from the interior stencil).  The oracle's
set-up at this size takes about 90 s on one core; the GPU tests read the file.

Run from the repository root:  python tests/golden/make_large_grid.py
"""
import json
import os
import sys

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
sys.path.insert(0, ROOT)
import oracle as O  # noqa: E402
import synth  # noqa: E402

D, P, M = 2, 3, 1024


def samples(n1: int, count: int, seed: int) -> np.ndarray:
    rng = np.random.default_rng(seed)
    idx = set(rng.integers(0, n1 * n1, count).tolist())
    for line in (0, 1, n1 - 2, n1 - 1):
        for k in range(0, n1, 4):
            idx.add(line * n1 + k)   # grid row
            idx.add(k * n1 + line)   # grid column
    return np.array(sorted(idx), dtype=np.int64)


def main():
    orc = O.Problem(D, P, M, vcycle=False, coarse_direct=False)
    u = synth.initial_guess(D, P, M, seed=1)
    b = synth.rhs_normal(D, P, M, seed=0)
    x = synth.rhs_normal(D, P, M, seed=3)
    ec = synth.rhs_normal(D, 1, M, seed=4)
    r = orc.residual(u, b)
    dc = orc.restrict(x)
    up = orc.prolong_add(ec, u)
    sw = orc.sweep(u, b, ordering=O.COLOUR, s=3)
    fi = samples(orc.n1, 1500, 11)
    ci = samples(orc.n1c, 1500, 12)
    out = {
        "what": "oracle residual, restriction, prolongation update, one coloured sweep; 2-D p=3 m=1024",
        "inputs": {"u": "synth.initial_guess(2, 3, 1024, seed=1)", "b": "synth.rhs_normal(2, 3, 1024, seed=0)",
                   "x": "synth.rhs_normal(2, 3, 1024, seed=3)", "e_c": "synth.rhs_normal(2, 1, 1024, seed=4)"},
        "n": orc.n, "nc": orc.nc,
        "residual": {"index": fi.tolist(), "value": [repr(float(v)) for v in r[fi]]},
        "prolong_add": {"index": fi.tolist(), "value": [repr(float(v)) for v in up[fi]]},
        "restrict": {"index": ci.tolist(), "value": [repr(float(v)) for v in dc[ci]]},
        "sweep": {"index": fi.tolist(), "value": [repr(float(v)) for v in sw[fi]]},
        "norms": {"residual_l2": repr(float(np.linalg.norm(r))), "restrict_l2": repr(float(np.linalg.norm(dc))),
                  "prolong_l2": repr(float(np.linalg.norm(up))), "sweep_l2": repr(float(np.linalg.norm(sw)))},
    }
    path = os.path.join(os.path.dirname(os.path.abspath(__file__)), "large_grid_2d_p3_m1024.json")
    with open(path, "w") as f:
        json.dump(out, f, separators=(",", ":"))
    print("wrote", path, os.path.getsize(path), "bytes")


if __name__ == "__main__":
    main()
