"""Writes grid_3d_p3_m64.json: oracle values of the fine residual r = b - A u,
one coloured Schwarz sweep (3x3x3 blocks, colour period 3) and one two-level
cycle (coloured sweep, lumped restriction to p = 1, one V(2,2) red-black
Gauss-Seidel cycle on the coarse level, prolongation) for the 3-D p = 3
Poisson problem on 64 x 64 x 64 elements (274 625 fine DOFs), at sampled
positions, plus the 2-norms of the whole vectors.

Inputs are the seeded synthetic vectors of `synth` (u: initial_guess seed 1,
b: rhs_normal seed 0).  Samples: 1500 uniform random positions plus every 4th
point (in both in-plane directions) of the two outermost grid planes next to
each of the six faces, where rows differ from the interior stencil.  The
oracle's brute-force 3-D assembly at this size takes about 20 minutes on one
core, so the GPU tests read the file.

Run from the repository root:  python tests/golden/make_grid_3d.py
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


def samples(n1: int, count: int, seed: int) -> np.ndarray:
    rng = np.random.default_rng(seed)
    idx = set(rng.integers(0, n1 ** 3, count).tolist())
    for plane in (0, 1, n1 - 2, n1 - 1):
        for a in range(0, n1, 4):
            for c in range(0, n1, 4):
                idx.add(plane + n1 * a + n1 * n1 * c)      # x = plane
                idx.add(a + n1 * plane + n1 * n1 * c)      # y = plane
                idx.add(a + n1 * c + n1 * n1 * plane)      # z = plane
    return np.array(sorted(idx), dtype=np.int64)


def main():
    t0 = time.time()
    orc = O.Problem(D, P, M, vcycle=True, coarse_direct=False)
    print(f"oracle set-up {time.time() - t0:.1f} s", flush=True)
    u = synth.initial_guess(D, P, M, seed=1)
    b = synth.rhs_normal(D, P, M, seed=0)
    r = orc.residual(u, b)
    sw = orc.sweep(u, b, ordering=O.COLOUR, s=3)
    cy = orc.cycle(u, b, ordering=O.COLOUR, s=3, coarse=O.VCYCLE, cnu1=2, cnu2=2)
    print(f"oracle operations done {time.time() - t0:.1f} s", flush=True)
    fi = samples(orc.n1, 1500, 13)

    def rec(v):
        return {"index": fi.tolist(), "value": [repr(float(x)) for x in v[fi]], "l2": repr(float(np.linalg.norm(v)))}

    out = {
        "what": "oracle residual, one coloured sweep (s=3) and one two-level cycle (V(2,2) coarse); 3-D p=3 m=64",
        "inputs": {"u": "synth.initial_guess(3, 3, 64, seed=1)", "b": "synth.rhs_normal(3, 3, 64, seed=0)"},
        "n": orc.n, "nc": orc.nc,
        "residual": rec(r), "sweep": rec(sw), "cycle": rec(cy),
    }
    path = os.path.join(os.path.dirname(os.path.abspath(__file__)), "grid_3d_p3_m64.json")
    with open(path, "w") as f:
        json.dump(out, f, separators=(",", ":"))
    print("wrote", path, os.path.getsize(path), "bytes")


if __name__ == "__main__":
    main()
