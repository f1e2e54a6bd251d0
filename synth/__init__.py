"""Seeded synthetic inputs shared by the oracle tests, the GPU tests and the benchmark.

This module holds none of the solver's arithmetic: it only draws random numbers
and shapes them.  Every generator is a pure function of its integer seed
(``numpy.random.Generator(PCG64(seed))``), so both sides of a parity test read
identical bits.

Workload recipes (the paper fixes none of these; it solves one manufactured
problem and reports convergence with random initial guesses):
  * right-hand sides: the load vector itself is i.i.d. N(0,1) per interior DOF;
  * random initial guesses: i.i.d. U(-1,1) per DOF (asymptotic-rate runs);
  * coefficient fields: kappa = exp(g) per element, g a zero-mean Gaussian field
    with separable squared-exponential covariance sigma^2 exp(-|x-y|^2 / (2 l^2))
    sampled at element centroids;
  * batches: per-problem (m, p) drawn from a SeedSequence spawn.
"""
from __future__ import annotations

import numpy as np


def rng(seed: int) -> np.random.Generator:
    return np.random.Generator(np.random.PCG64(seed))


def n_dofs(d: int, p: int, m: int) -> int:
    """Interior DOFs of the degree-p, C^{p-1} space on m^d elements: (m+p-2)^d."""
    return (m + p - 2) ** d


def rhs_normal(d: int, p: int, m: int, seed: int = 0) -> np.ndarray:
    """Load vector b ~ N(0,1) i.i.d. per interior DOF (x-fastest order)."""
    return rng(seed).standard_normal(n_dofs(d, p, m))


def initial_guess(d: int, p: int, m: int, seed: int = 0) -> np.ndarray:
    """Random initial guess, U(-1,1) per DOF."""
    return rng(seed).uniform(-1.0, 1.0, n_dofs(d, p, m))


def _se_factor(m: int, sigma: float, ell: float) -> np.ndarray:
    """Square-root factor L (L L^T = C) of the 1-D squared-exponential covariance on
    the m element centroids, from the symmetric eigendecomposition (negative
    round-off eigenvalues clipped to zero)."""
    x = (np.arange(m) + 0.5) / m
    C = sigma ** 2 * np.exp(-(x[:, None] - x[None, :]) ** 2 / (2.0 * ell ** 2))
    lam, V = np.linalg.eigh(C)
    return V * np.sqrt(np.clip(lam, 0.0, None))[None, :]


def kappa_grf(d: int, m: int, sigma: float, ell: float, seed: int) -> np.ndarray:
    """kappa_e = exp(g_e) per element (x fastest), g a separable SE Gaussian field."""
    L = _se_factor(m, sigma, ell)
    z = rng(seed).standard_normal((m,) * d)          # indices (z, y, x) in C order
    g = z
    for axis in range(d):
        g = np.moveaxis(np.tensordot(L, g, axes=([1], [axis])), 0, axis)
    return np.exp(g).ravel().copy()


def batch_specs(nprob: int = 256, seed: int = 4, m_lo: int = 32, m_hi: int = 128, p_choices=(2, 3, 4)):
    """Per-problem (m, p, kappa-seed, rhs-seed) from SeedSequence(seed).spawn(nprob)."""
    specs = []
    for child in np.random.SeedSequence(seed).spawn(nprob):
        g = np.random.Generator(np.random.PCG64(child))
        m = int(g.integers(m_lo, m_hi + 1))
        p = int(g.choice(p_choices))
        ks, rs = (int(v) for v in g.integers(0, 2 ** 31 - 1, size=2))
        specs.append({"m": m, "p": p, "kappa_seed": ks, "rhs_seed": rs})
    return specs
