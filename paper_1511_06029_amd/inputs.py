"""Seeded synthetic inputs shared by the tests, the benchmark and the oracle.

This module only draws random numbers and lays them out; it holds none of the
method's arithmetic (no contraction, no apply, no solve).  Every generator is
deterministic in its seed (numpy PCG64), so the HIP path and the CPU oracle
always see identical arrays and no cross-language RNG parity is needed.

A QTT matrix is a list of FP64 arrays ``cores[k]`` of shape
``(r_{k-1}, m_k, n_k, r_k)`` (row-major, last index fastest); this is the
layout ``qtt_matrix_load`` takes.
"""
from __future__ import annotations

import numpy as np

__all__ = [
    "rng", "gaussian_qtt", "perturbed_identity_pair", "identity_qtt",
    "rhs", "uneven_widths", "poisson_arrivals", "serving_operators",
    "WORKLOADS",
]


def rng(seed):
    return np.random.Generator(np.random.PCG64(int(seed)))


def gaussian_qtt(ranks, m, n=None, seed=0):
    """Cores with i.i.d. N(0,1) entries scaled by 1/sqrt(n_k r_{k-1}), so a
    core maps unit-variance inputs to unit-variance outputs."""
    n = m if n is None else n
    g = rng(seed)
    cores = []
    for k in range(len(m)):
        shape = (ranks[k], m[k], n[k], ranks[k + 1])
        cores.append(g.standard_normal(shape) / np.sqrt(n[k] * ranks[k]))
    return cores


def identity_qtt(m):
    """Rank-1 cores delta(i_k, j_k): the identity as a Kronecker product of
    identities."""
    return [np.eye(mk).reshape(1, mk, mk, 1).copy() for mk in m]


def perturbed_identity_pair(ranks, m, seed=0, eps=0.1):
    """A diagonally dominant operator and an approximate inverse of the same
    ranks.

    With E_k(a, i, j, b) = [a == 0][b == 0][i == j] (the identity sitting in
    rank channel 0) and g_k i.i.d. N(0,1) scaled by 1/sqrt(m_k r_{k-1}):
        A    cores: E_k + eps * g_k
        Ainv cores: E_k - eps * g_k
    The product Ainv A equals I up to second order in eps."""
    g = rng(seed)
    A, Ainv = [], []
    for k in range(len(m)):
        shape = (ranks[k], m[k], m[k], ranks[k + 1])
        pert = eps * g.standard_normal(shape) / np.sqrt(m[k] * ranks[k])
        E = np.zeros(shape)
        E[0, :, :, 0] = np.eye(m[k])
        A.append(E + pert)
        Ainv.append(E - pert)
    return A, Ainv


def rhs(N, K, seed=0):
    """N x K block of N(0,1) right-hand sides (Fortran order: columns
    contiguous)."""
    return np.asfortranarray(rng(seed).standard_normal((N, K)))


def uneven_widths(nblocks=64, seed=0, choices=(1, 2, 4, 8, 16, 32)):
    """Widths of uneven RHS blocks drawn uniformly from `choices`."""
    return [int(x) for x in rng(seed).choice(np.asarray(choices), size=nblocks)]


def poisson_arrivals(n_requests, rate_per_s, seed=0):
    """Arrival times (seconds from 0) of a Poisson stream."""
    gaps = rng(seed).exponential(1.0 / rate_per_s, size=n_requests)
    return np.cumsum(gaps)


def serving_operators(n_ops=12, levels=(5, 6, 7, 8), rank_lo=16, rank_hi=32, seed=0):
    """Descriptions of resident operators: level count L drawn from `levels`,
    one interior rank r drawn from [rank_lo, rank_hi], profile [1, r, ..., r, 1],
    mode size 8."""
    g = rng(seed)
    ops = []
    for t in range(n_ops):
        L = int(g.choice(np.asarray(levels)))
        r = int(g.integers(rank_lo, rank_hi + 1))
        ops.append({"L": L, "ranks": [1] + [r] * (L - 1) + [1], "seed": seed * 1000 + t})
    return ops


# Workloads of the paper's volume problems (mode-8 octree digits, ranks <= 32).
WORKLOADS = {
    "volume_L4": {"L": 4, "eps": 1e-10, "K": 1, "rhs_seed": 11},
    "synthetic_L6": {"L": 6, "ranks": [1, 16, 32, 32, 32, 16, 1], "K": (1, 16),
                     "core_seed": 21, "rhs_seed": 22},
    "refine_L7": {"L": 7, "ranks": [1, 24, 32, 32, 32, 32, 24, 1], "K": 8,
                  "eps": 0.1, "core_seed": 31, "rhs_seed": 32, "rtol": 1e-8},
    "batched_L7": {"L": 7, "ranks": [1, 24, 32, 32, 32, 32, 24, 1], "nblocks": 64,
                   "core_seed": 41, "width_seed": 42, "rhs_seed": 43},
    "serving": {"n_ops": 12, "levels": (5, 6, 7, 8), "rate": 200.0, "k_max": 16,
                "budget_bytes": 200 * 10 ** 9, "seed": 51},
}
