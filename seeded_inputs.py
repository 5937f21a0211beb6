"""Seeded synthetic inputs shared by the oracle, the tests and the benchmark.

This module draws random numbers and lays out parameter lists; it holds none of the
method's arithmetic (no residual, no decoder, no solver).  Every generator is a
numpy PCG64 stream keyed by an explicit integer seed, so the oracle and the HIP path
receive bit-identical inputs.

Contents
  * parameter sets mu = (a, lambda) on the Burgers box D = [1, 1e4] x [5, 20] (the paper's own
    workload uses lambda in [5, 25]: the range is an argument) as tensor linspace training grids
    and uniform held-out draws,
  * the Gaussian test matrix C of the weak compatibility constraint
    (Section 3.1: C has i.i.d. normal entries),
  * Glorot-uniform initial weights for the shallow masked autoencoders,
  * random latent vectors and multipliers for kernel-level parity cases.
"""
from __future__ import annotations

import numpy as np

A_RANGE = (1.0, 1.0e4)
LAM_RANGE = (5.0, 20.0)


def rng(seed: int) -> np.random.Generator:
    return np.random.Generator(np.random.PCG64(int(seed)))


def training_grid(n_a: int, n_lam: int, lam_range=LAM_RANGE) -> np.ndarray:
    """Tensor grid of (a, lambda), endpoints included, a-fastest.  Shape [n_a*n_lam, 2]."""
    a = np.linspace(A_RANGE[0], A_RANGE[1], n_a)
    lam = np.linspace(lam_range[0], lam_range[1], n_lam)
    aa, ll = np.meshgrid(a, lam, indexing="xy")
    return np.stack([aa.ravel(), ll.ravel()], axis=1).astype(np.float64)


def heldout_mu(n: int, seed: int, exclude: np.ndarray | None = None, lam_range=LAM_RANGE) -> np.ndarray:
    """n parameter points drawn uniformly from D, rejecting exact hits on `exclude`."""
    g = rng(seed)
    out = []
    ex = set() if exclude is None else {tuple(p) for p in np.asarray(exclude)}
    while len(out) < n:
        p = (g.uniform(*A_RANGE), g.uniform(*lam_range))
        if p not in ex:
            out.append(p)
    return np.asarray(out, dtype=np.float64).reshape(n, 2)


def gaussian_matrix(rows: int, cols: int, seed: int) -> np.ndarray:
    """i.i.d. N(0,1) matrix (row-major float64)."""
    return rng(seed).standard_normal((rows, cols))


def glorot_uniform(fan_in: float, fan_out: float, shape, g: np.random.Generator) -> np.ndarray:
    bound = np.sqrt(6.0 / (float(fan_in) + float(fan_out)))
    return g.uniform(-bound, bound, size=shape)


def uniform(shape, lo: float, hi: float, seed: int) -> np.ndarray:
    return rng(seed).uniform(lo, hi, size=shape)


def normal(shape, seed: int, scale: float = 1.0) -> np.ndarray:
    return scale * rng(seed).standard_normal(size=shape)


def spawn_seeds(seed: int, n: int) -> list[int]:
    """n independent child seeds derived from one seed (SeedSequence.spawn)."""
    ss = np.random.SeedSequence(int(seed))
    return [int(c.generate_state(1)[0]) for c in ss.spawn(n)]


def mlp_init(sizes, seed: int) -> list:
    """Glorot-uniform weights and zero biases of a dense network with layer widths `sizes`
    (input first).  Returns [(W [out][in], b [out]), ...]; one spawned seed per layer."""
    seeds = spawn_seeds(seed, len(sizes) - 1)
    out = []
    for k in range(len(sizes) - 1):
        fi, fo = sizes[k], sizes[k + 1]
        out.append((glorot_uniform(fi, fo, (fo, fi), rng(seeds[k])), np.zeros(fo)))
    return out


def train_split(n: int, frac_test: float, seed: int):
    """Seeded permutation of range(n) split into (train, test) index arrays."""
    p = rng(seed).permutation(n)
    n_test = int(round(frac_test * n))
    return np.sort(p[n_test:]), np.sort(p[:n_test])


def epoch_order(n: int, seed: int, epoch: int) -> np.ndarray:
    """Minibatch visiting order of one training epoch (a seeded permutation of range(n))."""
    return np.random.Generator(np.random.PCG64([int(seed), int(epoch)])).permutation(n)


def model_assignment(n: int, n_models: int, seed: int) -> np.ndarray:
    """Model index of each of n solves, split evenly over n_models in a seeded random order."""
    return rng(seed).permutation(np.arange(n) % n_models)
