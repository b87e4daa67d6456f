"""Seeded generators for random matrix product operators.

An MPO core has shape (chi_left, d_out, d_in, chi_right), legs ordered
(left, out, in, right) as in the paper's Sec. 2 definition of an MPO; the
boundary bonds are 1.

Recipe (all configs): ``numpy.random.default_rng(seed)`` (PCG64) draws
``standard_normal`` core by core in C order, A_1..A_L first, then B_1..B_L,
then (if asked) W_1..W_L.  Every entry is scaled by 1/sqrt(chi).  With
``decay=True`` each core l < L is multiplied along its right bond by
diag(exp(-k/6)), k = 0..chi_l-1, so that the bond spectra decay and the
randomized range finder of Sec. 3 has structure to find.

The paper's own generator (Sec. 5.1: entries uniform on [alpha, 1], then the
tensor train normalized) is available as :func:`uniform_alpha_mpo`.
"""
from __future__ import annotations

import numpy as np


def _bond_dims(L: int, chi: int) -> list[int]:
    """Nominal bond dimensions chi_0..chi_L with chi_0 = chi_L = 1."""
    return [1] + [chi] * (L - 1) + [1]


def gaussian_mpo(rng: np.random.Generator, L: int, d: int, chi: int,
                 decay: bool = False, decay_rate: float = 1.0 / 6.0) -> list[np.ndarray]:
    """Draw L Gaussian cores (chi_{l-1}, d, d, chi_l) from ``rng`` in C order."""
    dims = _bond_dims(L, chi)
    cores = []
    for l in range(L):
        shape = (dims[l], d, d, dims[l + 1])
        core = rng.standard_normal(shape) / np.sqrt(chi)
        if decay and l < L - 1:
            w = np.exp(-decay_rate * np.arange(dims[l + 1]))
            core = core * w[None, None, None, :]
        cores.append(np.ascontiguousarray(core, dtype=np.float64))
    return cores


def uniform_alpha_mpo(rng: np.random.Generator, L: int, d: int, chi: int,
                      alpha: float) -> list[np.ndarray]:
    """Entries uniform on [alpha, 1] (Sec. 5.1), each core scaled to unit
    Frobenius norm so the train stays in floating-point range."""
    dims = _bond_dims(L, chi)
    cores = []
    for l in range(L):
        core = rng.uniform(alpha, 1.0, size=(dims[l], d, d, dims[l + 1]))
        core = core / np.linalg.norm(core)
        cores.append(np.ascontiguousarray(core, dtype=np.float64))
    return cores


def string_sum_mpo(L: int, d: int, weights) -> list[np.ndarray]:
    """sum_k w_k E_k x E_k x ... x E_k over L sites, E_k the k-th d x d
    matrix unit (entry (k // d, k % d) = 1), as an MPO of bond dimension
    len(weights) <= d^2 with diagonal bonds and the weights on site 0.  The
    strings are orthonormal on every set of sites, so every bond's
    spectrum is |w| (sorted): degenerate or steep spectra on demand."""
    n = len(weights)
    if n > d * d:
        raise ValueError("at most d^2 strings")
    units = np.zeros((n, d, d))
    for k in range(n):
        units[k, k // d, k % d] = 1.0
    cores = []
    for l in range(L):
        cl = 1 if l == 0 else n
        cr = 1 if l == L - 1 else n
        core = np.zeros((cl, d, d, cr))
        for k in range(n):
            core[0 if l == 0 else k, :, :, 0 if l == L - 1 else k] = units[k] * (weights[k] if l == 0 else 1.0)
        cores.append(core)
    return cores


def reflector_product_mpo(rng: np.random.Generator, L: int, d: int) -> list[np.ndarray]:
    """A product of L orthogonal d x d matrices (bond dimension 1), each the
    Householder reflector I - 2 v v^T / (v^T v) of a Gaussian v."""
    cores = []
    for _ in range(L):
        v = rng.standard_normal(d)
        cores.append((np.eye(d) - 2.0 * np.outer(v, v) / (v @ v)).reshape(1, d, d, 1))
    return cores


def make_problem(L: int, d: int, chi_a: int, chi_b: int | None = None, seed: int = 0,
                 decay: bool = False, chi_w: int | None = None):
    """A, B (and W if ``chi_w``) drawn from one stream in the order A, B, W."""
    chi_b = chi_a if chi_b is None else chi_b
    rng = np.random.default_rng(seed)
    A = gaussian_mpo(rng, L, d, chi_a, decay)
    B = gaussian_mpo(rng, L, d, chi_b, decay)
    if chi_w is None:
        return A, B
    W = gaussian_mpo(rng, L, d, chi_w, decay=False)
    return A, B, W


def make_pair(L: int, d: int, chi: int, seed: int = 0, decay: bool = False):
    return make_problem(L, d, chi, chi, seed, decay)


def multi_pair_chis(n_pairs: int = 16, choices=(16, 32, 64, 128), seed: int = 0) -> list[int]:
    """Bond dimension of each pair of the ragged multi-pair workload."""
    rng = np.random.default_rng(seed)
    return [int(c) for c in rng.choice(np.array(choices), n_pairs)]


def make_multi_pair(n_pairs: int = 16, L: int = 24, d: int = 2, choices=(16, 32, 64, 128),
                    base_seed: int = 1000, decay: bool = True):
    """Pairs i = 0..n-1 with chi_i from :func:`multi_pair_chis`, seed base_seed + i.
    Returns a list of (A, B, chi_i)."""
    chis = multi_pair_chis(n_pairs, choices)
    out = []
    for i, chi in enumerate(chis):
        A, B = make_pair(L, d, chi, seed=base_seed + i, decay=decay)
        out.append((A, B, chi))
    return out


# Workload table: name -> generator arguments and fit options.  Sizes follow the
# five benchmark configurations of this project (plain FP64 dense check, sketch
# vs no sketch, precision, batching, differentiation).
CONFIGS = {
    "dense_L8": dict(L=8, d=2, chi=8, decay=False, seed=0, chi_c=16, sweeps=4, sketch_p=-1),
    "sketch_L20": dict(L=20, d=2, chi=32, decay=True, seed=0, chi_c=64, sweeps=6, sketch_p=10),
    "precision_L40": dict(L=40, d=2, chi=64, decay=True, seed=0, chi_c=128, sweeps=6, sketch_p=16),
    "batched_L64": dict(L=64, d=2, chi=128, decay=True, seed=0, chi_c=256, sweeps=4, sketch_p=16),
    "multipair_L24": dict(n_pairs=16, L=24, d=2, decay=True, base_seed=1000, sweeps=4, sketch_p=16),
    "grad_L30": dict(L=30, d=2, chi=64, decay=True, seed=0, chi_c=128, chi_w=32, sweeps=4,
                     sketch_p=16),
}
