"""Randomized projection of the bonds of an input MPO (Sec. 3.2, Fig.
random_update and Fig. random_env, Table 1).  Test infrastructure: only
tests/, the package's smoke check and bench.py's CPU baseline use it.

Sec. 3.2 inserts a separate randomized projector Q Q^T on each A bond and on
each B bond that a contraction sums over, which cuts that bond from chi to
k (k = O(chi^{1/2})) in the environments, O(chi^4 d^3) -> O(chi^3 k d^3),
and in the two-site contraction, O(chi^4 d^4) -> O(chi^3 k d^4).  With a
projector on every bond the contractions are those of the projected
operator

    A~ = A_1 P_1 A_2 P_2 ... P_{L-1} A_L,   P_l = Q_l Q_l^T,

so the fit of A~ B~ is what the randomized fit computes, and the projected
cores Q_{l-1}^T A_l Q_l (k x d x d x k) are formed once (reading 26).

Q_l (chi_l x k_l, k_l = min(k, chi_l)) comes from the Gaussian range finder
of Sec. 3.1 applied to the bond's row space of the core on its left: X =
core l-1 unfolded as (chi_{l-1} d^2) x chi_l, Y = X^T Omega, Q R = Y with
R_jj >= 0.  Omega is the Philox stream of module philox with bond = l and
a stream id of its own for A and for B (never one of the sweeps' ids).  A
bond with k >= chi_l keeps Q_l = I.  The projection only pays when the core
has a decaying singular spectrum across that bond (the caveat of Sec. 3.2),
so the projectors are taken from the cores as given, before any
orthogonalization.
"""
from __future__ import annotations

import numpy as np

from . import canon, philox

A_STREAM = 1 << 30
B_STREAM = (1 << 30) + 1


def bond_projectors(cores, k: int, seed: int = 0, pair: int = 0, stream: int = A_STREAM):
    """[None, Q_1, ..., Q_{L-1}, None]: Q_l is chi_l x min(k, chi_l)."""
    L = len(cores)
    Qs = [None] * (L + 1)
    for l in range(1, L):
        chi = cores[l - 1].shape[3]
        X = cores[l - 1].reshape(-1, chi)
        if k >= chi:
            Qs[l] = np.eye(chi)
            continue
        Om = philox.gaussian_matrix(X.shape[0], k, seed, pair, stream, l)
        Qs[l], _ = canon.qr_pos(X.T @ Om)
    return Qs


def project_bonds(cores, k: int, seed: int = 0, pair: int = 0, stream: int = A_STREAM):
    """The projected cores Q_{l-1}^T A_l Q_l (bond dims min(k, chi_l))."""
    Qs = bond_projectors(cores, k, seed, pair, stream)
    L = len(cores)
    out = []
    for i in range(L):
        c = np.asarray(cores[i], dtype=np.float64)
        if i > 0:  # the left bond is bond i (1-based)
            c = np.tensordot(Qs[i], c, axes=(0, 0))
        if i < L - 1:
            c = np.tensordot(c, Qs[i + 1], axes=(3, 0))
        out.append(c)
    return out


def project_pair(A, B, k: int, seed: int = 0, pair: int = 0):
    """A~ and B~ with the A and B streams."""
    return (project_bonds(A, k, seed, pair, A_STREAM), project_bonds(B, k, seed, pair, B_STREAM))
