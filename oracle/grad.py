"""Gradient of the fitted product at frozen truncation bases (FP64 oracle;
test infrastructure, see oracle/__init__.py).

This part is not in the paper: it differentiates the result of the serial
fit (Alg. 5) with respect to the input cores, holding every truncation basis
fixed.  After the last sweep C is in site-canonical form with its
orthogonality centre at one end (the last site after a forward sweep, the
first after a backward one, Alg. 3): all other cores are isometries.  With
those isometries frozen, the fit of a product X is the orthogonal projection
Pi(X) onto the MPOs that share them and have a free centre core (the centre
of the best approximation in that set, Sec. 2.3.2).  For a fixed MPO W:

    loss(A, B) = <W, Pi(A B)>_F = <Pi(W), A B>_F,

linear in every core of A and of B.  Pi(W) keeps the isometries and takes
the centre core from the two-layer environment of (isometries, W); the
gradient with respect to A_l (B_l) is the network <Pi(W), A B> with A_l (B_l)
removed, closed with the three-layer left and right environments of
(Pi(W), A, B) (Sec. 2.3.3, Fig. envs).

Pins (tests/test_oracle_grad.py): brute-force dense projector on tiny chains;
central finite differences (exact up to rounding for a multilinear loss);
an independent torch.autograd FP64 evaluation; Pi idempotent and symmetric.
"""
from __future__ import annotations

import numpy as np

from .fit import env_left, env_right


def projected_w(C, centre, W):
    """Cores of Pi(W): C's isometries and the centre core of W's projection.
    C must have its centre at site 0 or at site L-1 (0-based)."""
    L = len(C)
    if centre == L - 1:
        E = np.ones((1, 1))
        for l in range(L - 1):
            T = np.tensordot(E, C[l], axes=([0], [0]))            # [w, s, u, c']
            E = np.tensordot(T, W[l], axes=([0, 1, 2], [0, 1, 2]))  # [c', w']
        mid = np.tensordot(E, W[L - 1], axes=([1], [0]))           # [c, s, u, 1]
        return [np.array(c, copy=True) for c in C[:L - 1]] + [mid]
    if centre == 0:
        F = np.ones((1, 1))
        for l in range(L - 1, 0, -1):
            T = np.tensordot(C[l], F, axes=([3], [0]))              # [c, s, u, w']
            F = np.tensordot(T, W[l], axes=([1, 2, 3], [1, 2, 3]))  # [c, w]
        mid = np.tensordot(W[0], F, axes=([3], [1]))               # [1, s, u, c]
        return [mid] + [np.array(c, copy=True) for c in C[1:]]
    raise ValueError("the centre must be the first or the last site")


def loss(A, B, C, centre, W) -> float:
    P = projected_w(C, centre, W)
    E = np.ones((1, 1, 1))
    for p, a, b in zip(P, A, B):
        E = env_left(E, p, a, b)
    return float(E.reshape(-1)[0])


def grad(A, B, C, centre, W):
    """(loss, [dloss/dA_l], [dloss/dB_l]) by left / right environments."""
    P = projected_w(C, centre, W)
    L = len(A)
    Le = [None] * (L + 1)
    Re = [None] * (L + 1)
    Le[0] = np.ones((1, 1, 1))
    Re[L] = np.ones((1, 1, 1))
    for l in range(L):
        Le[l + 1] = env_left(Le[l], P[l], A[l], B[l])
    for l in range(L - 1, -1, -1):
        Re[l] = env_right(Re[l + 1], P[l], A[l], B[l])
    gA, gB = [], []
    for l in range(L):
        # T[a, b, s, u, x'] = sum_x Le[x, a, b] P[x, s, u, x']
        T = np.tensordot(Le[l], P[l], axes=([0], [0]))
        # close with R[x', a', b']: T2[a, b, s, u, a', b']
        T2 = np.tensordot(T, Re[l + 1], axes=([4], [0]))
        # dA[a, s, t, a'] = sum_{b, u, b'} T2[a, b, s, u, a', b'] B[b, t, u, b']
        gA.append(np.tensordot(T2, B[l], axes=([1, 3, 5], [0, 2, 3])).transpose(0, 1, 3, 2))
        # dB[b, t, u, b'] = sum_{a, s, a'} T2[a, b, s, u, a', b'] A[a, s, t, a']
        gB.append(_gB(T2, A[l]))
    return float(Le[L].reshape(-1)[0]), gA, gB


def _gB(T2, A):
    # T2[a, b, s, u, a', b'] A[a, s, t, a'] -> [b, u, b', t] -> [b, t, u, b']
    G = np.tensordot(T2, A, axes=([0, 2, 4], [0, 1, 3]))
    return G.transpose(0, 3, 1, 2)
