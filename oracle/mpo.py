"""MPO utilities of the oracle (Sec. 2): dense expansion, naive product
(Alg. 1), Frobenius inner products and norms, and the two error measures.

Cores are (chi_left, d_out, d_in, chi_right) as in the Sec. 2 definition.  The
product C = A B contracts the input leg of A with the output leg of B (Sec. 2,
Fig. mpo_mpo (a)); C's cores carry (left, out = A's out, in = B's in, right).

Pins (tests/test_oracle_mpo.py): dense expansion against explicit index sums;
naive product against the dense matrix product; inner product, norm and
difference norm against dense Frobenius values.
"""
from __future__ import annotations

import numpy as np


def bond_dims(cores) -> list[int]:
    return [cores[0].shape[0]] + [c.shape[3] for c in cores]


def dense(cores) -> np.ndarray:
    """The d^L x d^L matrix X(x, y) of an MPO, x = (x_1..x_L) row-major with x_1
    the most significant digit (Sec. 2)."""
    T = cores[0]  # (1, d, d, chi)
    T = T.reshape(T.shape[1], T.shape[2], T.shape[3])  # (X, Y, chi)
    for core in cores[1:]:
        # T[X, Y, a] core[a, s, t, a'] -> [X s, Y t, a']
        T = np.einsum("xya,astb->xsytb", T, core)
        X, s, Y, t, b = T.shape
        T = T.reshape(X * s, Y * t, b)
    return T[:, :, 0]


def naive_product(A, B):
    """Alg. 1: C_l(i_a, i_b, s, u, j_a, j_b) = sum_t A_l(i_a, s, t, j_a) B_l(i_b, t, u, j_b),
    regrouped into bonds of dimension chi_A * chi_B (Sec. 2.1)."""
    C = []
    for a, b in zip(A, B):
        c = np.einsum("astc,btud->absucd", a, b)
        ca, d1, _, cc = a.shape
        cb, _, d2, cd = b.shape  # C's input leg is B's (1 for an MPS)
        C.append(np.ascontiguousarray(c.reshape(ca * cb, d1, d2, cc * cd)))
    return C


def transfer_inner(X, Y) -> float:
    """<X, Y>_F = sum_{x,y} X(x,y) Y(x,y) by a left-to-right transfer pass
    (real entries, no conjugation)."""
    E = np.ones((1, 1))
    for x, y in zip(X, Y):
        # E[a, b] x[a, s, t, a'] y[b, s, t, b'] -> E'[a', b']
        T = np.tensordot(E, x, axes=([0], [0]))                # [b, s, t, a']
        E = np.tensordot(T, y, axes=([0, 1, 2], [0, 1, 2]))    # [a', b']
    return float(E[0, 0])


def three_layer_inner(C, A, B) -> float:
    """<C, A B>_F via left environments of the (C, A, B) network (Sec. 2.3.3)."""
    E = np.ones((1, 1, 1))
    for c, a, b in zip(C, A, B):
        T = np.tensordot(E, a, axes=([1], [0]))              # [x, z, s, t, Y]
        T = np.tensordot(T, b, axes=([1, 3], [0, 1]))        # [x, s, Y, u, Z]
        E = np.tensordot(c, T, axes=([0, 1, 2], [0, 1, 3]))  # [X, Y, Z]
    return float(E[0, 0, 0])


def product_norm2(A, B) -> float:
    """||A B||_F^2 by a four-layer transfer pass, O(L chi^5 d^3) (FP64)."""
    E = np.ones((1, 1, 1, 1))  # [p, q, r, s]: bonds of A, B, A, B
    for a, b in zip(A, B):
        # sum over the outer legs x, u and the inner legs t, v of each copy
        T = np.tensordot(E, a, axes=([0], [0]))                # [q, r, s, x, t, P]
        T = np.tensordot(T, b, axes=([0, 4], [0, 1]))          # [r, s, x, P, u, Q]
        T = np.tensordot(T, a, axes=([0, 2], [0, 1]))          # [s, P, u, Q, v, R]
        E = np.tensordot(T, b, axes=([0, 4, 2], [0, 1, 2]))    # [P, Q, R, S]
    return float(E[0, 0, 0, 0])


def left_orth_norm(cores) -> float:
    """Frobenius norm of an MPO by a Householder-QR left-orthogonalization
    sweep: the norm ends up in the last core (Sec. 2.3.1, site-canonical form)."""
    carry = np.ones((1, 1))
    for core in cores:
        c = np.tensordot(carry, core, axes=(1, 0))  # (r, d, d, chi)
        r, d1, d2, chi = c.shape
        X = c.reshape(r * d1 * d2, chi)
        if X.shape[0] >= X.shape[1]:
            _, R = np.linalg.qr(X)
        else:
            R = X
        carry = R
    return float(np.linalg.norm(carry))


def diff_norm(X, Y) -> float:
    """||X - Y||_F of two MPOs on the same sites from the direct-sum MPO of X and
    -Y, left-orthogonalized by Householder QR.  Accurate to ~1e-15 relative,
    unlike <X,X> - 2<X,Y> + <Y,Y>, which floors at sqrt(machine eps) (the caveat
    of Sec. 5.2)."""
    L = len(X)
    D = []
    for l in range(L):
        x, y = X[l], Y[l]
        xl, d1, d2, xr = x.shape
        yl, _, _, yr = y.shape
        if L == 1:
            D.append(x - y)
        elif l == 0:
            D.append(np.concatenate([x, -y], axis=3))
        elif l == L - 1:
            D.append(np.concatenate([x, y], axis=0))
        else:
            z = np.zeros((xl + yl, d1, d2, xr + yr))
            z[:xl, :, :, :xr] = x
            z[xl:, :, :, xr:] = y
            D.append(z)
    return left_orth_norm(D)


def rel_diff(C, Cref) -> float:
    """Parity measure: ||C - Cref||_F / ||Cref||_F as operators."""
    return diff_norm(C, Cref) / left_orth_norm(Cref)


def fit_error_dense(A, B, C) -> float:
    """||A B - C||_F / ||A B||_F from dense matrices (small L only)."""
    P = dense(A) @ dense(B)
    return float(np.linalg.norm(P - dense(C)) / np.linalg.norm(P))


def fit_error_transfer(A, B, C, ab_norm2: float | None = None) -> float:
    """eps^2 = 1 + (||C||^2 - 2 <C, AB>) / ||AB||^2 from transfer passes; floors
    near sqrt(machine eps) (Sec. 5.2)."""
    n2 = product_norm2(A, B) if ab_norm2 is None else ab_norm2
    cc = left_orth_norm(C) ** 2
    cab = three_layer_inner(C, A, B)
    return float(np.sqrt(max(0.0, n2 - 2.0 * cab + cc) / n2))
