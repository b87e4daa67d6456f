"""Canonical forms of the oracle (Sec. 2.3.1).

* Site-canonical form: QR sweeps from the left and RQ sweeps from the right.
  The QR is Householder (LAPACK via numpy) with the sign convention R_jj >= 0,
  which makes the factorization unique for full column rank.  Where a core
  reshaped to a (rows x cols) matrix has fewer rows than columns the bond is
  clipped: the orthogonal factor is the identity and the whole matrix is
  carried into the neighbour.
* Vidal / inverse canonical form: from a right-canonical train, a left-to-right
  SVD sweep gives Lambda_l and Psi_l = Lambda_{l-1} Gamma_l Lambda_l = U_l S_l,
  Y_l = Lambda_l^{-1}; then every Psi_l Y_l is left orthogonal and every
  Y_{l-1} Psi_l is right orthogonal.  Singular values at or below
  INV_TRUNC * sigma_1 are truncated before the inversion, as the paper allows
  for stability (Sec. 2.3.1, inverse canonical form): they, their singular
  vectors and their Y entries become zero, so the bond keeps its size with
  zero padding and Psi_l Y_l stays a (partial) isometry.

Pins (tests/test_oracle_canon.py): the dense operator is unchanged by every
gauge routine; orthogonality relations of each form; Householder QR with the
sign convention equals the Cholesky factor of the Gram matrix (uniqueness).
"""
from __future__ import annotations

import numpy as np


def qr_pos(X: np.ndarray):
    """Economic Householder QR, X = Q R with R_jj >= 0."""
    Q, R = np.linalg.qr(X)
    s = np.where(np.diag(R) < 0, -1.0, 1.0)
    return Q * s[None, :], R * s[:, None]


def sign_fix_columns(U: np.ndarray):
    """Sign of each column chosen so its largest-magnitude entry is positive
    (first index on ties).  Returns the +-1 vector."""
    idx = np.argmax(np.abs(U), axis=0)
    s = np.sign(U[idx, np.arange(U.shape[1])])
    s[s == 0] = 1.0
    return s


def left_orthogonalize(cores):
    """QR sweep l = 1..L-1 (Alg. 5 preprocessing), then the norm is split off
    the last core.  Returns (left-orthogonal cores, Frobenius norm)."""
    cores = [np.array(c, dtype=np.float64, copy=True) for c in cores]
    L = len(cores)
    for l in range(L - 1):
        cl, d1, d2, cr = cores[l].shape
        X = cores[l].reshape(cl * d1 * d2, cr)
        if X.shape[0] >= X.shape[1]:
            Q, R = qr_pos(X)
        else:
            Q, R = np.eye(X.shape[0]), X
        cores[l] = Q.reshape(cl, d1, d2, Q.shape[1])
        cores[l + 1] = np.tensordot(R, cores[l + 1], axes=(1, 0))
    nu = float(np.linalg.norm(cores[-1]))
    cores[-1] = cores[-1] / nu
    return cores, nu


def right_orthogonalize(cores):
    """RQ sweep l = L..2 (Sec. 2.3.1): each core becomes right orthogonal and the
    remaining factor moves left.  Uses X^T = Q R (R_jj >= 0), i.e. X = R^T Q^T."""
    cores = [np.array(c, dtype=np.float64, copy=True) for c in cores]
    L = len(cores)
    for l in range(L - 1, 0, -1):
        cl, d1, d2, cr = cores[l].shape
        X = cores[l].reshape(cl, d1 * d2 * cr)
        if X.shape[0] <= X.shape[1]:
            Qt, Rt = qr_pos(X.T)
            core, carry = Qt.T, Rt.T
        else:
            core, carry = np.eye(X.shape[1]), X
        cores[l] = core.reshape(core.shape[0], d1, d2, cr)
        cores[l - 1] = np.tensordot(cores[l - 1], carry, axes=(3, 0))
    return cores


def mixed_canonical(cores, left):
    """Site-canonical form around the two sites left, left+1 (0-based, Sec.
    2.3.1): QR sweep over sites 0..left-1 (carried into site `left`) and RQ
    sweep over sites L-1..left+2 (carried into site left+1), with the same
    clipping rule as left_orthogonalize / right_orthogonalize.  The two
    centre sites hold everything else; the operator is unchanged."""
    cores = [np.array(c, dtype=np.float64, copy=True) for c in cores]
    L = len(cores)
    for l in range(left):
        cl, d1, d2, cr = cores[l].shape
        X = cores[l].reshape(cl * d1 * d2, cr)
        if X.shape[0] >= X.shape[1]:
            Q, R = qr_pos(X)
        else:
            Q, R = np.eye(X.shape[0]), X
        cores[l] = Q.reshape(cl, d1, d2, Q.shape[1])
        cores[l + 1] = np.tensordot(R, cores[l + 1], axes=(1, 0))
    for l in range(L - 1, left + 1, -1):
        cl, d1, d2, cr = cores[l].shape
        X = cores[l].reshape(cl, d1 * d2 * cr)
        if X.shape[0] <= X.shape[1]:
            Qt, Rt = qr_pos(X.T)
            core, carry = Qt.T, Rt.T
        else:
            core, carry = np.eye(X.shape[1]), X
        cores[l] = core.reshape(core.shape[0], d1, d2, cr)
        cores[l - 1] = np.tensordot(cores[l - 1], carry, axes=(3, 0))
    return cores


# Relative cut of singular values (truncation before inversion, Sec. 2.3.1,
# and the drop rule of the two-site update): values at or below
# INV_TRUNC * sigma_1 are set to zero.  At this level an FP64 singular
# value decomposition still fixes the vectors of the smallest kept values to
# about 1e-10, and 1/sigma amplifies rounding by at most 1e6.
INV_TRUNC = 1e-6


def truncate_inverse(U, S, Vt, thresh: float = INV_TRUNC):
    """Zero the singular triplets with S_j <= thresh * S_0 (Sec. 2.3.1: very
    small singular values may be truncated before they are inverted).
    Returns (U, S, Vt, Y, count) with Y the pseudo-inverse of diag(S)."""
    keep = S > thresh * S[0] if len(S) else np.zeros(0, dtype=bool)
    U = U * keep[None, :]
    Vt = Vt * keep[:, None]
    S = np.where(keep, S, 0.0)
    Y = np.where(keep, 1.0 / np.where(keep, S, 1.0), 0.0)
    return U, S, Vt, Y, int(np.sum(~keep))


def inverse_canonical(right_canonical_cores, thresh: float = INV_TRUNC):
    """Left-to-right SVD sweep of a right-canonical train into the inverse
    canonical form (Psi_1..Psi_L, Y_1..Y_{L-1}) of Sec. 2.3.1.

    SVD signs follow the same rule as the 2-site update (largest-magnitude
    entry of each U column positive).  Singular values at or below
    thresh * sigma_1 are truncated (truncate_inverse).  Returns
    (Psi, Y, n_trunc)."""
    cores = [np.array(c, dtype=np.float64, copy=True) for c in right_canonical_cores]
    L = len(cores)
    Psi, Y = [None] * L, [None] * (L - 1)
    n_guard = 0
    carry = None
    for l in range(L):
        core = cores[l] if carry is None else np.tensordot(carry, cores[l], axes=(1, 0))
        if l == L - 1:
            Psi[l] = core
            break
        cl, d1, d2, cr = core.shape
        X = core.reshape(cl * d1 * d2, cr)
        U, S, Vt = np.linalg.svd(X, full_matrices=False)
        r = min(X.shape)
        U, S, Vt = U[:, :r], S[:r], Vt[:r]
        s = sign_fix_columns(U)
        U, Vt = U * s[None, :], Vt * s[:, None]
        U, S, Vt, Yl, nt = truncate_inverse(U, S, Vt, thresh)
        n_guard += nt
        Psi[l] = (U * S[None, :]).reshape(cl, d1, d2, r)
        Y[l] = Yl
        carry = S[:, None] * Vt
    return Psi, Y, n_guard


def merge_inverse_canonical(Psi, Y):
    """C_l = Psi_l Y_l for l < L and C_L = Psi_L (Sec. 4.7, inverse form)."""
    L = len(Psi)
    C = []
    for l in range(L):
        if l < L - 1:
            C.append(Psi[l] * Y[l][None, None, None, :])
        else:
            C.append(np.array(Psi[l], copy=True))
    return C
