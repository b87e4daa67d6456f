"""Pins of the oracle's gauge routines (Sec. 2.3.1) against dense algebra and
the defining orthogonality relations."""
import numpy as np
import pytest

from oracle import canon, mpo
from synth import gaussian_mpo, make_pair


def _left_orth_err(core):
    cl, d1, d2, cr = core.shape
    X = core.reshape(cl * d1 * d2, cr)
    return np.abs(X.T @ X - np.eye(cr)).max()


def _right_orth_err(core):
    cl = core.shape[0]
    X = core.reshape(cl, -1)
    return np.abs(X @ X.T - np.eye(cl)).max()


def test_qr_pos_is_unique_cholesky_factor():
    X = np.random.default_rng(0).standard_normal((40, 12))
    Q, R = canon.qr_pos(X)
    # the R of a QR with positive diagonal is the transposed Cholesky factor of X^T X
    Lc = np.linalg.cholesky(X.T @ X)
    assert np.allclose(R, Lc.T, rtol=0, atol=1e-12 * np.abs(R).max())
    assert np.allclose(Q @ R, X, atol=1e-13)


def test_left_orthogonalize_preserves_operator_and_clips():
    A, _ = make_pair(6, 2, 8, seed=0)
    Ao, nu = canon.left_orthogonalize(A)
    assert [c.shape[3] for c in Ao[:-1]] == [4, 8, 8, 8, 8]  # 1*2*2 = 4 clips bond 1
    assert np.allclose(nu * mpo.dense(Ao), mpo.dense(A), atol=1e-12 * np.abs(mpo.dense(A)).max())
    for core in Ao[:-1]:
        assert _left_orth_err(core) < 1e-13
    assert abs(np.linalg.norm(Ao[-1]) - 1.0) < 1e-14
    assert abs(nu - np.linalg.norm(mpo.dense(A))) < 1e-12 * nu


def test_right_orthogonalize_preserves_operator_and_clips():
    A, _ = make_pair(6, 2, 8, seed=1)
    Ar = canon.right_orthogonalize(A)
    assert [c.shape[3] for c in Ar[:-1]] == [8, 8, 8, 8, 4]
    assert np.allclose(mpo.dense(Ar), mpo.dense(A), atol=1e-12 * np.abs(mpo.dense(A)).max())
    for core in Ar[1:]:
        assert _right_orth_err(core) < 1e-13


@pytest.mark.parametrize("L,chi", [(6, 3), (7, 8)])
def test_inverse_canonical_relations(L, chi):
    A, _ = make_pair(L, 2, chi, seed=2, decay=True)
    Ao, _ = canon.left_orthogonalize(A)
    Cr = canon.right_orthogonalize(Ao)
    Psi, Y, n_guard = canon.inverse_canonical(Cr)
    assert n_guard == 0
    C = canon.merge_inverse_canonical(Psi, Y)
    assert np.allclose(mpo.dense(C), mpo.dense(Cr), atol=1e-12)
    for l in range(L - 1):
        # Psi_l Y_l is left orthogonal
        assert _left_orth_err(Psi[l] * Y[l][None, None, None, :]) < 1e-12
        # Y_l Psi_{l+1} is right orthogonal
        assert _right_orth_err(Y[l][:, None, None, None] * Psi[l + 1]) < 1e-12
        # Lambda_l are the Schmidt values of the normalized operator across bond l
        D = mpo.dense(Cr)
        dl = 2 ** (l + 1)
        M = D.reshape(dl, 2 ** L // dl, dl, 2 ** L // dl).transpose(0, 2, 1, 3).reshape(dl * dl, -1)
        sv = np.linalg.svd(M, compute_uv=False)[:len(Y[l])]
        assert np.allclose(1.0 / Y[l], sv, rtol=1e-10)


def test_sign_rule():
    U = np.array([[0.1, -0.9], [-0.8, 0.2], [0.3, 0.9]])
    s = canon.sign_fix_columns(U)
    assert list(s) == [-1.0, -1.0]  # first index wins the tie in column 2


def test_inverse_canonical_truncates_tiny_schmidt_values():
    """A train whose middle bond carries one Schmidt value of relative size
    1e-15: it is truncated before inversion (zero S, Y and singular vectors),
    the merged train reproduces the operator to that size, and Psi Y stays a
    partial isometry (identity on the kept directions, zero on the dropped)."""
    rng = np.random.default_rng(7)
    L, d, chi = 4, 2, 3
    # left-orthonormal cores with a prescribed spectrum at bond 2 (0-based 1)
    lam = np.array([1.0, 0.5, 1e-15])
    cores = []
    dims = [1, 4, 3, 4, 1]
    for l in range(L):
        a, b = dims[l], dims[l + 1]
        X = rng.standard_normal((a * d * d, b))
        Q, _ = np.linalg.qr(X) if a * d * d >= b else (np.eye(a * d * d, b), None)
        cores.append(Q[:, :b].reshape(a, d, d, b))
    cores[1] = cores[1] * lam[None, None, None, :]
    # right-canonicalize, which keeps the Schmidt spectrum of the operator
    Cr = canon.right_orthogonalize(cores)
    D0 = mpo.dense(Cr)
    Psi, Y, n_trunc = canon.inverse_canonical(Cr)
    assert n_trunc == 1
    assert np.count_nonzero(Y[1]) == 2 and Y[1][2] == 0.0
    C = canon.merge_inverse_canonical(Psi, Y)
    assert np.linalg.norm(mpo.dense(C) - D0) <= 1e-14 * np.linalg.norm(D0)
    W = (Psi[1] * Y[1][None, None, None, :]).reshape(-1, 3)
    assert np.allclose(W.T @ W, np.diag([1.0, 1.0, 0.0]), atol=1e-12)


def test_truncate_inverse_rule():
    U = np.eye(3)
    S = np.array([2.0, 1e-11, 1e-13])
    Vt = np.eye(3)
    U2, S2, Vt2, Y, n = canon.truncate_inverse(U, S, Vt, 1e-12)
    assert n == 1 and list(S2) == [2.0, 1e-11, 0.0]
    assert np.allclose(Y, [0.5, 1e11, 0.0])
    assert not U2[:, 2].any() and not Vt2[2].any()
