"""Pins of the randomized bond projection (oracle/bondproj.py, Sec. 3.2):
each checks it against something other than its own code path."""
import numpy as np
import pytest

from oracle import bondproj, mpo, philox
from oracle import fit as ofit
from synth import make_pair
from synth.mpo_inputs import gaussian_mpo


def _dense_with_projectors(cores, Ps):
    """A_1 P_1 A_2 ... P_{L-1} A_L as a dense (d^L x d^L) matrix, by explicit
    index sums over (left bond, out, in) carried site by site, with the
    projector matrices applied between cores."""
    T = cores[0][0]  # (d, d, chi)
    d = T.shape[0]
    T = T.reshape(d, d, -1)
    for l in range(1, len(cores)):
        T = np.einsum("xya,ab->xyb", T, Ps[l])
        T = np.einsum("xya,astb->xsytb", T, cores[l])
        n = T.shape[0] * T.shape[1]
        T = T.reshape(n, n, T.shape[-1])
    return T[:, :, 0]


def test_identity_when_k_covers_every_bond():
    A, _ = make_pair(6, 2, 8, seed=3, decay=True)
    At = bondproj.project_bonds(A, 64)
    for a, b in zip(A, At):
        assert a.shape == b.shape
        assert np.array_equal(a, b)


def test_dense_definition_and_projector_properties():
    """The projected cores reproduce the operator with P_l = Q_l Q_l^T
    inserted on every bond (dense index sums), and Q_l is an orthonormal
    basis of X^T Omega (X = core l-1 unfolded on its right bond, Omega the
    Philox matrix of bond l)."""
    rng = np.random.default_rng(5)
    A = gaussian_mpo(rng, 4, 2, 6, decay=True)
    k = 3
    Qs = bondproj.bond_projectors(A, k, seed=7, pair=2)
    At = bondproj.project_bonds(A, k, seed=7, pair=2)
    for l in range(1, 4):
        Q = Qs[l]
        chi = A[l - 1].shape[3]
        assert Q.shape == (chi, min(k, chi))
        assert np.allclose(Q.T @ Q, np.eye(Q.shape[1]), atol=1e-13)
        if k < chi:
            X = A[l - 1].reshape(-1, chi)
            Y = X.T @ philox.gaussian_matrix(X.shape[0], k, 7, 2, bondproj.A_STREAM, l)
            R = Q.T @ Y
            assert np.allclose(Q @ R, Y, atol=1e-12 * np.abs(Y).max())
            assert np.allclose(np.tril(R, -1), 0.0, atol=1e-12 * np.abs(Y).max())
            assert np.all(np.diag(R) >= 0)
    Ps = [None] + [Q @ Q.T for Q in Qs[1:4]]
    want = _dense_with_projectors(A, Ps)
    got = mpo.dense(At)
    assert np.allclose(got, want, atol=1e-13 * np.abs(want).max())
    assert [c.shape[3] for c in At[:-1]] == [min(k, A[l].shape[3]) for l in range(3)]


def test_rank_deficient_bonds_are_kept_exactly():
    """A core whose right unfolding has rank r <= k: X P = X, so the
    projected operator equals the original one."""
    rng = np.random.default_rng(11)
    A = gaussian_mpo(rng, 5, 2, 8, decay=False)
    r = 3
    for l in range(4):
        X = A[l].reshape(-1, A[l].shape[3])
        X = (X @ rng.standard_normal((X.shape[1], r))) @ rng.standard_normal((r, X.shape[1]))
        A[l] = X.reshape(A[l].shape)
    At = bondproj.project_bonds(A, 4, seed=1)
    Dt, D = mpo.dense(At), mpo.dense(A)
    assert np.linalg.norm(Dt - D) <= 1e-12 * np.linalg.norm(D)


def test_projection_error_within_the_range_finder_bound():
    """For each bond: |X - X Q Q^T|_F against the tail of X's singular values
    beyond the target rank (Halko-Martinsson-Tropp, Thm. 10.5 in
    expectation, factor (1 + t/(p-1))^{1/2} with t = k - p, p = 5); a
    projector built from the wrong side or a missing Q^T would miss by O(1)."""
    A, _ = make_pair(8, 2, 32, seed=2, decay=True)
    k, p = 12, 5
    Qs = bondproj.bond_projectors(A, k, seed=3)
    for l in range(1, 8):
        X = A[l - 1].reshape(-1, A[l - 1].shape[3])
        if k >= X.shape[1]:
            continue
        s = np.linalg.svd(X, compute_uv=False)
        tail = np.sqrt(np.sum(s[k - p:] ** 2))
        err = np.linalg.norm(X - X @ Qs[l] @ Qs[l].T)
        assert err <= 3.0 * np.sqrt(1 + (k - p) / (p - 1)) * tail + 1e-13 * s[0]
        assert err >= np.sqrt(np.sum(s[k:] ** 2)) * (1 - 1e-12)  # Eckart-Young


def test_streams_of_A_and_B_differ_and_the_fit_uses_the_projected_pair():
    A, B = make_pair(6, 2, 8, seed=4, decay=True)
    At, Bt = bondproj.project_pair(A, B, 4, seed=9)
    Qa = bondproj.bond_projectors(A, 4, seed=9, stream=bondproj.A_STREAM)
    Qb = bondproj.bond_projectors(A, 4, seed=9, stream=bondproj.B_STREAM)
    assert not np.allclose(Qa[3], Qb[3])
    # the fit of the projected pair approaches the projected product, not A B
    r = ofit.fit_serial(At, Bt, 64, 2)
    assert mpo.fit_error_dense(At, Bt, r.C) < 1e-10
    assert mpo.fit_error_dense(A, B, r.C) > 1e-6
