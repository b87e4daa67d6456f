"""Pins of the zip-up oracle (oracle/zipup.py, Alg. 2), each against
something other than its own code path."""
import numpy as np
import pytest

from oracle import mpo, zipup
from synth import make_pair
from synth.mpo_inputs import gaussian_mpo


def test_exact_regime_reproduces_the_product():
    """chi_max above every rank: no truncation, C = A B (dense)."""
    A, B = make_pair(5, 2, 3, seed=1)
    C = zipup.zipup(A, B, 64)
    D = mpo.dense(mpo.naive_product(A, B))
    assert np.linalg.norm(mpo.dense(C) - D) <= 1e-12 * np.linalg.norm(D)


@pytest.mark.parametrize("sketch_p", [-1, 4])
def test_isometries_and_eckart_young_lower_bound(sketch_p):
    """Every core but the last is left-orthogonal (U of an SVD); the error of
    the truncated product is at least the best rank-chi error of the dense
    product across any single bond (Eckart-Young)."""
    A, B = make_pair(6, 2, 4, seed=2, decay=True)
    chi = 6
    C = zipup.zipup(A, B, chi, sketch_p=sketch_p, seed=3)
    for c in C[:-1]:
        U = c.reshape(-1, c.shape[3])
        G = U.T @ U
        keep = np.diag(G) > 0.5  # dropped columns (drop rule) are zero
        assert np.allclose(G[np.ix_(keep, keep)], np.eye(int(keep.sum())), atol=1e-12)
        assert np.all(c.shape[3] <= chi)
    D = mpo.dense(mpo.naive_product(A, B))
    err = np.linalg.norm(mpo.dense(C) - D)
    L, d = 6, 2
    T = D.reshape([d] * L + [d] * L)
    for cut in range(1, L):
        rows = list(range(cut)) + [L + i for i in range(cut)]
        cols = [i for i in range(2 * L) if i not in rows]
        Mcut = np.transpose(T, rows + cols).reshape(d ** (2 * cut), -1)
        s = np.linalg.svd(Mcut, compute_uv=False)
        assert err >= np.sqrt(np.sum(s[chi:] ** 2)) * (1 - 1e-10)
    if sketch_p < 0:  # a sanity bound for the plain SVD (the zip-up has no global error control)
        assert err < 0.5 * np.linalg.norm(D)


def test_input_gauge_does_not_matter():
    """Alg. 2 works on the right-canonical form, which a change of gauge on
    a bond of A (X_l G, G^-1 X_{l+1}) does not alter."""
    A, B = make_pair(6, 2, 5, seed=4, decay=True)
    rng = np.random.default_rng(9)
    A2 = [a.copy() for a in A]
    G = rng.standard_normal((5, 5)) + 3 * np.eye(5)
    A2[2] = np.tensordot(A2[2], G, axes=(3, 0))
    A2[3] = np.tensordot(np.linalg.inv(G), A2[3], axes=(1, 0))
    C1 = zipup.zipup(A, B, 7)
    C2 = zipup.zipup(A2, B, 7)
    for a, b in zip(C1, C2):
        assert np.allclose(a, b, atol=1e-11 * np.abs(b).max())


def test_sketch_spanning_the_range_equals_plain_svd():
    """With k = chi_max + p at least every M_l's rank the range finder's Q
    spans M_l's range, so the randomized zip-up is the plain one."""
    rng = np.random.default_rng(6)
    A = gaussian_mpo(rng, 5, 2, 3)
    B = gaussian_mpo(rng, 5, 2, 3)
    Cp = zipup.zipup(A, B, 64)
    Cr = zipup.zipup(A, B, 40, sketch_p=30, seed=2)
    assert mpo.rel_diff(Cr, Cp) < 1e-11
