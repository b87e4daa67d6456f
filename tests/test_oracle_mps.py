"""Pins of the oracle's MPO-MPS fit (Sec. 1: the MPS as an MPO whose input
leg has dimension 1; the initial guess is then B, fit.default_guess) against
dense matrix-vector algebra."""
import numpy as np
import pytest

from oracle import fit, mpo
from synth.mpo_inputs import gaussian_mpo


def _mps(rng, L, d, chi, decay=True):
    return [b[:, :, :1, :].copy() for b in gaussian_mpo(rng, L, d, chi, decay=decay)]


def _dense_av(A, B):
    """A (d^L x d^L) applied to the vector of the MPS B (d^L)."""
    return mpo.dense(A) @ mpo.dense(B)[:, 0]


@pytest.mark.parametrize("schedule", ["serial", "even_odd"])
@pytest.mark.parametrize("sketch_p", [-1, 3])
def test_exact_regime_is_the_matrix_vector_product(schedule, sketch_p):
    rng = np.random.default_rng(3)
    A, B = gaussian_mpo(rng, 7, 2, 3), _mps(rng, 7, 2, 3)
    run = fit.fit_serial if schedule == "serial" else fit.fit_even_odd
    r = run(A, B, 64, 2, sketch_p=sketch_p, seed=1)
    assert all(c.shape[2] == 1 for c in r.C)
    y = _dense_av(A, B)
    assert np.linalg.norm(mpo.dense(r.C)[:, 0] - y) <= 1e-12 * np.linalg.norm(y)


def test_L2_is_the_truncated_svd_of_the_vector():
    """Two sites: C is the rank-r SVD of A v reshaped (d x d) (Eckart-Young)."""
    rng = np.random.default_rng(4)
    d = 3
    A, B = gaussian_mpo(rng, 2, d, 3), _mps(rng, 2, d, 3)
    y = _dense_av(A, B)
    sv = np.linalg.svd(y.reshape(d, d), compute_uv=False)
    for r in (1, 2):
        res = fit.fit_serial(A, B, r, 1)
        err = np.linalg.norm(mpo.dense(res.C)[:, 0] - y)
        assert abs(err - np.sqrt(np.sum(sv[r:] ** 2))) <= 1e-12 * np.linalg.norm(y)


def test_error_bounded_below_at_every_cut():
    rng = np.random.default_rng(5)
    L, d, chi = 8, 2, 4
    A, B = gaussian_mpo(rng, L, d, 4, decay=True), _mps(rng, L, d, 4)
    y = _dense_av(A, B)
    r = fit.fit_serial(A, B, chi, 3, sketch_p=2, seed=2)
    err = np.linalg.norm(mpo.dense(r.C)[:, 0] - y)
    for cut in range(1, L):
        s = np.linalg.svd(y.reshape(d ** cut, -1), compute_uv=False)
        assert err >= np.sqrt(np.sum(s[chi:] ** 2)) * (1 - 1e-10)
    assert err < 0.5 * np.linalg.norm(y)


def test_default_guess():
    rng = np.random.default_rng(6)
    A, B = gaussian_mpo(rng, 4, 2, 3), gaussian_mpo(rng, 4, 2, 3)
    assert fit.default_guess(A, B) is A
    Bm = _mps(rng, 4, 2, 3)
    assert fit.default_guess(A, Bm) is Bm
    with pytest.raises(ValueError):
        fit.default_guess(A, [b[:, :1] for b in Bm])  # neither input has C's legs
