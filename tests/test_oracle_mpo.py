"""Pins of the oracle's MPO utilities against brute-force dense algebra."""
import itertools

import numpy as np
import pytest

from oracle import mpo
from synth import gaussian_mpo, make_pair


def _rand(L, d, chi, seed):
    return gaussian_mpo(np.random.default_rng(seed), L, d, chi)


def test_dense_matches_index_sum():
    X = _rand(3, 2, 3, 0)
    D = mpo.dense(X)
    for x in itertools.product(range(2), repeat=3):
        for y in itertools.product(range(2), repeat=3):
            v = (X[0][0, x[0], y[0], :] @ X[1][:, x[1], y[1], :] @ X[2][:, x[2], y[2], 0])
            row = x[0] * 4 + x[1] * 2 + x[2]
            col = y[0] * 4 + y[1] * 2 + y[2]
            assert abs(D[row, col] - v) < 1e-14


def test_naive_product_is_matrix_product():
    A, B = make_pair(4, 2, 3, seed=1)
    C = mpo.naive_product(A, B)
    assert [c.shape[3] for c in C[:-1]] == [9, 9, 9]
    P = mpo.dense(A) @ mpo.dense(B)
    assert np.allclose(mpo.dense(C), P, atol=1e-13, rtol=0)


def test_naive_product_d3():
    rng = np.random.default_rng(2)
    A = gaussian_mpo(rng, 3, 3, 2)
    B = gaussian_mpo(rng, 3, 3, 3)
    assert np.allclose(mpo.dense(mpo.naive_product(A, B)), mpo.dense(A) @ mpo.dense(B),
                       atol=1e-13)


def test_inner_products_and_norms():
    A, B = make_pair(5, 2, 3, seed=4)
    C = _rand(5, 2, 4, 5)
    dA, dB, dC = mpo.dense(A), mpo.dense(B), mpo.dense(C)
    assert np.isclose(mpo.transfer_inner(A, C), np.sum(dA * dC), rtol=1e-12)
    assert np.isclose(mpo.three_layer_inner(C, A, B), np.sum(dC * (dA @ dB)), rtol=1e-12)
    assert np.isclose(mpo.product_norm2(A, B), np.sum((dA @ dB) ** 2), rtol=1e-12)
    assert np.isclose(mpo.left_orth_norm(C), np.linalg.norm(dC), rtol=1e-13)


@pytest.mark.parametrize("scale", [1.0, 1e-6, 1e-11])
def test_diff_norm_below_sqrt_eps(scale):
    X = _rand(6, 2, 4, 6)
    E = _rand(6, 2, 3, 7)
    # Y = X + scale * E as an MPO: direct sum of X and scale*E
    Ys = [e.copy() for e in E]
    Ys[0] = Ys[0] * scale
    Y = []
    for l in range(6):
        x, e = X[l], Ys[l]
        if l == 0:
            Y.append(np.concatenate([x, e], axis=3))
        elif l == 5:
            Y.append(np.concatenate([x, e], axis=0))
        else:
            z = np.zeros((x.shape[0] + e.shape[0], 2, 2, x.shape[3] + e.shape[3]))
            z[:x.shape[0], :, :, :x.shape[3]] = x
            z[x.shape[0]:, :, :, x.shape[3]:] = e
            Y.append(z)
    exact = scale * np.linalg.norm(mpo.dense(E))
    got = mpo.diff_norm(Y, X)
    assert abs(got - exact) <= 1e-9 * exact + 1e-14 * np.linalg.norm(mpo.dense(X))


def test_fit_error_transfer_matches_dense():
    A, B = make_pair(6, 2, 3, seed=8)
    C = _rand(6, 2, 5, 9)
    assert abs(mpo.fit_error_transfer(A, B, C) - mpo.fit_error_dense(A, B, C)) < 1e-7
