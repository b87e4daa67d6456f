"""Pins of the oracle's fits on inputs with prescribed bond spectra
(synth.string_sum_mpo times a product of reflectors): an exactly degenerate
spectrum cut between its clusters, and a steep one that crosses the drop
rule of the truncated SVD (Sec. 3.1, values below 1e-6 sigma_1 dropped).
The product's truncations are known in closed form: every bond's spectrum
is the weights', with the same strings at every cut, so the best
approximation keeps the largest strings and the fit must reproduce it."""
import numpy as np
import pytest

from oracle import fit, mpo
from synth import reflector_product_mpo, string_sum_mpo

DEGENERATE = [1.0, 0.6, 0.6, 0.6, 0.3, 0.3, 0.1, 0.05, 0.01]
STEEP = [10 ** (-1.1 * k) for k in range(9)]


def _problem(weights, L=6, d=3, seed=0):
    A = string_sum_mpo(L, d, weights)
    B = reflector_product_mpo(np.random.default_rng(seed), L, d)
    return A, B


def _kept_product(weights, keep, L=6, d=3, seed=0):
    """Dense product with only the strings in `keep`."""
    A = string_sum_mpo(L, d, [w if k in keep else 0.0 for k, w in enumerate(weights)])
    B = reflector_product_mpo(np.random.default_rng(seed), L, d)
    return mpo.dense(mpo.naive_product(A, B))


def test_generator_spectra():
    """Every cut of A B has the weights as its singular values (the strings
    are orthonormal on both sides, the reflectors orthogonal)."""
    L, d = 6, 3
    A, B = _problem(DEGENERATE)
    T = mpo.dense(mpo.naive_product(A, B)).reshape([d] * (2 * L))
    for cut in range(1, L):
        rows = list(range(cut)) + [L + i for i in range(cut)]
        cols = [i for i in range(2 * L) if i not in rows]
        s = np.linalg.svd(np.transpose(T, rows + cols).reshape(d ** (2 * cut), -1), compute_uv=False)
        assert np.allclose(s[:9], sorted(DEGENERATE, reverse=True), atol=1e-14)
        assert np.all(s[9:] < 1e-14)


@pytest.mark.parametrize("schedule", ["serial", "even_odd"])
@pytest.mark.parametrize("sketch_p", [-1, 2])
def test_degenerate_cut_between_clusters(schedule, sketch_p):
    """chi_C = 6 keeps the clusters {1}, {0.6 x 3}, {0.3 x 2}: the fit is
    that sum of strings (unique although each cluster's basis is not)."""
    A, B = _problem(DEGENERATE)
    run = fit.fit_serial if schedule == "serial" else fit.fit_even_odd
    r = run(A, B, 6, 2, sketch_p=sketch_p, seed=1)
    want = _kept_product(DEGENERATE, range(6))
    assert np.linalg.norm(mpo.dense(r.C) - want) <= 1e-13 * np.linalg.norm(want)
    assert r.bond_dims == [1, 6, 6, 6, 6, 6, 1]


@pytest.mark.parametrize("schedule", ["serial", "even_odd"])
@pytest.mark.parametrize("sketch_p", [-1, 2])
def test_steep_spectrum_follows_the_drop_rule(schedule, sketch_p):
    """chi_C = 9 would keep every string; the drop rule removes those below
    1e-6 of the largest (10^-6.6 and smaller), the smallest kept being
    10^-5.5."""
    A, B = _problem(STEEP)
    run = fit.fit_serial if schedule == "serial" else fit.fit_even_odd
    r = run(A, B, 9, 2, sketch_p=sketch_p, seed=1)
    want = _kept_product(STEEP, [k for k, w in enumerate(STEEP) if w > 1e-6 * STEEP[0]])
    assert len([w for w in STEEP if w > 1e-6]) == 6
    assert np.linalg.norm(mpo.dense(r.C) - want) <= 1e-13 * np.linalg.norm(want)
