"""mpo_contract_exact_check: the fit error ||A B - C||_F / ||A B||_F from
transfer passes on the GPU, against dense and oracle values."""
import numpy as np
import pytest

from oracle import fit as ofit
from oracle import mpo
from synth import gaussian_mpo, make_pair

pytestmark = pytest.mark.gpu


def test_against_dense_L8():
    from paper_2606_23274_amd.api import fit_error
    A, B = make_pair(8, 2, 8, seed=0)
    C = ofit.fit_serial(A, B, 16, 2).C
    err, n2 = fit_error(A, B, C)
    D = mpo.dense(A) @ mpo.dense(B)
    assert abs(n2 - np.linalg.norm(D) ** 2) <= 1e-12 * np.linalg.norm(D) ** 2
    ref = mpo.fit_error_dense(A, B, C)
    assert abs(err - ref) <= 1e-9 * max(ref, 1e-3)


def test_exact_regime_and_zero():
    from paper_2606_23274_amd.api import fit_error
    A, B = make_pair(6, 2, 3, seed=4)
    C = mpo.naive_product(A, B)
    err, _ = fit_error(A, B, C)
    assert err < 1e-6  # the difference of squares floors near sqrt(eps)
    Z = [np.zeros_like(c) for c in C]
    err0, _ = fit_error(A, B, Z)
    assert abs(err0 - 1.0) < 1e-12


@pytest.mark.parametrize("L,chi,chi_c", [(20, 16, 32), (64, 8, 16)])
def test_against_oracle_transfer(L, chi, chi_c):
    """Longer chains (norms down to about 1e-100 at L=64): the per-site
    normalization keeps every pass in range."""
    from paper_2606_23274_amd.api import fit_error
    A, B = make_pair(L, 2, chi, seed=L, decay=True)
    C = ofit.fit_serial(A, B, chi_c, 1, sketch_p=4, seed=1).C
    err, n2 = fit_error(A, B, C)
    n2_ref = mpo.product_norm2(A, B)
    assert abs(n2 - n2_ref) <= 1e-10 * n2_ref
    ref = mpo.fit_error_transfer(A, B, C, n2_ref)
    assert abs(err - ref) <= 1e-7


def test_ragged_physical_dim():
    from paper_2606_23274_amd.api import fit_error
    rng = np.random.default_rng(3)
    A = gaussian_mpo(rng, 5, 3, 4)
    B = gaussian_mpo(rng, 5, 3, 5)
    C = ofit.fit_serial(A, B, 7, 2).C
    err, _ = fit_error(A, B, C)
    ref = mpo.fit_error_dense(A, B, C)
    assert abs(err - ref) <= 1e-9 * max(ref, 1e-3)
