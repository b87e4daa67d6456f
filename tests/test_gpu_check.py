"""mpo_contract_exact_check: the fit error ||A B - C||_F / ||A B||_F on the
GPU, by Householder-QR sweeps of the naive product and the difference MPO
(route 0, small bonds) or by transfer passes (route 1), against dense and
oracle values."""
import numpy as np
import pytest

from oracle import fit as ofit
from oracle import mpo
from synth import gaussian_mpo, make_pair

pytestmark = pytest.mark.gpu


def test_against_dense_L8():
    """Route 0 (chi_A chi_B + chi_C = 80) against the dense 256 x 256 product."""
    from paper_2606_23274_amd.api import fit_error
    A, B = make_pair(8, 2, 8, seed=0)
    C = ofit.fit_serial(A, B, 16, 2).C
    err, n2, meth = fit_error(A, B, C, with_method=True)
    assert meth == 0
    D = mpo.dense(A) @ mpo.dense(B)
    assert abs(n2 - np.linalg.norm(D) ** 2) <= 1e-12 * np.linalg.norm(D) ** 2
    ref = mpo.fit_error_dense(A, B, C)
    assert abs(err - ref) <= 1e-12 * max(ref, 1e-3)


@pytest.mark.parametrize("scale", [1e-4, 1e-8, 1e-11])
def test_exact_regime_below_sqrt_eps(scale):
    """C = the naive product perturbed by a known relative amount: route 0
    resolves it far below sqrt(eps) (the dense difference is the reference;
    the oracle's difference-MPO norm agrees with it)."""
    from paper_2606_23274_amd.api import fit_error
    A, B = make_pair(6, 2, 3, seed=4)
    P = mpo.naive_product(A, B)
    rng = np.random.default_rng(7)
    C = [c.copy() for c in P]
    C[3] = C[3] + scale * np.linalg.norm(C[3]) * rng.standard_normal(C[3].shape) / np.sqrt(C[3].size)
    err, _, meth = fit_error(A, B, C, with_method=True)
    assert meth == 0
    D = mpo.dense(A) @ mpo.dense(B)
    ref = np.linalg.norm(D - mpo.dense(C)) / np.linalg.norm(D)
    assert abs(err - ref) <= 1e-3 * ref + 1e-14
    err_exact, _ = fit_error(A, B, P)
    assert err_exact < 1e-13


def test_exact_regime_and_zero():
    from paper_2606_23274_amd.api import fit_error
    A, B = make_pair(6, 2, 3, seed=4)
    C = mpo.naive_product(A, B)
    err, _ = fit_error(A, B, C)
    assert err < 1e-12
    Z = [np.zeros_like(c) for c in C]
    err0, _ = fit_error(A, B, Z)
    assert abs(err0 - 1.0) < 1e-12
    C1 = [c.copy() for c in C]  # one site: D = P - C at the single core
    err1, _ = fit_error([A[0][:, :, :, :1]], [B[0][:, :, :, :1]], [C1[0][:, :, :, :1]])
    assert err1 < 1e-14


def test_route_1_for_large_bonds():
    """Bonds above 512 take the transfer passes (difference of squares)."""
    from paper_2606_23274_amd.api import fit_error
    A, B = make_pair(10, 2, 24, seed=8, decay=True)
    C = ofit.fit_serial(A, B, 32, 1, sketch_p=4, seed=1).C
    err, n2, meth = fit_error(A, B, C, with_method=True)
    assert meth == 1
    ref = mpo.fit_error_transfer(A, B, C)
    assert abs(err - ref) <= 1e-7


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
    err, _, meth = fit_error(A, B, C, with_method=True)
    assert meth == 0
    ref = mpo.fit_error_dense(A, B, C)
    assert abs(err - ref) <= 1e-12 * max(ref, 1e-3)


def test_qr_route_matches_oracle_diff_norm():
    """Route 0 against the oracle's own difference-MPO norm (Householder QR
    on the host) on a longer chain with ragged bonds."""
    from paper_2606_23274_amd.api import fit_error
    A, B = make_pair(16, 2, 6, seed=16, decay=True)
    C = ofit.fit_serial(A, B, 11, 1, sketch_p=2, seed=3).C
    err, n2, meth = fit_error(A, B, C, with_method=True)
    assert meth == 0
    P = mpo.naive_product(A, B)
    nrm = mpo.left_orth_norm(P)
    ref = mpo.diff_norm(P, C) / nrm
    assert abs(n2 - nrm ** 2) <= 1e-12 * nrm ** 2
    assert abs(err - ref) <= 1e-12 * ref
