"""The allocation-free exact check (mpo_contract_exact_check_static) against
the workspace variant (mpo_contract_exact_check): the same fit errors on two
calls in a row, the second with a smaller input (the static scratch keeps the
first call's contents), and a clear error for an input beyond its size."""
import numpy as np
import pytest

from oracle import fit as ofit
from oracle import mpo
from synth import make_pair

pytestmark = pytest.mark.gpu


def test_static_check_matches_workspace_variant():
    from paper_2606_23274_amd.api import fit_error
    cases = [(8, 8, 16, 0), (5, 3, 4, 1)]  # the second input is smaller
    for L, chi, chi_c, seed in cases:
        A, B = make_pair(L, 2, chi, seed=seed, decay=True)
        for C in (ofit.fit_serial(A, B, chi_c, 1).C, mpo.naive_product(A, B)):
            e_ws, n_ws, m_ws = fit_error(A, B, C, with_method=True)
            e_st, n_st, m_st = fit_error(A, B, C, with_method=True, static=True)
            assert m_ws == m_st == 0
            assert abs(e_st - e_ws) <= 1e-10 * max(e_ws, 1e-3)
            assert abs(n_st - n_ws) <= 1e-12 * n_ws


def test_static_check_rejects_large_inputs():
    from paper_2606_23274_amd._lib import MpoError
    from paper_2606_23274_amd.api import fit_error
    A, B = make_pair(12, 2, 40, seed=2, decay=True)
    C = [np.ones((1 if l == 0 else 4, 2, 2, 1 if l == 11 else 4)) for l in range(12)]
    with pytest.raises(MpoError) as e:
        fit_error(A, B, C, static=True)
    assert "WORKSPACE" in str(e.value)
