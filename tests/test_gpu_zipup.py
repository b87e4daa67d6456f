"""Zip-up (Alg. 2) on the GPU (mpo_zipup) against the oracle's, and the fit
started from it (Alg. 5 with the zip-up initial guess)."""
import numpy as np
import pytest

from oracle import fit as ofit
from oracle import mpo, zipup
from synth import make_pair

pytestmark = pytest.mark.gpu


@pytest.mark.parametrize("L,chi,chi_max,p", [(6, 3, 64, -1), (8, 8, 12, -1), (8, 8, 12, 4), (10, 16, 24, 8),
                                             (7, 5, 9, 2)])
def test_zipup_matches_oracle(L, chi, chi_max, p):
    from paper_2606_23274_amd.api import zipup as gz
    A, B = make_pair(L, 2, chi, seed=L * chi, decay=True)
    C = gz(A, B, chi_max, sketch_p=p, seed=5)
    ref = zipup.zipup(A, B, chi_max, sketch_p=p, seed=5)
    assert [c.shape for c in C] == [r.shape for r in ref]
    assert mpo.rel_diff(C, ref) < 1e-10
    for c, r in zip(C, ref):  # the same gauge: the cores themselves agree
        assert np.linalg.norm(c - r) <= 1e-9 * np.linalg.norm(r)


def test_zipup_at_the_headline_size():
    """L=40 chi=64 chi_C=128 with the sketch p=16 (the randomized zip-up of
    Sec. 2.2 / 3.1)."""
    from paper_2606_23274_amd.api import zipup as gz
    A, B = make_pair(40, 2, 64, seed=0, decay=True)
    C = gz(A, B, 128, sketch_p=16, seed=0)
    ref = zipup.zipup(A, B, 128, sketch_p=16, seed=0)
    assert mpo.rel_diff(C, ref) < 1e-10


def test_fit_from_zipup_guess():
    """Alg. 5 from the zip-up guess: the device fit equals the oracle's fit
    from the oracle's zip-up; the zip-up itself approximates A B, and one
    sweep from it ends no worse than one sweep from the guess A."""
    from paper_2606_23274_amd.api import FitContext, fit_error
    from paper_2606_23274_amd.api import zipup as gz
    A, B = make_pair(10, 2, 8, seed=3, decay=True)
    C0 = gz(A, B, 16, sketch_p=4, seed=1)
    e_zip = fit_error(A, B, C0)[0]
    ctx = FitContext([(A, B)], 16, precision="fp64", sketch_p=4, seed=2, c_init=[C0])
    try:
        ctx.sweep(1)
        C = ctx.export_numpy(0)
    finally:
        ctx.close()
    ref = ofit.fit_serial(A, B, 16, 1, sketch_p=4, seed=2, C_init=zipup.zipup(A, B, 16, sketch_p=4, seed=1))
    assert mpo.rel_diff(C, ref.C) < 1e-10
    ctx = FitContext([(A, B)], 16, precision="fp64", sketch_p=4, seed=2)
    try:
        ctx.sweep(1)
        e1_A = fit_error(A, B, ctx.export_numpy(0))[0]
    finally:
        ctx.close()
    e1_zip = fit_error(A, B, C)[0]
    print("zip-up", e_zip, "one sweep from it", e1_zip, "one sweep from A", e1_A)
    assert e_zip < 0.8  # (chi_C = 16 against chi_A chi_B = 64: a coarse guess, but a guess of A B)
    assert e1_zip <= 1.01 * e1_A
