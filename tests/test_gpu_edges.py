"""Degenerate shapes of the fit on the GPU against the oracle: the shortest
trains (L = 2, where the fit is one truncated SVD of the product, and
L = 3), scalar physical legs (d = 1: a chain of matrices), rank-one fits
(chi_C = 1), and the shortest MPO-MPS product."""
import numpy as np
import pytest

from oracle import fit as ofit
from oracle import mpo
from synth.mpo_inputs import gaussian_mpo

pytestmark = pytest.mark.gpu

_ORACLE = {"serial": ofit.fit_serial, "even_odd": ofit.fit_even_odd}


def _gpu(A, B, chi, sweeps, **kw):
    from paper_2606_23274_amd.api import FitContext
    ctx = FitContext([(A, B)], chi, precision="fp64", **kw)
    try:
        ctx.sweep(sweeps)
        return ctx.export_numpy(0), ctx.bond_dims(0)
    finally:
        ctx.close()


@pytest.mark.parametrize("schedule", ["serial", "even_odd"])
@pytest.mark.parametrize("sketch_p", [-1, 1])
@pytest.mark.parametrize("L, d, chi, chi_c, mps", [
    (2, 2, 3, 3, False),    # one bond: the truncated SVD of A B
    (3, 2, 4, 5, False),
    (6, 1, 4, 3, False),    # d = 1: matrices on the bonds only
    (7, 2, 4, 1, False),    # rank-one fit
    (2, 3, 4, 2, True),     # the shortest MPO-MPS product
])
def test_degenerate_shapes(schedule, sketch_p, L, d, chi, chi_c, mps):
    rng = np.random.default_rng(L * 100 + d * 10 + chi_c)
    A = gaussian_mpo(rng, L, d, chi, decay=True)
    B = gaussian_mpo(rng, L, d, chi, decay=True)
    if mps:
        B = [b[:, :, :1, :].copy() for b in B]
    C, dims = _gpu(A, B, chi_c, 2, schedule=schedule, sketch_p=sketch_p, seed=3)
    ref = _ORACLE[schedule](A, B, chi_c, 2, sketch_p=sketch_p, seed=3)
    assert dims == ref.bond_dims
    d_rel = mpo.rel_diff(C, ref.C)
    print(schedule, sketch_p, L, d, chi_c, mps, d_rel)
    assert d_rel < 1e-10
