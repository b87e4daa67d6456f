"""Device fits on inputs with prescribed bond spectra (see
test_oracle_spectra.py): an exactly degenerate spectrum cut between its
clusters, where the singular vectors inside a cluster are not unique (so the
dense operator, which is, is compared), and a steep spectrum across the drop
rule, where the smallest kept value is 3e-6 of the largest and the Gram
eigenproblem resolves it to about 1e-5 relative."""
import numpy as np
import pytest

from oracle import fit, mpo
from synth import reflector_product_mpo, string_sum_mpo

pytestmark = pytest.mark.gpu

DEGENERATE = [1.0, 0.6, 0.6, 0.6, 0.3, 0.3, 0.1, 0.05, 0.01]
STEEP = [10 ** (-1.1 * k) for k in range(9)]


def _problem(weights, L=6, d=3, seed=0):
    return string_sum_mpo(L, d, weights), reflector_product_mpo(np.random.default_rng(seed), L, d)


def _gpu(A, B, chi, sweeps, **kw):
    from paper_2606_23274_amd.api import FitContext
    ctx = FitContext([(A, B)], chi, **kw)
    try:
        ctx.sweep(sweeps)
        return ctx.export_numpy(0), ctx.bond_dims(0)
    finally:
        ctx.close()


_ORACLE = {"serial": fit.fit_serial, "even_odd": fit.fit_even_odd}


@pytest.mark.parametrize("schedule", ["serial", "even_odd"])
@pytest.mark.parametrize("sketch_p", [-1, 2])
@pytest.mark.parametrize("weights, chi", [(DEGENERATE, 6), (STEEP, 9)], ids=["degenerate", "steep"])
def test_prescribed_spectrum_fp64(schedule, sketch_p, weights, chi):
    A, B = _problem(weights)
    C, dims = _gpu(A, B, chi, 2, precision="fp64", schedule=schedule, sketch_p=sketch_p, seed=1)
    ref = _ORACLE[schedule](A, B, chi, 2, sketch_p=sketch_p, seed=1)
    assert dims == ref.bond_dims
    D, R = mpo.dense(C), mpo.dense(ref.C)
    d = np.linalg.norm(D - R) / np.linalg.norm(R)
    print(schedule, sketch_p, chi, d)
    assert d < 1e-10


@pytest.mark.parametrize("schedule", ["serial", "even_odd"])
def test_degenerate_fp32(schedule):
    A, B = _problem(DEGENERATE)
    C, dims = _gpu(A, B, 6, 2, precision="fp32", schedule=schedule, sketch_p=2, seed=1)
    ref = _ORACLE[schedule](A, B, 6, 2, sketch_p=2, seed=1)
    assert dims == ref.bond_dims
    D, R = mpo.dense(C), mpo.dense(ref.C)
    assert np.linalg.norm(D - R) / np.linalg.norm(R) < 1e-5
