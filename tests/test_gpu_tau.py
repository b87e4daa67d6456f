"""Tolerance truncation of Sec. 2.3.4 on the GPU (opts.tau > 0) against the
oracle's fits with the same tolerance: the bond dims (integer decisions the
device takes from its FP64 eigenvalues) and the cores."""
import numpy as np
import pytest

from oracle import fit as ofit
from oracle import mpo
from synth import make_pair

pytestmark = pytest.mark.gpu


def _run(A, B, chi, schedule, sketch_p, tau, sweeps, precision="fp64", seed=5):
    from paper_2606_23274_amd.api import FitContext
    ctx = FitContext([(A, B)], chi, precision=precision, schedule=schedule, sketch_p=sketch_p,
                     seed=seed, tau=tau)
    try:
        ctx.sweep(sweeps)
        return ctx.bond_dims(), ctx.export_numpy(), [ctx.singular_values(b) for b in (1, len(A) // 2)]
    finally:
        ctx.close()


def _oracle(A, B, chi, schedule, sketch_p, tau, sweeps, seed=5):
    run = ofit.fit_serial if schedule == "serial" else ofit.fit_even_odd
    return run(A, B, chi, sweeps, sketch_p=sketch_p, seed=seed, tau=tau)


@pytest.mark.parametrize("schedule", ["serial", "even_odd"])
@pytest.mark.parametrize("sketch_p", [-1, 3])
@pytest.mark.parametrize("tau", [1.0, 2.0, 4.0])
def test_tau_fit_matches_oracle(schedule, sketch_p, tau):
    A, B = make_pair(8, 2, 6, seed=3, decay=True)
    dims, C, _ = _run(A, B, 12, schedule, sketch_p, tau, 2)
    ref = _oracle(A, B, 12, schedule, sketch_p, tau, 2)
    print(schedule, sketch_p, tau, dims, ref.bond_dims)
    assert dims == ref.bond_dims
    assert mpo.rel_diff(C, ref.C) < 1e-10


@pytest.mark.parametrize("schedule", ["serial", "even_odd"])
def test_tau_fit_several_tiles(schedule):
    """L = 12, chi = 16, chi_C = 40, p = 6: two-site matrices of several
    GEMM tiles with ragged edges, bonds cut by the rule to sizes between 1
    and the cap over three sweeps."""
    A, B = make_pair(12, 2, 16, seed=11, decay=True)
    dims, C, S = _run(A, B, 40, schedule, 6, 1.5, 3)
    ref = _oracle(A, B, 40, schedule, 6, 1.5, 3)
    print(schedule, dims, ref.bond_dims)
    assert dims == ref.bond_dims
    assert 1 < min(dims[2:-2]) and max(dims) < 40  # the rule decides, not the cap
    assert mpo.rel_diff(C, ref.C) < 1e-10
    assert all(len(s) == dims[b] for s, b in zip(S, (1, 6)))


def test_tau_fp32_dims_and_cores():
    A, B = make_pair(8, 2, 6, seed=3, decay=True)
    dims, C, _ = _run(A, B, 12, "serial", 3, 2.0, 2, precision="fp32")
    ref = _oracle(A, B, 12, "serial", 3, 2.0, 2)
    assert dims == ref.bond_dims
    assert mpo.rel_diff(C, ref.C) < 1e-5


def test_tau_zero_and_tiny_agree():
    """A tolerance below every tail keeps the fixed-cap fit's dims and cores."""
    A, B = make_pair(8, 2, 6, seed=3, decay=True)
    d0, C0, _ = _run(A, B, 12, "serial", 3, 0.0, 2)
    d1, C1, _ = _run(A, B, 12, "serial", 3, 1e-300, 2)
    assert d0 == d1
    assert mpo.rel_diff(C1, C0) < 1e-13


def test_tau_gradient_is_refused():
    from paper_2606_23274_amd import _lib
    from paper_2606_23274_amd.api import FitContext
    A, B = make_pair(6, 2, 4, seed=1, decay=True)
    ctx = FitContext([(A, B)], 8, precision="fp64", tau=1.0)
    try:
        ctx.sweep(1)
        with pytest.raises(_lib.MpoError) as e:
            ctx.grad(ctx.export_numpy())
        assert e.value.status == 6
    finally:
        ctx.close()
