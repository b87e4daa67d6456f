"""Parity of the HIP serial fit with the FP64 oracle (relative Frobenius
distance of the fitted operators, gauge independent).

Tolerances: 1e-10 for FP64, 1e-5 for FP32, 3e-3 for BF16.  The randomized
sweep is compared after its first forward pass for FP32/BF16: from the first
backward pass on, the sketch M Omega acts on columns expressed in C's right
gauge, which is a discontinuous function of rounding (sign rule, near-equal
singular values), so reduced-precision runs and the FP64 oracle draw
effectively different sketches.  Later sweeps are compared on the fit error
instead."""
import numpy as np
import pytest

from oracle import fit as ofit
from oracle import mpo
from synth import make_pair

pytestmark = pytest.mark.gpu


def gpu_fit(A, B, chi_c, sweeps, **kw):
    from paper_2606_23274_amd.api import FitContext
    ctx = FitContext([(A, B)], chi_c, **kw)
    try:
        ctx.sweep(sweeps)
        return ctx.export_numpy(0), ctx.bond_dims(0)
    finally:
        ctx.close()


def test_dense_L8_fp64_plain():
    """L=8, chi=8, chi_C=16, plain FP64, 4 sweeps, checked against the dense
    256 x 256 product."""
    A, B = make_pair(8, 2, 8, seed=0)
    C, dims = gpu_fit(A, B, 16, 4, precision="fp64", sketch_p=-1)
    ref = ofit.fit_serial(A, B, 16, 4)
    assert dims == ref.bond_dims
    assert mpo.rel_diff(C, ref.C) < 1e-10
    assert abs(mpo.fit_error_dense(A, B, C) - mpo.fit_error_dense(A, B, ref.C)) < 1e-10


@pytest.mark.parametrize("sweeps", [1, 2, 4])
def test_sketch_fp64(sweeps):
    A, B = make_pair(10, 2, 8, seed=3, decay=True)
    C, dims = gpu_fit(A, B, 16, sweeps, precision="fp64", sketch_p=4, seed=7)
    ref = ofit.fit_serial(A, B, 16, sweeps, sketch_p=4, seed=7)
    assert dims == ref.bond_dims
    assert mpo.rel_diff(C, ref.C) < 1e-10


def test_plain_fp32():
    A, B = make_pair(10, 2, 8, seed=4, decay=True)
    C, _ = gpu_fit(A, B, 16, 4, precision="fp32", sketch_p=-1)
    ref = ofit.fit_serial(A, B, 16, 4)
    assert mpo.rel_diff(C, ref.C) < 1e-5


def test_sketch_fp32_first_sweep():
    A, B = make_pair(12, 2, 8, seed=5, decay=True)
    C, _ = gpu_fit(A, B, 16, 1, precision="fp32", sketch_p=4, seed=1)
    ref = ofit.fit_serial(A, B, 16, 1, sketch_p=4, seed=1)
    assert mpo.rel_diff(C, ref.C) < 1e-5


def test_sketch_bf16x3_first_sweep():
    """Split BF16 (hi + lo operands, three BF16 products) meets 3e-3."""
    A, B = make_pair(12, 2, 8, seed=5, decay=True)
    C, _ = gpu_fit(A, B, 16, 1, precision="bf16x3", sketch_p=4, seed=1)
    ref = ofit.fit_serial(A, B, 16, 1, sketch_p=4, seed=1)
    assert mpo.rel_diff(C, ref.C) < 3e-3


@pytest.mark.xfail(reason="pure BF16 operands: each product carries ~2^-9 relative rounding and "
                          "the environments chain it over every site (measured 2.35e-2 here)",
                   strict=True)
def test_sketch_bf16_pure_first_sweep():
    """Pure BF16 against the BF16 bar of 3e-3 (the split-BF16 mode meets it)."""
    A, B = make_pair(12, 2, 8, seed=5, decay=True)
    C, _ = gpu_fit(A, B, 16, 1, precision="bf16", sketch_p=4, seed=1)
    ref = ofit.fit_serial(A, B, 16, 1, sketch_p=4, seed=1)
    assert mpo.rel_diff(C, ref.C) < 3e-3


def test_ragged_dims_fp64():
    """Bond dimensions that are not multiples of the tiles, d = 3."""
    rng = np.random.default_rng(11)
    from synth import gaussian_mpo
    A = gaussian_mpo(rng, 6, 3, 5, decay=True)
    B = gaussian_mpo(rng, 6, 3, 7, decay=True)
    C, dims = gpu_fit(A, B, 13, 3, precision="fp64", sketch_p=2, seed=3)
    ref = ofit.fit_serial(A, B, 13, 3, sketch_p=2, seed=3)
    assert dims == ref.bond_dims
    assert mpo.rel_diff(C, ref.C) < 1e-10


def _random_mpo(seed, L, d, dims):
    rng = np.random.default_rng(seed)
    return [rng.standard_normal((dims[l], d, d, dims[l + 1])) / np.sqrt(dims[l + 1]) for l in range(L)]


@pytest.mark.parametrize("precision,sketch_p,tol", [("fp64", -1, 1e-10), ("fp64", 4, 1e-10),
                                                    ("fp32", -1, 1e-5)])
def test_initial_guess(precision, sketch_p, tol):
    """Fit from a given initial guess (Alg. 5 input C), with unclipped bond
    dims (12 next to the boundary, where d^2 = 4), against the oracle from the
    same guess."""
    A, B = make_pair(10, 2, 8, seed=21, decay=True)
    C0 = _random_mpo(22, 10, 2, [1] + [12] * 9 + [1])
    sweeps = 2 if precision == "fp64" else 1
    C, dims = gpu_fit(A, B, 16, sweeps, precision=precision, sketch_p=sketch_p, seed=7, c_init=[C0])
    ref = ofit.fit_serial(A, B, 16, sweeps, sketch_p=sketch_p, seed=7, C_init=C0)
    assert dims == ref.bond_dims
    assert mpo.rel_diff(C, ref.C) < tol


@pytest.mark.parametrize("sketch_p", [-1, 10])
def test_cfg2_L20_six_sweeps(sketch_p):
    """The plain-and-sketched FP64 configuration: L=20, d=2, chi_A=chi_B=32
    with exp(-k/6) bond weights, chi_C=64, plain and p=10 (k=74), 6 sweeps.
    The first sweep is checked at 1e-10 directly; sweeps 2..6 by single
    updates at five positions each (both directions), resumed from the
    oracle's state just before them (first_sweep, first_bond, c_init); the
    fit error per sweep (fit_err, transfer passes) of the uninterrupted device
    fit matches the oracle's."""
    from paper_2606_23274_amd.api import FitContext
    A, B = make_pair(20, 2, 32, seed=0, decay=True)
    traj, cases, state, count = {}, [], {}, {}

    def on_update(sweep, l, Cs):
        if (sweep % 2 == 0 and l == 19) or (sweep % 2 == 1 and l == 1):
            traj[sweep + 1] = Cs
        if sweep > 0:
            pos = count.get(sweep, 0)
            count[sweep] = pos + 1
            if pos in (0, 5, 9, 13, 18):
                cases.append((sweep, pos, state["C"], l - 1, Cs))
        state["C"] = Cs

    ofit.fit_serial(A, B, 64, 6, sketch_p=sketch_p, seed=0, on_update=on_update)
    n2 = mpo.product_norm2(A, B)
    ctx = FitContext([(A, B)], 64, precision="fp64", sketch_p=sketch_p, seed=0, track_error=True)
    try:
        eps = ctx.sweep(6, errors=True)[0]
        C6 = ctx.export_numpy(0)
    finally:
        ctx.close()
    for s in range(6):
        ref = mpo.fit_error_transfer(A, B, traj[s + 1], n2)
        assert abs(eps[s] - ref) <= 1e-7, (s, eps[s], ref)
    C1, dims = gpu_fit(A, B, 64, 1, precision="fp64", sketch_p=sketch_p, seed=0)
    assert dims == mpo.bond_dims(traj[1])
    assert mpo.rel_diff(C1, traj[1]) < 1e-10
    errs = []
    for sweep, pos, before, i, after in cases:
        ctx = FitContext([(A, B)], 64, precision="fp64", sketch_p=sketch_p, seed=0, c_init=[before],
                         first_sweep=sweep, first_bond=pos)
        try:
            ctx.updates(1)
            C = ctx.export_numpy(0)
            assert ctx.bond_dims(0) == mpo.bond_dims(after)
        finally:
            ctx.close()
        errs.append(mpo.rel_diff(C, after))
    print("sketch_p", sketch_p, "single-update distances", ["%.1e" % e for e in errs],
          "uninterrupted after 6:", mpo.rel_diff(C6, traj[6]))
    assert len(errs) == 25 and max(errs) < 1e-10
