"""Parity of the batched even/odd inverse-gauge schedule (Alg. 4, Sec. 4)
with the oracle's even/odd fit, and of the multi-pair grouped launch."""
import numpy as np
import pytest

from oracle import fit as ofit
from oracle import mpo
from synth import make_pair

pytestmark = pytest.mark.gpu


def gpu_fit_pairs(pairs, chi_c, sweeps, **kw):
    from paper_2606_23274_amd.api import FitContext
    ctx = FitContext(pairs, chi_c, schedule="even_odd", **kw)
    try:
        ctx.sweep(sweeps)
        return [ctx.export_numpy(i) for i in range(len(pairs))], [ctx.bond_dims(i) for i in range(len(pairs))]
    finally:
        ctx.close()


@pytest.mark.parametrize("sweeps", [1, 3])
@pytest.mark.parametrize("sketch_p", [-1, 4])
def test_even_odd_fp64(sweeps, sketch_p):
    A, B = make_pair(10, 2, 6, seed=2, decay=True)
    (C,), (dims,) = gpu_fit_pairs([(A, B)], 12, sweeps, precision="fp64", sketch_p=sketch_p, seed=5)
    ref = ofit.fit_even_odd(A, B, 12, sweeps, sketch_p=sketch_p, seed=5)
    assert dims == ref.bond_dims
    assert mpo.rel_diff(C, ref.C) < 1e-10


def test_even_odd_fp32_first_sweep():
    A, B = make_pair(12, 2, 8, seed=3, decay=True)
    (C,), _ = gpu_fit_pairs([(A, B)], 16, 1, precision="fp32", sketch_p=4, seed=2)
    ref = ofit.fit_even_odd(A, B, 16, 1, sketch_p=4, seed=2)
    assert mpo.rel_diff(C, ref.C) < 1e-5


def test_even_odd_exact_regime():
    A, B = make_pair(6, 2, 3, seed=1)
    (C,), _ = gpu_fit_pairs([(A, B)], 9, 3, precision="fp64")
    assert mpo.fit_error_dense(A, B, C) < 1e-11


def test_multi_pair_ragged():
    """Several independent pairs with different bond dimensions in one
    grouped launch per stage; each pair matches its own oracle fit."""
    pairs, chis = [], [3, 6, 4]
    for i, chi in enumerate(chis):
        pairs.append(make_pair(8, 2, chi, seed=100 + i, decay=True))
    caps = [2 * c for c in chis]
    Cs, dims = gpu_fit_pairs(pairs, 10, 2, precision="fp64", sketch_p=2, seed=9, pair_chi_max=caps)
    for i, (A, B) in enumerate(pairs):
        ref = ofit.fit_even_odd(A, B, caps[i], 2, sketch_p=2, seed=9, pair=i)
        assert dims[i] == ref.bond_dims
        assert mpo.rel_diff(Cs[i], ref.C) < 1e-10


def test_even_odd_initial_guess_fp64():
    """The even/odd fit from a given initial guess against the oracle."""
    A, B = make_pair(10, 2, 8, seed=31, decay=True)
    rng = np.random.default_rng(32)
    dims = [1, 4, 12, 12, 12, 12, 12, 12, 12, 4, 1]
    C0 = [rng.standard_normal((dims[l], 2, 2, dims[l + 1])) / np.sqrt(dims[l + 1]) for l in range(10)]
    C, _ = gpu_fit_pairs([(A, B)], 16, 2, precision="fp64", sketch_p=-1, c_init=[C0])
    ref = ofit.fit_even_odd(A, B, 16, 2, C_init=C0)
    assert mpo.rel_diff(C[0], ref.C) < 1e-10


# (tolerance of the first half-step and its per-bond blocks, of the resumed
# second half-step and its blocks)
@pytest.mark.parametrize("precision,tol,tol_resumed", [("fp64", 1e-10, 5e-10), ("fp32", 1e-5, 1e-5)])
@pytest.mark.parametrize("sketch_p", [-1, 8])
def test_half_steps_from_oracle_states(precision, tol, tol_resumed, sketch_p):
    """Each half-step of the inverse-gauge schedule from a given state: the
    first one from the initial guess (mpo_fit_updates of one half-step), the
    second one resumed from the oracle's merged train after the first
    (first_half = 1: its inverse canonical form and environments), each
    against the oracle's same step.  A whole FP32 sweep is not compared: the
    second half-step's sketch acts on columns in the basis of the first
    half-step's V, which is not fixed inside nearly degenerate singular pairs
    at FP32 precision.  The resumed FP64 half-step (train and blocks) is
    held to 5e-10: it
    starts from the inverse canonical form of a merged train whose singular
    values reach 1.2e-6 of the largest, and the environments divide the rows
    of each Psi by them, so a canonical form accurate to eps in norm per
    bond leaves errors of eps / 1.2e-6 (about 1e-10) in those rows."""
    from paper_2606_23274_amd.api import FitContext
    A, B = make_pair(16, 2, 32, seed=44, decay=True)
    hs0 = {}

    def on_half_step(sweep, q, Cm):
        hs0.setdefault(q, Cm)

    from tests.gpu_util import block_dist, device_blocks, oracle_block
    blk0, blk1 = {}, {}
    ofit.fit_even_odd(A, B, 64, 1, sketch_p=sketch_p, seed=3, on_half_step=on_half_step, n_half_steps=1,
                      on_bond=lambda s, q, l, M, f, P0, Y0: blk0.__setitem__(l, oracle_block(f)))
    ctx = FitContext([(A, B)], 64, precision=precision, schedule="even_odd", sketch_p=sketch_p, seed=3)
    try:
        ctx.updates(1)
        assert ctx.position() == (0, 1)
        C0 = ctx.export_numpy(0)
        b0 = device_blocks(ctx, 0, sorted(blk0))
    finally:
        ctx.close()
    e0 = mpo.rel_diff(C0, hs0[0])
    ref1 = ofit.fit_even_odd(A, B, 64, 1, sketch_p=sketch_p, seed=3, C_init=hs0[0], first_half=1,
                             on_bond=lambda s, q, l, M, f, P0, Y0: blk1.__setitem__(l, oracle_block(f)))
    ctx = FitContext([(A, B)], 64, precision=precision, schedule="even_odd", sketch_p=sketch_p, seed=3,
                     c_init=[hs0[0]], first_half=1)
    try:
        ctx.updates(1)
        assert ctx.position() == (1, 0)
        C1 = ctx.export_numpy(0)
        dims = ctx.bond_dims(0)
        b1 = device_blocks(ctx, 0, sorted(blk1))
    finally:
        ctx.close()
    e1 = mpo.rel_diff(C1, ref1.C)
    be0 = max(block_dist(b0[l], blk0[l]) for l in blk0)
    be1 = max(block_dist(b1[l], blk1[l]) for l in blk1)
    print(precision, sketch_p, "half-step distances", e0, e1, "blocks", be0, be1)
    assert dims == ref1.bond_dims
    assert max(e0, be0) <= tol
    assert max(e1, be1) <= tol_resumed
