"""MPO-MPS fits on the GPU (mpo_fit_opts.mps, Sec. 1: B an MPS stored with a
unit input leg, C likewise, the default guess B) against the oracle's
fit_serial / fit_even_odd on the same inputs, and the refusals."""
import numpy as np
import pytest

from oracle import fit as ofit
from oracle import mpo
from synth.mpo_inputs import gaussian_mpo

pytestmark = pytest.mark.gpu


def _pair(L, d, chi_a, chi_b, seed):
    rng = np.random.default_rng(seed)
    A = gaussian_mpo(rng, L, d, chi_a, decay=True)
    B = [b[:, :, :1, :].copy() for b in gaussian_mpo(rng, L, d, chi_b, decay=True)]
    return A, B


def _gpu(pairs, chi, sweeps, **kw):
    from paper_2606_23274_amd.api import FitContext
    ctx = FitContext(pairs, chi, **kw)
    try:
        assert ctx._setup.mps
        ctx.sweep(sweeps)
        return [ctx.export_numpy(i) for i in range(len(pairs))], [ctx.bond_dims(i) for i in range(len(pairs))]
    finally:
        ctx.close()


_ORACLE = {"serial": ofit.fit_serial, "even_odd": ofit.fit_even_odd}


@pytest.mark.parametrize("schedule", ["serial", "even_odd"])
@pytest.mark.parametrize("sketch_p", [-1, 3])
@pytest.mark.parametrize("sweeps", [1, 2])
def test_mps_fp64_matches_oracle(schedule, sketch_p, sweeps):
    """L = 10, d = 2, chi^A = 6, chi^B = 5, chi_C = 8: truncating bonds."""
    A, B = _pair(10, 2, 6, 5, seed=1)
    (C,), (dims,) = _gpu([(A, B)], 8, sweeps, precision="fp64", schedule=schedule, sketch_p=sketch_p, seed=4)
    ref = _ORACLE[schedule](A, B, 8, sweeps, sketch_p=sketch_p, seed=4)
    assert all(c.shape[2] == 1 for c in C)
    assert dims == ref.bond_dims
    d = mpo.rel_diff(C, ref.C)
    print("mps", schedule, sketch_p, sweeps, d)
    assert d < 1e-10


@pytest.mark.parametrize("schedule", ["serial", "even_odd"])
def test_mps_d3_fp32(schedule):
    """d = 3 (ragged against the 64-wide tiles), FP32 at 1e-5."""
    A, B = _pair(7, 3, 5, 4, seed=2)
    (C,), (dims,) = _gpu([(A, B)], 10, 2, precision="fp32", schedule=schedule, sketch_p=4, seed=2)
    ref = _ORACLE[schedule](A, B, 10, 2, sketch_p=4, seed=2)
    assert dims == ref.bond_dims
    d = mpo.rel_diff(C, ref.C)
    print("mps fp32", schedule, d)
    assert d < 1e-5


def test_mps_exact_regime_is_the_matrix_vector_product():
    A, B = _pair(8, 2, 3, 3, seed=3)
    (C,), _ = _gpu([(A, B)], 64, 2, precision="fp64")
    y = mpo.dense(A) @ mpo.dense(B)[:, 0]
    assert np.linalg.norm(mpo.dense(C)[:, 0] - y) <= 1e-11 * np.linalg.norm(y)


@pytest.mark.parametrize("tau", [0.3, 1.0])
def test_mps_tolerance_truncation(tau):
    """Sec. 2.3.4's tolerance picks ranks below the cap on the inner bonds."""
    A, B = _pair(10, 2, 6, 5, seed=5)
    (C,), (dims,) = _gpu([(A, B)], 12, 2, precision="fp64", sketch_p=-1, tau=tau)
    ref = ofit.fit_serial(A, B, 12, 2, tau=tau)
    assert dims == ref.bond_dims
    assert mpo.rel_diff(C, ref.C) < 1e-10


def test_mps_initial_guess_and_resume():
    """c_init with MPS cores, and first_sweep = 1 resuming a one-sweep fit."""
    A, B = _pair(9, 2, 5, 4, seed=6)
    ref1 = ofit.fit_serial(A, B, 7, 1, sketch_p=2, seed=3)
    ref2 = ofit.fit_serial(A, B, 7, 2, sketch_p=2, seed=3)
    (C,), (dims,) = _gpu([(A, B)], 7, 1, precision="fp64", sketch_p=2, seed=3, c_init=[ref1.C], first_sweep=1)
    assert dims == ref2.bond_dims
    assert mpo.rel_diff(C, ref2.C) < 1e-10


def test_mps_multi_pair_ragged_even_odd():
    pairs = [_pair(8, 2, ca, cb, seed=20 + i) for i, (ca, cb) in enumerate([(3, 4), (6, 2), (5, 5)])]
    caps = [6, 9, 12]
    Cs, dims = _gpu(pairs, 12, 2, precision="fp64", schedule="even_odd", sketch_p=2, seed=9, pair_chi_max=caps)
    for i, (A, B) in enumerate(pairs):
        ref = ofit.fit_even_odd(A, B, caps[i], 2, sketch_p=2, seed=9, pair=i)
        assert dims[i] == ref.bond_dims
        assert mpo.rel_diff(Cs[i], ref.C) < 1e-10


def test_mps_larger_serial():
    """L = 24, chi^A = chi^B = 32, chi_C = 48, p = 8, one sweep: several GEMM
    tiles per operand and a ragged tail."""
    A, B = _pair(24, 2, 32, 32, seed=7)
    (C,), (dims,) = _gpu([(A, B)], 48, 1, precision="fp64", sketch_p=8, seed=1)
    ref = ofit.fit_serial(A, B, 48, 1, sketch_p=8, seed=1)
    assert dims == ref.bond_dims
    d = mpo.rel_diff(C, ref.C)
    print("mps larger", d)
    assert d < 1e-10


def test_mps_refusals():
    from paper_2606_23274_amd import _lib
    from paper_2606_23274_amd.api import FitContext
    A, B = _pair(8, 2, 3, 3, seed=8)
    for kw in ({"track_error": True}, {"schedule": "parallel", "n_parts": 2}):
        with pytest.raises(_lib.MpoError) as e:
            FitContext([(A, B)], 6, precision="fp64", **kw)
        assert e.value.status == 6
    ctx = FitContext([(A, B)], 6, precision="fp64")
    try:
        ctx.sweep(1)
        W = [np.ones((1, 2, 2, 1)) for _ in range(8)]
        with pytest.raises(_lib.MpoError) as e:
            ctx.grad(W)
        assert e.value.status == 6
    finally:
        ctx.close()


def test_mps_split_bf16_first_sweep():
    """Split BF16 contractions (FP64 factorizations) at the BF16 bar of 3e-3."""
    A, B = _pair(12, 2, 8, 8, seed=9)
    (C,), (dims,) = _gpu([(A, B)], 12, 1, precision="bf16x3", sketch_p=4, seed=2)
    ref = ofit.fit_serial(A, B, 12, 1, sketch_p=4, seed=2)
    assert dims == ref.bond_dims
    d = mpo.rel_diff(C, ref.C)
    print("mps bf16x3", d)
    assert d < 3e-3


def test_mps_even_odd_second_half_resume():
    """first_half = 1 from an MPS guess: the second half-step alone, as the
    oracle's resumed even/odd fit."""
    A, B = _pair(9, 2, 5, 4, seed=10)
    g = ofit.fit_serial(A, B, 6, 1, sketch_p=2, seed=5).C
    ref = ofit.fit_even_odd(A, B, 6, 1, sketch_p=2, seed=5, C_init=g, first_half=1)
    (C,), (dims,) = _gpu([(A, B)], 6, 1, precision="fp64", schedule="even_odd", sketch_p=2, seed=5,
                         c_init=[g], first_half=1)
    assert dims == ref.bond_dims
    assert mpo.rel_diff(C, ref.C) < 1e-10


def test_mps_graph_replay_matches_eager():
    """A captured sweep replays the eager one bit for bit."""
    A, B = _pair(10, 2, 6, 5, seed=11)
    outs = []
    for graph in (False, True):
        (C,), _ = _gpu([(A, B)], 8, 4, precision="fp32", sketch_p=3, seed=1, capture_graph=graph)
        outs.append(C)
    for a, b in zip(*outs):
        assert np.array_equal(a, b)


@pytest.mark.parametrize("s,b", [(0, 3), (1, 5)])
def test_mps_resume_mid_sweep(s, b):
    """first_bond = b inside sweep s from the oracle's state after b updates:
    the next update, and the rest of the sweep, as the uninterrupted fit."""
    A, B = _pair(9, 2, 5, 4, seed=12)
    states = []
    ofit.fit_serial(A, B, 6, s + 1, sketch_p=2, seed=5,
                    on_update=lambda sweep, l, Cs: states.append((sweep, l, [c.copy() for c in Cs])))
    in_sweep = [st for st in states if st[0] == s]
    before, after, end = in_sweep[b - 1][2], in_sweep[b][2], in_sweep[-1][2]
    from paper_2606_23274_amd.api import FitContext
    for n, want in ((1, after), (None, end)):
        ctx = FitContext([(A, B)], 6, precision="fp64", sketch_p=2, seed=5, c_init=[before], first_sweep=s,
                         first_bond=b)
        try:
            if n is None:
                ctx.sweep(1)
            else:
                ctx.updates(n)
            C = ctx.export_numpy(0)
        finally:
            ctx.close()
        assert [c.shape for c in C] == [c.shape for c in want]
        assert mpo.rel_diff(C, want) < 1e-10
