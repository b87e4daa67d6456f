"""The serial randomized fit at the headline configuration's full size:
L=40, d=2, chi_A=chi_B=64 with exp(-k/6) bond weights, chi_C=128, sketch
p=16 (Philox seed 0), the size and launch configuration the benchmark times.

The FP64 oracle's six sweeps (about 6 s each on 16 host cores) are the
reference.  The device's first sweep is compared element by element through
the exported train; in sweeps 2..6 single updates at five positions each
(both directions) are compared after resuming from the oracle's state just
before them (first_sweep, first_bond, c_init; the resumed oracle equals the
uninterrupted one to rounding, which the oracle's own tests pin).
Tolerances: FP64 1e-10, FP32 contractions 1e-5, split BF16 3e-3 (relative
Frobenius distance of the MPO C, all cores at once), with the same bond
dimensions.  Pure BF16 (one BF16 product per term) misses 3e-3 and is marked
as an expected failure with its measured distance."""
import numpy as np
import pytest

from oracle import fit as ofit
from oracle import mpo
from synth import make_pair

pytestmark = pytest.mark.gpu

L, D, CHI, CHI_C, P, SEED, SWEEPS = 40, 2, 64, 128, 16, 0, 6


POSITIONS = (0, 8, 19, 30, 38)  # updates already done in the sweep: both ends, the middle, between


@pytest.fixture(scope="module")
def case():
    """One run of the oracle's six sweeps: the train after the first sweep,
    and the states around single updates of sweeps 2..6: for each (sweep,
    position) the train before the update and the two cores it changes
    (0-based sites i, i+1) after it."""
    A, B = make_pair(L, D, CHI, seed=SEED, decay=True)
    traj, cases, state, count = {}, [], {}, {}

    def on_update(sweep, l, Cs):
        if sweep == 0 and l == L - 1:
            traj[1] = Cs
        if sweep > 0:
            pos = count.get(sweep, 0)
            count[sweep] = pos + 1
            if pos in POSITIONS:
                i = l - 1
                cases.append((sweep, pos, state["C"], i, Cs[i].copy(), Cs[i + 1].copy()))
        state["C"] = Cs

    ofit.fit_serial(A, B, CHI_C, SWEEPS, sketch_p=P, seed=SEED, on_update=on_update)
    return A, B, traj, cases


@pytest.fixture(scope="module")
def tables(case):
    from paper_2606_23274_amd.api import autotune
    A, B = case[0], case[1]
    cache = {}

    def get(precision):
        if precision not in cache:
            cache[precision] = autotune([(A, B)], CHI_C, precision=precision, sketch_p=P, seed=SEED,
                                        reps=3)
        return cache[precision]
    return get


PRECISIONS = [("fp64", 1e-10), ("fp32", 1e-5), ("bf16x3", 3e-3),
              pytest.param("bf16", 3e-3, marks=pytest.mark.xfail(
                  reason="pure BF16 operands: 2^-9 rounding chained through the environments, "
                         "about 3e-2 from the oracle after one sweep", strict=True))]


def _run(A, B, precision, table, sweeps=1, **kw):
    from paper_2606_23274_amd.api import FitContext
    ctx = FitContext([(A, B)], CHI_C, precision=precision, schedule="serial", sketch_p=P, seed=SEED,
                     tuning=table, **kw)
    try:
        ctx.sweep(sweeps)
        return ctx.export_numpy(0), ctx.bond_dims(0)
    finally:
        ctx.close()


@pytest.mark.parametrize("precision,tol", PRECISIONS)
def test_first_sweep_full_size(case, tables, precision, tol):
    A, B, traj, _ = case
    C, dims = _run(A, B, precision, tables(precision))
    ref = traj[1]
    assert dims == mpo.bond_dims(ref)
    assert all(np.isfinite(c).all() for c in C)
    err = mpo.rel_diff(C, ref)
    print(precision, "relative distance to the oracle after sweep 1:", err)
    assert err <= tol


@pytest.mark.parametrize("precision,tol", PRECISIONS[:3])
def test_single_updates_full_size(case, tables, precision, tol):
    """Single two-site updates of sweeps 2..6 (both directions, so the
    backward branch V = orth(B_k^T Z S^-1), C_l = Q Z S at k = 144 too), each
    started from the oracle's state just before it (first_sweep, first_bond,
    c_init) and compared with the oracle's state just after it.  Whole later
    sweeps are not compared: from the second update of a backward sweep the
    sketch acts on columns in the basis of the previous update's V, which is
    not fixed inside nearly degenerate singular pairs at the working
    precision, so longer stretches differ by the sketch's own error."""
    from paper_2606_23274_amd.api import FitContext
    A, B, _, cases = case
    assert len(cases) == len(POSITIONS) * (SWEEPS - 1)
    errs = []
    for sweep, pos, before, i, ci, cn in cases:
        after = [c for c in before]
        after[i], after[i + 1] = ci, cn
        ctx = FitContext([(A, B)], CHI_C, precision=precision, schedule="serial", sketch_p=P, seed=SEED,
                         tuning=tables(precision), c_init=[before], first_sweep=sweep, first_bond=pos)
        try:
            ctx.updates(1)
            C = ctx.export_numpy(0)
            dims = ctx.bond_dims(0)
            assert ctx.position() == (sweep, pos + 1) or (pos == L - 2 and ctx.position() == (sweep + 1, 0))
        finally:
            ctx.close()
        assert dims == mpo.bond_dims(after), (sweep, pos)
        errs.append(mpo.rel_diff(C, after))
    print(precision, "relative distance after single updates:", ["%.1e" % e for e in errs])
    assert max(errs) <= tol
