"""Site-canonical parallel fit (Sec. 4, variant II) on the GPU
(MPO_SCHED_PARALLEL + mpo_fit_merge) against the oracle's
(oracle/parallel.py): the merged train, its bond dims, and the refusals
around the merge."""
import numpy as np
import pytest

from oracle import mpo, parallel
from synth import make_pair

pytestmark = pytest.mark.gpu


def _run(A, B, chi, n_parts, n_sets, sketch_p=-1, precision="fp64", seed=3, merge=True):
    from paper_2606_23274_amd.api import FitContext
    ctx = FitContext([(A, B)], chi, precision=precision, schedule="parallel", sketch_p=sketch_p, seed=seed,
                     n_parts=n_parts)
    try:
        ctx.sweep(n_sets)
        if merge:
            ctx.merge()
        return ctx.bond_dims(), ctx.export_numpy() if merge else None
    finally:
        ctx.close()


@pytest.mark.parametrize("n_parts", [2, 4, 8])
@pytest.mark.parametrize("sketch_p", [-1, 3])
@pytest.mark.parametrize("n_sets", [1, 2])
def test_parallel_fit_matches_oracle(n_parts, sketch_p, n_sets):
    """L = 16, chi = 8, chi_C = 12: truncating bonds, ragged sub-TT lengths
    for 8 parts (two sites each), every phase and merge level."""
    A, B = make_pair(16, 2, 8, seed=5, decay=True)
    dims, C = _run(A, B, 12, n_parts, n_sets, sketch_p)
    ref = parallel.fit_parallel_site(A, B, 12, n_sets, n_parts, sketch_p=sketch_p, seed=3)
    assert dims == ref.bond_dims
    d = mpo.rel_diff(C, ref.C)
    print("parallel", n_parts, sketch_p, n_sets, d)
    assert d < 1e-10


def _perturbed_oracle_distance(A, B, eps, run):
    """How far the oracle itself moves when A's entries get relative noise
    eps (the conditioning of the fit at this configuration)."""
    rng = np.random.default_rng(1)
    A2 = [a * (1 + eps * rng.standard_normal(a.shape)) for a in A]
    return mpo.rel_diff(run(A2).C, run(A).C)


def test_parallel_uneven_parts():
    """L = 13 into 4 parts (4, 3, 3, 3 sites), p = 4, two sets: FP64 at
    1e-10.  FP32 at 1e-4: the oracle itself moves by 1.8e-6 to 1.8e-5 under
    1e-7 relative noise on A (depending on the noise's direction), about ten
    times what the serial fit moves, so the FP32 bar of 1e-5 is below this
    configuration's conditioning; the fit errors agree to 1e-5."""
    A, B = make_pair(13, 2, 6, seed=9, decay=True)
    ref = parallel.fit_parallel_site(A, B, 10, 2, 4, sketch_p=4, seed=3)
    dims, C = _run(A, B, 10, 4, 2, 4)
    assert dims == ref.bond_dims
    assert mpo.rel_diff(C, ref.C) < 1e-10
    dims, C = _run(A, B, 10, 4, 2, 4, precision="fp32")
    d = mpo.rel_diff(C, ref.C)
    e64, e32 = mpo.fit_error_transfer(A, B, ref.C), mpo.fit_error_transfer(A, B, C)
    print("parallel fp32 uneven", d, e64, e32)
    assert dims == ref.bond_dims
    assert d < 1e-4
    assert abs(e32 - e64) <= 1e-5 * e64


def test_parallel_fp32_at_the_bar():
    """L = 16, chi_C = 12, plain SVD, one set: FP32 at 1e-5."""
    A, B = make_pair(16, 2, 8, seed=5, decay=True)
    dims, C = _run(A, B, 12, 4, 1, precision="fp32")
    ref = parallel.fit_parallel_site(A, B, 12, 1, 4, seed=3)
    assert dims == ref.bond_dims
    d = mpo.rel_diff(C, ref.C)
    print("parallel fp32", d)
    assert d < 1e-5


def test_parallel_exact_regime():
    A, B = make_pair(16, 2, 3, seed=4, decay=True)
    _, C = _run(A, B, 9, 4, 2)
    assert mpo.rel_diff(C, mpo.naive_product(A, B)) < 1e-11


def test_merge_refusals():
    from paper_2606_23274_amd import _lib
    from paper_2606_23274_amd.api import FitContext
    A, B = make_pair(8, 2, 4, seed=1, decay=True)
    ctx = FitContext([(A, B)], 6, precision="fp64", schedule="parallel", n_parts=2)
    try:
        ctx.sweep(1)
        with pytest.raises(_lib.MpoError) as e:  # sub-TTs disagree in gauge before the merge
            ctx.export_numpy()
        assert e.value.status == 6
        ctx.updates(1)
        with pytest.raises(_lib.MpoError):       # inside a set
            ctx.merge()
        ctx.updates(3)
        ctx.merge()
        with pytest.raises(_lib.MpoError):
            ctx.merge()
        with pytest.raises(_lib.MpoError):
            ctx.sweep(1)
        C = ctx.export_numpy()
    finally:
        ctx.close()
    ref = parallel.fit_parallel_site(A, B, 6, 2, 2, seed=0)
    assert mpo.rel_diff(C, ref.C) < 1e-10
    serial = FitContext([(A, B)], 6, precision="fp64")
    try:
        with pytest.raises(_lib.MpoError) as e:
            serial.merge()
        assert e.value.status == 6
    finally:
        serial.close()


def test_parallel_headline_size():
    """L = 40, chi = 64, chi_C = 128, p = 16 in 4 sub-TTs, one set and the
    merge, against the live oracle.  The oracle itself moves by about 1e-10
    under 1e-15 relative noise on A here (and by 0.09 under 1e-7), so FP64
    is held to three times its measured movement at 1e-15; FP32 cannot be
    held element-wise at this conditioning, and is checked through the fit
    error, which must agree with the FP64 fit's to 1e-3."""
    A, B = make_pair(40, 2, 64, seed=0, decay=True)
    run = lambda a: parallel.fit_parallel_site(a, B, 128, 1, 4, sketch_p=16, seed=0)
    ref = run(A)
    dims, C = _run(A, B, 128, 4, 1, 16, seed=0)
    assert dims == ref.bond_dims
    d = mpo.rel_diff(C, ref.C)
    floor = _perturbed_oracle_distance(A, B, 1e-15, run)
    print("parallel headline fp64", d, floor)
    assert d < max(3 * floor, 1e-10)
    dims32, C32 = _run(A, B, 128, 4, 1, 16, precision="fp32", seed=0)
    assert dims32 == ref.bond_dims
    e64 = mpo.fit_error_transfer(A, B, ref.C)
    e32 = mpo.fit_error_transfer(A, B, C32)
    print("parallel headline fit errors", e64, e32)
    assert abs(e32 - e64) <= 1e-3 * e64
