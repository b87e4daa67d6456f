"""Resume (mpo_fit_opts.first_sweep), the fit error per sweep (fit_err of
mpo_fit_sweep), the singular values of each bond (mpo_fit_singular_values)
and a two-site matrix of lower rank than the bond cap, against the oracle."""
import numpy as np
import pytest

from oracle import fit as ofit
from oracle import mpo
from synth import gaussian_mpo, make_pair

pytestmark = pytest.mark.gpu


def _ctx(pairs, chi_c, **kw):
    from paper_2606_23274_amd.api import FitContext
    return FitContext(pairs, chi_c, **kw)


@pytest.mark.parametrize("sketch_p", [-1, 4])
@pytest.mark.parametrize("s", [1, 2, 3])
def test_resume_serial_fp64(s, sketch_p):
    """From the oracle's result after s sweeps, one resumed device sweep
    (first_sweep = s: backward for odd s) equals the oracle's resumed sweep."""
    A, B = make_pair(10, 2, 8, seed=3, decay=True)
    Cs = ofit.fit_serial(A, B, 16, s, sketch_p=sketch_p, seed=7).C
    ref = ofit.fit_serial(A, B, 16, 1, sketch_p=sketch_p, seed=7, C_init=Cs, first_sweep=s)
    ctx = _ctx([(A, B)], 16, precision="fp64", sketch_p=sketch_p, seed=7, c_init=[Cs], first_sweep=s)
    try:
        ctx.sweep(1)
        C = ctx.export_numpy(0)
        dims = ctx.bond_dims(0)
    finally:
        ctx.close()
    assert dims == ref.bond_dims
    assert mpo.rel_diff(C, ref.C) < 1e-10


def test_resume_even_odd_stream():
    """Even/odd: first_sweep offsets the Philox stream (2 sweep + q)."""
    A, B = make_pair(10, 2, 6, seed=2, decay=True)
    ref = ofit.fit_even_odd(A, B, 12, 1, sketch_p=4, seed=5, first_sweep=3)
    ctx = _ctx([(A, B)], 12, precision="fp64", schedule="even_odd", sketch_p=4, seed=5, first_sweep=3)
    try:
        ctx.sweep(1)
        C = ctx.export_numpy(0)
    finally:
        ctx.close()
    assert mpo.rel_diff(C, ref.C) < 1e-10


@pytest.mark.parametrize("schedule", ["serial", "even_odd"])
def test_fit_error_per_sweep(schedule):
    """fit_err after each sweep against the dense error of the oracle's C
    (L=8); the transfer passes floor near 1e-8."""
    A, B = make_pair(8, 2, 8, seed=0)
    run = ofit.fit_serial if schedule == "serial" else ofit.fit_even_odd
    ctx = _ctx([(A, B)], 12, precision="fp64", schedule=schedule, sketch_p=-1, track_error=True)
    try:
        eps = ctx.sweep(3, errors=True)[0]
    finally:
        ctx.close()
    for s in range(3):
        ref = mpo.fit_error_dense(A, B, run(A, B, 12, s + 1).C)
        assert abs(eps[s] - ref) <= 1e-7, (s, eps[s], ref)


def test_fit_error_needs_tracking():
    from paper_2606_23274_amd._lib import MpoError
    A, B = make_pair(6, 2, 3, seed=1)
    ctx = _ctx([(A, B)], 6, precision="fp64")
    try:
        with pytest.raises(MpoError):
            ctx.sweep(1, errors=True)
    finally:
        ctx.close()


@pytest.mark.parametrize("schedule", ["serial", "even_odd"])
def test_singular_values(schedule):
    """Each bond's singular values from its last update, against the
    oracle's (normalized cores), after two sweeps."""
    A, B = make_pair(10, 2, 6, seed=12, decay=True)
    last = {}
    if schedule == "serial":
        rec = {}
        orig = ofit.factorize

        def spy(M, *a, **k):
            f = orig(M, *a, **k)
            rec.setdefault("list", []).append(f.S.copy())
            return f

        ofit.factorize = spy
        try:
            ofit.fit_serial(A, B, 12, 2, sketch_p=3, seed=4)
        finally:
            ofit.factorize = orig
        order = list(range(1, 10)) + list(range(9, 0, -1))
        for l, S in zip(order, rec["list"]):
            last[l] = S
    else:
        def on_bond(sweep, q, l, M, f, Psi0, Y0):
            last[l] = f.S.copy()
        ofit.fit_even_odd(A, B, 12, 2, sketch_p=3, seed=4, on_bond=on_bond)
    ctx = _ctx([(A, B)], 12, precision="fp64", schedule=schedule, sketch_p=3, seed=4)
    try:
        ctx.sweep(2)
        for l in range(1, 10):
            S = ctx.singular_values(l)
            assert S.shape == last[l].shape
            assert np.abs(S - last[l]).max() <= 1e-10 * last[l][0], l
    finally:
        ctx.close()


def _identity_mpo(L, d, chi):
    out = []
    for l in range(L):
        cl = 1 if l == 0 else chi
        cr = 1 if l == L - 1 else chi
        core = np.zeros((cl, d, d, cr))
        for i in range(d):
            core[0, i, i, 0] = 1.0
        out.append(core)
    return out


@pytest.mark.parametrize("sketch_p", [-1, 2])
@pytest.mark.parametrize("schedule", ["serial", "even_odd"])
def test_rank_deficient_product(schedule, sketch_p):
    """B = the identity on a bond of dimension 2, so A B = A has half the
    structural rank chi^A chi^B: the two-site matrices have fewer nonzero
    singular values than the bond cap.  The extra values are dropped on both
    sides (no NUMERIC failure), the fit reproduces A and matches the oracle."""
    L, d, chi = 8, 2, 3
    A = gaussian_mpo(np.random.default_rng(50), L, d, chi)
    B = _identity_mpo(L, d, 2)
    run = ofit.fit_serial if schedule == "serial" else ofit.fit_even_odd
    ref = run(A, B, 6, 3, sketch_p=sketch_p, seed=1)
    ctx = _ctx([(A, B)], 6, precision="fp64", schedule=schedule, sketch_p=sketch_p, seed=1)
    try:
        ctx.sweep(3)
        C = ctx.export_numpy(0)
        dims = ctx.bond_dims(0)
        dropped = ctx.truncations()
    finally:
        ctx.close()
    assert dims == ref.bond_dims
    assert dropped > 0
    assert mpo.fit_error_dense(A, B, C) < 1e-12
    assert mpo.rel_diff(C, ref.C) < 1e-10
