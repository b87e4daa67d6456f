"""The adjoint at frozen truncation bases (mpo_fit_grad) against the FP64
oracle gradient at the same bases, central differences of the library's own
loss, and the torch.autograd.Function wrapper."""
import numpy as np
import pytest
import torch

from oracle import fit as ofit
from oracle import grad as ograd
from oracle import mpo
from synth import gaussian_mpo, make_pair

pytestmark = pytest.mark.gpu


def _rel(a, b):
    num = np.sqrt(sum(np.linalg.norm(x - y) ** 2 for x, y in zip(a, b)))
    den = np.sqrt(sum(np.linalg.norm(y) ** 2 for y in b))
    return num / den


def _gpu_state(A, B, chi_c, sweeps, precision, **kw):
    from paper_2606_23274_amd.api import FitContext
    ctx = FitContext([(A, B)], chi_c, precision=precision, **kw)
    ctx.sweep(sweeps)
    C = ctx.export_numpy(0)
    C[0] = C[0] / ctx.norm_factor(0)
    centre = len(A) - 1 if sweeps % 2 == 1 else 0
    return ctx, C, centre


@pytest.mark.parametrize("sweeps", [1, 2])
@pytest.mark.parametrize("recompute", [False, True])
def test_grad_fp64_against_oracle(sweeps, recompute):
    A, B = make_pair(9, 2, 5, seed=21, decay=True)
    W = gaussian_mpo(np.random.default_rng(77), 9, 2, 3)
    ctx, C, centre = _gpu_state(A, B, 10, sweeps, "fp64", sketch_p=3, seed=2)
    try:
        loss, gA, gB = ctx.grad(W, recompute_env=recompute)
    finally:
        ctx.close()
    # the GPU's frozen bases agree with the oracle fit's to 1e-10
    ref_fit = ofit.fit_serial(A, B, 10, sweeps, sketch_p=3, seed=2)
    assert ref_fit.centre == centre
    assert mpo.rel_diff(C, ref_fit.C_norm) < 1e-10
    f, rA, rB = ograd.grad(A, B, ref_fit.C_norm, centre, W)  # the oracle's own bases
    assert abs(loss - f) <= 1e-10 * abs(f)
    assert _rel([g.cpu().numpy() for g in gA], rA) < 1e-10
    assert _rel([g.cpu().numpy() for g in gB], rB) < 1e-10


def test_grad_recompute_identical():
    A, B = make_pair(11, 2, 4, seed=3, decay=True)
    W = gaussian_mpo(np.random.default_rng(5), 11, 2, 2)
    ctx, _, _ = _gpu_state(A, B, 8, 2, "fp64", sketch_p=-1)
    try:
        l0, a0, b0 = ctx.grad(W, recompute_env=False)
        l1, a1, b1 = ctx.grad(W, recompute_env=True)
    finally:
        ctx.close()
    assert l0 == l1
    for x, y in zip(a0 + b0, a1 + b1):
        assert torch.equal(x, y)


def test_grad_central_differences():
    """The loss is linear in each core, so central differences of the
    library's own loss (bases frozen) are exact up to rounding."""
    A, B = make_pair(7, 2, 4, seed=8, decay=True)
    W = gaussian_mpo(np.random.default_rng(9), 7, 2, 3)
    ctx, _, _ = _gpu_state(A, B, 8, 1, "fp64", sketch_p=2, seed=4)
    try:
        _, gA, gB = ctx.grad(W)
        rng = np.random.default_rng(1)
        h = 1e-3
        for which in ("A", "B"):
            for _ in range(6):
                X = [c.copy() for c in (A if which == "A" else B)]
                l = int(rng.integers(len(X)))
                idx = tuple(int(rng.integers(s)) for s in X[l].shape)
                Xp = [c.copy() for c in X]
                Xm = [c.copy() for c in X]
                Xp[l][idx] += h
                Xm[l][idx] -= h
                if which == "A":
                    fp, _, _ = ctx.grad(W, A=Xp, B=B)
                    fm, _, _ = ctx.grad(W, A=Xm, B=B)
                    g = gA[l].cpu().numpy()
                else:
                    fp, _, _ = ctx.grad(W, A=A, B=Xp)
                    fm, _, _ = ctx.grad(W, A=A, B=Xm)
                    g = gB[l].cpu().numpy()
                fd = (fp - fm) / (2 * h)
                assert abs(fd - g[idx]) <= 1e-8 * max(abs(fd), np.abs(g).max())
    finally:
        ctx.close()


def test_autograd_function():
    from paper_2606_23274_amd.api import FitContract
    A, B = make_pair(6, 2, 4, seed=12, decay=True)
    W = gaussian_mpo(np.random.default_rng(13), 6, 2, 2)
    ctx, _, _ = _gpu_state(A, B, 8, 2, "fp64", sketch_p=-1)
    try:
        At = [torch.tensor(a, device="cuda:0", requires_grad=True) for a in A]
        Bt = [torch.tensor(b, device="cuda:0", requires_grad=True) for b in B]
        loss = FitContract.apply(ctx, W, *At, *Bt)
        (3.0 * loss).backward()
        l2, gA, gB = ctx.grad(W)
    finally:
        ctx.close()
    assert abs(loss.item() - l2) <= 1e-12 * abs(l2)
    for t, g in zip(At + Bt, gA + gB):
        torch.testing.assert_close(t.grad, 3.0 * g, rtol=1e-12, atol=0)


def test_grad_fp32_full_size():
    """The differentiation configuration: L=30, d=2, chi_A=chi_B=64 with
    exp(-k/6) bond weights, chi_C=128, sketch p=16, W a seeded Gaussian MPO of
    bond dimension 32, environments recomputed.  The truncation bases are
    frozen after 4 sweeps of the FP64 oracle's fit; the device takes them as
    its initial guess with first_sweep = 4 (centre at the first site, as
    after the fourth, backward sweep) and computes the gradient in FP32.
    Checked against the oracle's FP64 gradient at the same bases (1e-5) and,
    entry by entry, against central differences (h = 1e-3) of the oracle's
    FP64 loss, which are exact up to rounding since the loss is linear in
    each core."""
    from paper_2606_23274_amd.api import FitContext
    A, B = make_pair(30, 2, 64, seed=0, decay=True)
    W = gaussian_mpo(np.random.default_rng(2024), 30, 2, 32)
    res = ofit.fit_serial(A, B, 128, 4, sketch_p=16, seed=0)
    assert res.centre == 0
    ctx = FitContext([(A, B)], 128, precision="fp32", sketch_p=16, seed=0, c_init=[res.C], first_sweep=4)
    try:
        loss, gA, gB = ctx.grad(W, recompute_env=True)
    finally:
        ctx.close()
    gA = [g.cpu().numpy() for g in gA]
    gB = [g.cpu().numpy() for g in gB]
    f, rA, rB = ograd.grad(A, B, res.C_norm, 0, W)
    print("FP32 gradient vs FP64: loss", abs(loss - f) / abs(f), "dA", _rel(gA, rA), "dB", _rel(gB, rB))
    assert abs(loss - f) <= 1e-5 * abs(f)
    assert _rel(gA, rA) < 1e-5
    assert _rel(gB, rB) < 1e-5
    rng = np.random.default_rng(31)
    h = 1e-3
    gmax = max(max(np.abs(g).max() for g in gA), max(np.abs(g).max() for g in gB))
    for which, X, G in (("A", A, gA), ("B", B, gB)):
        for _ in range(4):
            l = int(rng.integers(len(X)))
            idx = tuple(int(rng.integers(s)) for s in X[l].shape)
            Xp = [c.copy() for c in X]
            Xm = [c.copy() for c in X]
            Xp[l][idx] += h
            Xm[l][idx] -= h
            if which == "A":
                fd = (ograd.loss(Xp, B, res.C_norm, 0, W) - ograd.loss(Xm, B, res.C_norm, 0, W)) / (2 * h)
            else:
                fd = (ograd.loss(A, Xp, res.C_norm, 0, W) - ograd.loss(A, Xm, res.C_norm, 0, W)) / (2 * h)
            assert abs(fd - G[l][idx]) <= 1e-5 * gmax, (which, l, idx, fd, G[l][idx])


def test_grad_fp32_own_fit_full_size():
    """The same configuration at the device fit's own bases after 4 FP32
    sweeps: central differences (h = 1e-3) of the library's own FP32 loss
    agree with its gradient to FP32 rounding of the loss (about 1e-7 |loss|
    / h)."""
    from paper_2606_23274_amd.api import FitContext
    A, B = make_pair(30, 2, 64, seed=0, decay=True)
    W = gaussian_mpo(np.random.default_rng(2024), 30, 2, 32)
    ctx = FitContext([(A, B)], 128, precision="fp32", sketch_p=16, seed=0)
    try:
        ctx.sweep(4)
        loss, gA, gB = ctx.grad(W, recompute_env=True)
        assert np.isfinite(loss)
        rng = np.random.default_rng(32)
        h = 1e-3
        gmax = max(max(g.abs().max().item() for g in gA), max(g.abs().max().item() for g in gB))
        for _ in range(3):
            l = int(rng.integers(30))
            idx = tuple(int(rng.integers(s)) for s in A[l].shape)
            Ap = [c.copy() for c in A]
            Am = [c.copy() for c in A]
            Ap[l][idx] += h
            Am[l][idx] -= h
            fp, _, _ = ctx.grad(W, A=Ap, B=B, recompute_env=True)
            fm, _, _ = ctx.grad(W, A=Am, B=B, recompute_env=True)
            fd = (fp - fm) / (2 * h)
            assert abs(fd - gA[l][idx].item()) <= 1e-3 * gmax + 1e-6 * abs(loss) / h
    finally:
        ctx.close()
