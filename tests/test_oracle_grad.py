"""Pins of the gradient oracle (frozen truncation bases)."""
import numpy as np
import pytest
import torch

from oracle import fit as ofit
from oracle import grad as ograd
from oracle import mpo
from synth import gaussian_mpo, make_pair


def _vec_sites(cores):
    """X[(s1 u1), ..., (sL uL)] of an MPO with a trivial outer bond, as a
    (d^2)^(L-1) x d^2 matrix (all but the last site as rows)."""
    T = np.ones((1, 1))
    for c in cores:
        a, d1, d2, b = c.shape
        T = np.tensordot(T, c.reshape(a, d1 * d2, b), axes=([1], [0])).reshape(-1, b)
    return T.reshape(-1)


def _setup(L=4, chi=3, sweeps=1, seed=0):
    A, B = make_pair(L, 2, chi, seed=seed, decay=True)
    res = ofit.fit_serial(A, B, 4, sweeps)
    rng = np.random.default_rng(seed + 100)
    W = gaussian_mpo(rng, L, 2, 2)
    return A, B, res.C_norm, res.centre, W


@pytest.mark.parametrize("sweeps", [1, 2])
def test_loss_matches_dense_projector(sweeps):
    A, B, C, centre, W = _setup(sweeps=sweeps)
    L, dd = len(A), 4
    assert centre == (L - 1 if sweeps == 1 else 0)
    # dense isometry of the frozen cores and the projector onto span(V) x site
    if centre == L - 1:
        T = np.ones((1, 1))
        for c in C[:L - 1]:
            a, d1, d2, b = c.shape
            T = np.tensordot(T, c.reshape(a, dd, b), axes=([1], [0])).reshape(-1, b)
        V = T                                            # (dd^(L-1)) x chi
        Pm = lambda X: (V @ (V.T @ X.reshape(dd ** (L - 1), dd))).reshape(-1)
    else:
        T = np.ones((1, 1))
        for c in reversed(C[1:]):
            a, d1, d2, b = c.shape
            T = np.tensordot(c.reshape(a, dd, b), T, axes=([2], [0])).reshape(a, -1)
        V = T                                            # chi x (dd^(L-1))
        Pm = lambda X: ((X.reshape(dd, dd ** (L - 1)) @ V.T) @ V).reshape(-1)
    np.testing.assert_allclose(V @ V.T if centre == 0 else V.T @ V, np.eye(V.shape[0 if centre == 0 else 1]),
                               atol=1e-12)
    ab = _vec_sites(mpo.naive_product(A, B))
    w = _vec_sites(W)
    expect = float(w @ Pm(ab))
    got = ograd.loss(A, B, C, centre, W)
    assert abs(got - expect) <= 1e-12 * max(1.0, abs(expect))
    # symmetry of the projector: <W, Pi(AB)> = <Pi(W), AB>
    assert abs(float(Pm(w) @ ab) - expect) <= 1e-12 * max(1.0, abs(expect))


@pytest.mark.parametrize("sweeps", [1, 2])
def test_projector_idempotent(sweeps):
    A, B, C, centre, W = _setup(L=5, sweeps=sweeps, seed=3)
    P1 = ograd.projected_w(C, centre, W)
    P2 = ograd.projected_w(C, centre, P1)
    assert mpo.rel_diff(P2, P1) < 1e-12


@pytest.mark.parametrize("sweeps", [1, 2])
def test_gradient_central_differences(sweeps):
    A, B, C, centre, W = _setup(L=5, chi=3, sweeps=sweeps, seed=5)
    f, gA, gB = ograd.grad(A, B, C, centre, W)
    assert abs(f - ograd.loss(A, B, C, centre, W)) <= 1e-13 * abs(f)
    rng = np.random.default_rng(9)
    h = 1e-3
    for which, G in (("A", gA), ("B", gB)):
        for _ in range(12):
            l = int(rng.integers(len(A)))
            X = [c.copy() for c in (A if which == "A" else B)]
            idx = tuple(int(rng.integers(s)) for s in X[l].shape)
            Xp = [c.copy() for c in X]
            Xm = [c.copy() for c in X]
            Xp[l][idx] += h
            Xm[l][idx] -= h
            if which == "A":
                fd = (ograd.loss(Xp, B, C, centre, W) - ograd.loss(Xm, B, C, centre, W)) / (2 * h)
            else:
                fd = (ograd.loss(A, Xp, C, centre, W) - ograd.loss(A, Xm, C, centre, W)) / (2 * h)
            scale = max(abs(fd), np.abs(G[l]).max(), 1e-300)
            assert abs(fd - G[l][idx]) <= 1e-8 * scale


@pytest.mark.parametrize("sweeps", [1, 2])
def test_gradient_against_torch_autograd(sweeps):
    A, B, C, centre, W = _setup(L=6, chi=3, sweeps=sweeps, seed=11)
    f, gA, gB = ograd.grad(A, B, C, centre, W)
    P = [torch.from_numpy(p) for p in ograd.projected_w(C, centre, W)]
    At = [torch.tensor(a, dtype=torch.float64, requires_grad=True) for a in A]
    Bt = [torch.tensor(b, dtype=torch.float64, requires_grad=True) for b in B]
    E = torch.ones((1, 1, 1), dtype=torch.float64)
    for p, a, b in zip(P, At, Bt):
        # E'[x', a', b'] = E[x, a, b] P[x, s, u, x'] A[a, s, t, a'] B[b, t, u, b']
        E = torch.einsum("xab,xsuy,astc,btud->ycd", E, p, a, b)
    loss = E.reshape(-1)[0]
    loss.backward()
    assert abs(loss.item() - f) <= 1e-12 * abs(f)
    for l in range(len(A)):
        np.testing.assert_allclose(gA[l], At[l].grad.numpy(), rtol=1e-10, atol=1e-12 * np.abs(gA[l]).max())
        np.testing.assert_allclose(gB[l], Bt[l].grad.numpy(), rtol=1e-10, atol=1e-12 * np.abs(gB[l]).max())
