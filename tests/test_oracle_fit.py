"""Pins of the oracle's fit (Sec. 2.3, Alg. 3-5, Sec. 3.1, Sec. 4) against
brute-force dense algebra, closed forms and invariants."""
import numpy as np
import pytest

from oracle import canon, fit, mpo
from oracle.philox import gaussian_matrix
from synth import gaussian_mpo, make_pair


def _dense_unfold(D, L, d, l):
    """Dense operator reshaped across bond l (1-based) to (x_<=l y_<=l) x (x_>l y_>l)."""
    a = d ** l
    b = d ** (L - l)
    return D.reshape(a, b, a, b).transpose(0, 2, 1, 3).reshape(a * a, b * b)


def test_two_site_matrix_is_projected_dense_product():
    """Theta_l equals A B projected onto C's left and right isometries (Fig. derivatives)."""
    L, d = 5, 2
    A, B = make_pair(L, d, 3, seed=3)
    C = canon.right_orthogonalize(canon.left_orthogonalize(gaussian_mpo(
        np.random.default_rng(9), L, d, 4))[0])
    # make sites 1..l-1 left orthogonal (C mixed canonical around bond l = 3)
    l = 3
    Cl = [c.copy() for c in C]
    for j in range(l - 1):
        cl, d1, d2, cr = Cl[j].shape
        Q, R = canon.qr_pos(Cl[j].reshape(-1, cr))
        Cl[j] = Q.reshape(cl, d1, d2, Q.shape[1])
        Cl[j + 1] = np.tensordot(R, Cl[j + 1], axes=(1, 0))
    ones = np.ones((1, 1, 1))
    Lenv = ones
    for j in range(l - 1):
        Lenv = fit.env_left(Lenv, Cl[j], A[j], B[j])
    Renv = ones
    for j in range(L - 1, l, -1):
        Renv = fit.env_right(Renv, Cl[j], A[j], B[j])
    M = fit.two_site_matrix(Lenv, A[l - 1], B[l - 1], A[l], B[l], Renv)
    # dense: left isometry maps (x_<l, y_<l) -> c ; right maps c'' -> (x_>l+1, y_>l+1)
    P = mpo.dense(A) @ mpo.dense(B)
    # build left isometry explicitly: T[x, y, c]
    T = Cl[0][0]
    for j in range(1, l - 1):
        T = np.einsum("xyc,csuC->xsyuC", T, Cl[j]).reshape(T.shape[0] * d, T.shape[1] * d, -1)
    V = Cl[L - 1][:, :, :, 0]
    for j in range(L - 2, l, -1):
        V = np.einsum("csuC,Cxy->csxuy", Cl[j], V).reshape(Cl[j].shape[0], V.shape[1] * d,
                                                             V.shape[2] * d)
    nl, nr = d ** (l - 1), d ** (L - l - 1)
    P6 = P.reshape(nl, d, d, nr, nl, d, d, nr)  # x_<, s1, s2, x_>, y_<, u1, u2, y_>
    Theta = np.einsum("xyc,xabXyefY,FXY->caebfF", T, P6, V)
    n, m = M.shape
    assert np.allclose(M, Theta.reshape(n, m), atol=1e-13 * np.abs(M).max())


def test_L2_is_eckart_young():
    """L = 2: the fit is one truncated SVD of the d^2 x d^2 unfolding (Eckart-Young)."""
    rng = np.random.default_rng(4)
    A = gaussian_mpo(rng, 2, 3, 2)
    B = gaussian_mpo(rng, 2, 3, 2)
    res = fit.fit_serial(A, B, 3, 1)
    P = mpo.dense(A) @ mpo.dense(B)
    sv = np.linalg.svd(_dense_unfold(P, 2, 3, 1), compute_uv=False)
    tail = np.sqrt(np.sum(sv[3:] ** 2))
    err = np.linalg.norm(P - mpo.dense(res.C))
    assert abs(err - tail) < 1e-12 * np.linalg.norm(P)
    assert res.bond_dims == [1, 3, 1]


@pytest.mark.parametrize("sketch_p", [-1, 2])
@pytest.mark.parametrize("schedule", ["serial", "even_odd"])
def test_exact_rank_regime(schedule, sketch_p):
    """chi_C >= chi_A chi_B: the fit reproduces A B to rounding."""
    A, B = make_pair(6, 2, 3, seed=1)
    f = fit.fit_serial if schedule == "serial" else fit.fit_even_odd
    res = f(A, B, 9, 4, sketch_p=sketch_p)
    assert mpo.fit_error_dense(A, B, res.C) < 1e-12


def test_error_lower_bound_and_monotone():
    """Dense checks on the small dense workload (L=8, chi=8, chi_C=16, 4 sweeps):
    the error never increases from one update to the next (each update is a
    constrained minimizer over a set containing the current C), and it is
    bounded below by the tail of every dense bond unfolding."""
    L, d = 8, 2
    A, B = make_pair(L, d, 8, seed=0)
    errs = []
    res = fit.fit_serial(A, B, 16, 4,
                         on_update=lambda s, l, C: errs.append(mpo.fit_error_dense(A, B, C)))
    assert len(errs) == 4 * (L - 1)
    for e0, e1 in zip(errs, errs[1:]):
        assert e1 <= e0 * (1 + 1e-12) + 1e-14
    P = mpo.dense(A) @ mpo.dense(B)
    lb = 0.0
    for l in range(1, L):
        sv = np.linalg.svd(_dense_unfold(P, L, d, l), compute_uv=False)
        lb = max(lb, np.sqrt(np.sum(sv[res.bond_dims[l]:] ** 2)) / np.linalg.norm(P))
    assert errs[-1] >= lb * (1 - 1e-12)
    assert errs[-1] < 0.6


def test_forward_updates_leave_isometries():
    A, B = make_pair(8, 2, 6, seed=5, decay=True)
    res = fit.fit_serial(A, B, 12, 1)  # one forward pass
    C = [c.copy() for c in res.C]
    C[0] = C[0] / res.nu
    for core in C[:-1]:
        cl, d1, d2, cr = core.shape
        X = core.reshape(-1, cr)
        assert np.abs(X.T @ X - np.eye(cr)).max() < 1e-13


def test_backward_updates_leave_right_isometries():
    A, B = make_pair(8, 2, 6, seed=5, decay=True)
    res = fit.fit_serial(A, B, 12, 2)
    for core in res.C[1:]:
        X = core.reshape(core.shape[0], -1)
        assert np.abs(X @ X.T - np.eye(core.shape[0])).max() < 1e-13


def test_gauge_invariance_of_plain_fit():
    """Random invertible transforms on the bonds of A and B leave the (plain
    SVD) fit result unchanged as an operator."""
    L = 7
    A, B = make_pair(L, 2, 5, seed=6, decay=True)
    rng = np.random.default_rng(7)
    Ag, Bg = [a.copy() for a in A], [b.copy() for b in B]
    for X in (Ag, Bg):
        for l in range(L - 1):
            chi = X[l].shape[3]
            G = rng.standard_normal((chi, chi)) + 3 * np.eye(chi)
            X[l] = np.tensordot(X[l], G, axes=(3, 0))
            X[l + 1] = np.tensordot(np.linalg.inv(G), X[l + 1], axes=(1, 0))
    r0 = fit.fit_serial(A, B, 10, 4)
    r1 = fit.fit_serial(Ag, Bg, 10, 4)
    assert mpo.rel_diff(r1.C, r0.C) < 1e-10


def test_rsvd_full_width_is_svd_path():
    # chi^A chi^B = 64 >= n, m everywhere, so k = min(n, m): the plain SVD branch
    A, B = make_pair(6, 2, 8, seed=2, decay=True)
    r0 = fit.fit_serial(A, B, 8, 2)
    r1 = fit.fit_serial(A, B, 8, 2, sketch_p=1000)
    for a, b in zip(r0.C, r1.C):
        assert np.array_equal(a, b)


def test_rsvd_exact_when_rank_below_sketch():
    """rank(Theta) <= chi^A chi^B <= k: the sketch spans the range and the RSVD
    equals the SVD to rounding."""
    rng = np.random.default_rng(3)
    L = 8
    A = gaussian_mpo(rng, L, 2, 2, decay=True)
    B = gaussian_mpo(rng, L, 2, 3, decay=True)
    r0 = fit.fit_serial(A, B, 5, 4)
    r1 = fit.fit_serial(A, B, 5, 4, sketch_p=1)  # k = min(6, cap=6, n, m)
    assert min(r1.ks) < 16 and max(r1.ks) <= 6
    assert mpo.rel_diff(r1.C, r0.C) < 1e-10


def test_rsvd_error_statistics():
    """Halko-Martinsson-Tropp, Thm. 10.5 (the RSVD reference of Sec. 3.1):
    E||M - Q Q^T M||_F <= (1 + r/(p-1))^(1/2) tail_r; the rank-r truncation of
    Q Q^T M then adds at most tail_r.  Checked on the mean over 20 streams."""
    rng = np.random.default_rng(0)
    n, m, r, p = 60, 50, 10, 5
    U, _ = np.linalg.qr(rng.standard_normal((n, m)))
    V, _ = np.linalg.qr(rng.standard_normal((m, m)))
    s = np.exp(-np.arange(m) / 4.0)
    M = (U * s) @ V.T
    tail = np.sqrt(np.sum(s[r:] ** 2))
    errs = []
    for stream in range(20):
        f = fit.factorize(M, r, p, 10**9,
                          lambda mm, k, st=stream: gaussian_matrix(mm, k, 0, 0, st, 1))
        errs.append(np.linalg.norm(M - (f.U * f.S) @ f.Vt))
    bound = (1.0 + np.sqrt(1.0 + r / (p - 1.0))) * tail
    assert np.mean(errs) <= bound
    assert min(errs) >= tail * (1 - 1e-12)


def test_tau_truncation_rule():
    S = np.array([1.0, 0.5, 0.1, 0.01, 0.001])
    # threshold (tau/L)||S|| = 0.2 lies between the tails after r=2 (0.1005) and r=1 (0.51)
    assert fit.truncation_rank(S, 10, 10, tau=3 * 0.2 / np.linalg.norm(S), L=3) == 2
    assert fit.truncation_rank(S, 10, 10, tau=0.0, L=3) == 5
    assert fit.truncation_rank(S, 2, 10, tau=0.0, L=3) == 2


def test_even_odd_gauge_relations_and_fixed_point():
    """Exact-rank regime: after convergence a further even/odd sweep leaves C
    unchanged, and the inverse gauge relations hold."""
    A, B = make_pair(6, 2, 3, seed=4, decay=True)
    r1 = fit.fit_even_odd(A, B, 9, 3)
    r2 = fit.fit_even_odd(A, B, 9, 4)
    assert mpo.rel_diff(r2.C, r1.C) < 1e-12
    assert r1.n_guard == 0


def test_even_odd_approaches_serial():
    A, B = make_pair(10, 2, 6, seed=8, decay=True)
    e_s = mpo.fit_error_dense(A, B, fit.fit_serial(A, B, 12, 6).C)
    e_b = mpo.fit_error_dense(A, B, fit.fit_even_odd(A, B, 12, 8).C)
    assert e_b <= e_s * 1.05 + 1e-12


def _random_mpo(rng, L, d, dims):
    return [rng.standard_normal((dims[l], d, d, dims[l + 1])) / np.sqrt(dims[l + 1]) for l in range(L)]


@pytest.mark.parametrize("schedule", ["serial", "even_odd"])
def test_initial_guess_is_used_as_an_operator(schedule):
    """Alg. 5 takes the initial guess C as an input.  The fit sees it only
    through its right-orthogonal form, so a rescaled and gauge-transformed
    copy of the same operator gives the same result, while a different
    operator gives a different first sweep."""
    L, d = 7, 2
    A, B = make_pair(L, d, 5, seed=13, decay=True)
    rng = np.random.default_rng(14)
    dims = [1, 4, 9, 9, 9, 9, 4, 1]
    C0 = _random_mpo(rng, L, d, dims)
    Cg = [c.copy() for c in C0]
    Cg[0] *= 3.7
    for l in range(L - 1):
        chi = Cg[l].shape[3]
        G = rng.standard_normal((chi, chi)) + 3 * np.eye(chi)
        Cg[l] = np.tensordot(Cg[l], G, axes=(3, 0))
        Cg[l + 1] = np.tensordot(np.linalg.inv(G), Cg[l + 1], axes=(1, 0))
    run = fit.fit_serial if schedule == "serial" else fit.fit_even_odd
    r0 = run(A, B, 9, 1, C_init=C0)
    r1 = run(A, B, 9, 1, C_init=Cg)
    r2 = run(A, B, 9, 1)
    assert mpo.rel_diff(r1.C, r0.C) < 1e-10
    assert mpo.rel_diff(r2.C, r0.C) > 1e-6


def test_initial_guess_fixed_point():
    """Started from its own converged result, the plain fit stays there: the
    fit error does not rise and the operator moves by no more than the last
    sweeps did."""
    A, B = make_pair(7, 2, 5, seed=11, decay=True)
    r8 = fit.fit_serial(A, B, 8, 8)
    r9 = fit.fit_serial(A, B, 8, 9)
    r = fit.fit_serial(A, B, 8, 2, C_init=r8.C)
    e8 = mpo.fit_error_dense(A, B, r8.C)
    assert mpo.fit_error_dense(A, B, r.C) <= e8 + 1e-12
    assert mpo.rel_diff(r.C, r8.C) <= 10 * mpo.rel_diff(r9.C, r8.C) + 1e-12
