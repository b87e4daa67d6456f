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


def _brute_rank(S, tau, L):
    """Smallest count c >= 1 whose discarded tail meets the Sec. 2.3.4 rule,
    by trying every c in order (pure Python sums)."""
    tot = sum(float(x) * float(x) for x in S)
    for c in range(1, len(S) + 1):
        tail = sum(float(x) * float(x) for x in S[c:])
        if tail ** 0.5 <= (tau / L) * tot ** 0.5:
            return c
    return len(S)


def test_tau_rule_against_brute_force():
    rng = np.random.default_rng(21)
    for _ in range(200):
        n = int(rng.integers(1, 30))
        S = np.sort(np.exp(rng.uniform(-12, 0, n)))[::-1]
        tau, L = float(10 ** rng.uniform(-6, 0.5)), int(rng.integers(2, 50))
        assert fit.truncation_rank(S, 10 ** 6, 10 ** 6, tau, L) == _brute_rank(S, tau, L)
        assert fit.truncation_rank(S, 3, 10 ** 6, tau, L) == min(3, _brute_rank(S, tau, L))


@pytest.mark.parametrize("schedule", ["serial", "even_odd"])
def test_tau_L2_is_tolerance_truncated_svd(schedule):
    """L = 2: the tau fit is the SVD of the d^2 x d^2 unfolding cut at the
    smallest rank whose tail is at most (tau / 2) ||A B||_F (Eckart-Young
    with the rank of the rule, from LAPACK's singular values)."""
    rng = np.random.default_rng(5)
    A = gaussian_mpo(rng, 2, 3, 3, decay=True)
    B = gaussian_mpo(rng, 2, 3, 3, decay=True)
    P = mpo.dense(A) @ mpo.dense(B)
    sv = np.linalg.svd(_dense_unfold(P, 2, 3, 1), compute_uv=False)
    nP = np.linalg.norm(P)
    for c_want in (1, 2, 4):
        # a tolerance halfway (in log) between the tails of c_want and c_want - 1
        hi = np.sqrt(np.sum(sv[c_want - 1:] ** 2)) if c_want > 1 else nP
        lo = np.sqrt(np.sum(sv[c_want:] ** 2))
        tau = 2.0 * np.sqrt(lo * hi) / nP
        run = fit.fit_serial if schedule == "serial" else fit.fit_even_odd
        res = run(A, B, 9, 2, tau=tau)
        assert res.bond_dims == [1, c_want, 1]
        err = np.linalg.norm(P - mpo.dense(res.C))
        assert abs(err - lo) < 1e-12 * nP


@pytest.mark.parametrize("schedule", ["serial", "even_odd"])
def test_tau_below_every_tail_is_the_fixed_cap_fit(schedule):
    A, B = make_pair(6, 2, 4, seed=7, decay=True)
    run = fit.fit_serial if schedule == "serial" else fit.fit_even_odd
    r0 = run(A, B, 6, 2)
    r1 = run(A, B, 6, 2, tau=1e-300)
    assert r1.bond_dims == r0.bond_dims
    for a, b in zip(r0.C, r1.C):
        assert np.array_equal(a, b)


def test_tau_first_update_rank_and_error():
    """The first update (bond 1 from the same environments for every tau)
    keeps the rule's count of the two-site matrix's singular values, and
    what it discards is at most (tau / L) of that matrix's norm."""
    A, B = make_pair(8, 2, 6, seed=3, decay=True)
    A1, B1, _, caps = fit._preprocess(A, B)
    C = canon.right_orthogonalize(A1)
    R = [None] * 10
    R[9] = np.ones((1, 1, 1))
    for l in range(8, 2, -1):
        R[l] = fit.env_right(R[l + 1], C[l - 1], A1[l - 1], B1[l - 1])
    M = fit.two_site_matrix(np.ones((1, 1, 1)), A1[0], B1[0], A1[1], B1[1], R[3])
    sv = np.linalg.svd(M, compute_uv=False)
    prev = None
    ranks = []
    for tau in (0.0, 1.0, 2.0, 4.0):
        seen = {}
        fit.fit_serial(A, B, 12, 1, tau=tau, n_updates=1,
                       on_update=lambda sw, l, Cs: seen.setdefault("r", Cs[0].shape[3]))
        r = seen["r"]
        assert r == min(fit.truncation_rank(sv, 12, caps[0], tau, 8), len(sv))
        if tau > 0:
            assert np.sqrt(np.sum(sv[r:] ** 2)) <= tau / 8 * np.linalg.norm(sv) * (1 + 1e-12)
        if prev is not None:
            assert r <= prev
        prev = r
        ranks.append(r)
    assert ranks[0] > ranks[-1]  # the rule cuts below the cap here


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


# ---------------------------------------------------------------- resume
@pytest.mark.parametrize("sketch_p", [-1, 3])
@pytest.mark.parametrize("s", [1, 2, 3])
def test_resume_continues_the_fit(s, sketch_p):
    """first_sweep = s started from the result of s sweeps reproduces sweep
    s + 1 of the uninterrupted fit (Alg. 5): after a forward sweep C is left
    canonical and after a backward one right canonical, so the QR / RQ
    sweep of the resumed start leaves every core in place (R = I), and the
    Philox stream of sweep s is drawn again."""
    A, B = make_pair(9, 2, 4, seed=21, decay=True)
    rs = fit.fit_serial(A, B, 6, s, sketch_p=sketch_p, seed=5)
    r_cont = fit.fit_serial(A, B, 6, s + 1, sketch_p=sketch_p, seed=5)
    r_res = fit.fit_serial(A, B, 6, 1, sketch_p=sketch_p, seed=5, C_init=rs.C, first_sweep=s)
    assert r_res.bond_dims == r_cont.bond_dims
    assert mpo.rel_diff(r_res.C, r_cont.C) < 1e-12
    assert r_res.centre == r_cont.centre


def test_resume_stream_matters():
    """The resumed sweep draws the Philox stream of its own index: the same
    start with another first_sweep of the same direction differs."""
    A, B = make_pair(9, 2, 4, seed=21, decay=True)
    rs = fit.fit_serial(A, B, 6, 2, sketch_p=3, seed=5)
    r2 = fit.fit_serial(A, B, 6, 1, sketch_p=3, seed=5, C_init=rs.C, first_sweep=2)
    r4 = fit.fit_serial(A, B, 6, 1, sketch_p=3, seed=5, C_init=rs.C, first_sweep=4)
    assert mpo.rel_diff(r2.C, r4.C) > 1e-8


# ---------------------------------------------------------------- even/odd pins
def _left_isometry(cores, l, d):
    """T[x_<l, y_<l, c] of the first l-1 cores (1-based bond l)."""
    T = np.ones((1, 1, 1))
    for j in range(l - 1):
        c = cores[j]
        T = np.einsum("xyc,csuC->xsyuC", T, c).reshape(T.shape[0] * d, T.shape[1] * d, c.shape[3])
    return T


def _right_isometry(cores, l, d):
    """V[c'', x_>l+1, y_>l+1] of the cores after site l+1 (1-based bond l)."""
    L = len(cores)
    V = np.ones((1, 1, 1))
    for j in range(L - 1, l, -1):  # 0-based sites l+1 .. L-1 = 1-based l+2 .. L
        c = cores[j]
        V = np.einsum("csuC,Cxy->csxuy", c, V).reshape(c.shape[0], d * V.shape[1], d * V.shape[2])
    return V


def _even_odd_dense_check(A, B, chi_max, n_sweeps, sketch_p=-1, C_init=None, first_half=0):
    """Every update of fit_even_odd against brute force.

    Half-step h = 2 sweep + q updates the bonds of one parity from the
    environments as they stood at its start, and each update rebuilds L_l
    from U and R_{l+1} from V^T (Alg. 4, Sec. 4 with two-site sub-TTs).  So
    the left environment of bond l at half-step h is made of a light cone of
    isometries: site j < l contributes the U of bond j's update at half-step
    h - (l - j), or the initial train's Psi_j Y_j if that index is negative;
    the right environment mirrors this with the V^T of bond j - 1 for sites
    j > l + 1 (or Y_{j-1} Psi_j of the initial train).  Checked: Theta_l is
    the dense product A B (preprocessed) projected onto those isometries;
    without the sketch S_l is the leading part of that matrix's singular
    values (Eckart-Young, Alg. 3); U and V^T have orthonormal columns / rows
    (Psi_l Y_l left and Y_l Psi_{l+1} right orthogonal, Sec. 2.3.1)."""
    L, d = len(A), A[0].shape[1]
    A1, B1, _, _ = fit._preprocess(A, B)
    P = mpo.dense(A1) @ mpo.dense(B1)
    hist = {}  # (h, l) -> (U4, V4), h counted from the first half-step run
    init = {}
    seen = []
    h0 = []

    def left_core(j, h):  # 1-based site j, as seen by a bond right of it at half-step h
        if h < 0:
            return init["Psi"][j - 1] * init["Y"][j - 1][None, None, None, :]
        return hist[(h, j)][0]

    def right_core(j, h):  # 1-based site j, seen by a bond left of it
        if h < 0:
            return init["Y"][j - 2][:, None, None, None] * init["Psi"][j - 1]
        return hist[(h, j - 1)][1]

    def on_bond(sweep, q, l, M, f, Psi0, Y0):
        if not h0:
            h0.append(2 * sweep + q)
        h = 2 * sweep + q - h0[0]
        if not init:
            init["Psi"] = [p.copy() for p in Psi0]
            init["Y"] = [y.copy() for y in Y0]
            # the initial train: inverse canonical form of the right-
            # orthogonalized A (Sec. 2.3.1) with the same operator
            for j in range(L - 1):
                X = (Psi0[j] * Y0[j][None, None, None, :]).reshape(-1, Y0[j].size)
                W = (Y0[j][:, None, None, None] * Psi0[j + 1]).reshape(Y0[j].size, -1)
                kj = Y0[j] != 0
                assert np.abs(X[:, kj].T @ X[:, kj] - np.eye(kj.sum())).max() < 1e-12
                assert np.abs(W[kj] @ W[kj].T - np.eye(kj.sum())).max() < 1e-12
            Cm = canon.merge_inverse_canonical(Psi0, Y0)
            D0 = mpo.dense(A1 if C_init is None else C_init)
            D0 = D0 / np.linalg.norm(D0)  # the guess is taken at unit norm
            assert np.abs(mpo.dense(Cm) - D0).max() <= 1e-12 * np.abs(D0).max()
        Cl = [left_core(j, h - (l - j)) for j in range(1, l)]
        Cr = [None] * L
        for j in range(l + 2, L + 1):
            Cr[j - 1] = right_core(j, h - (j - 1 - l))
        T = _left_isometry(Cl, l, d)
        V = _right_isometry(Cr, l, d)
        nl, nr = d ** (l - 1), d ** (L - l - 1)
        P8 = P.reshape(nl, d, d, nr, nl, d, d, nr)  # x<, s1, s2, x>, y<, u1, u2, y>
        Th = np.einsum("xyc,xabXyefY,FXY->caebfF", T, P8, V).reshape(M.shape)
        scale = np.abs(Th).max()
        assert np.abs(M - Th).max() <= 1e-12 * scale, (sweep, q, l)
        if sketch_p < 0:
            sv = np.linalg.svd(Th, compute_uv=False)
            r = len(f.S)
            kept = f.S > 0
            assert np.allclose(f.S[kept], sv[:r][kept], rtol=1e-12, atol=1e-13 * sv[0]), (sweep, q, l)
        kept = f.S > 0
        Uk = f.U[:, kept]
        Vk = f.Vt[kept]
        assert np.abs(Uk.T @ Uk - np.eye(Uk.shape[1])).max() < 1e-12
        assert np.abs(Vk @ Vk.T - np.eye(Vk.shape[0])).max() < 1e-12
        cl = Cl[-1].shape[3] if Cl else 1
        cr = Cr[l + 1].shape[0] if l + 1 < L else 1
        r = len(f.S)
        # the environments of later half-steps use these isometries (the
        # dropped triplets are already zero)
        hist[(h, l)] = (f.U.reshape(cl, d, d, r), f.Vt.reshape(r, d, d, cr))
        seen.append((sweep, q, l))

    res = fit.fit_even_odd(A, B, chi_max, n_sweeps, sketch_p=sketch_p, on_bond=on_bond, C_init=C_init,
                           first_half=first_half)
    n_bonds = n_sweeps * (L - 1) - (len([l for l in range(1, L) if l % 2 == 1]) if first_half else 0)
    assert len(seen) == n_bonds
    return res


@pytest.mark.parametrize("sketch_p", [-1, 2])
@pytest.mark.parametrize("L,chi,chi_max", [(6, 3, 4), (7, 3, 5), (7, 2, 3)])
def test_even_odd_half_steps_against_dense_projection(L, chi, chi_max, sketch_p):
    """Truncating regime (chi_C below the structural rank chi^2): every bond of
    both half-steps of three sweeps checked against the dense product."""
    A, B = make_pair(L, 2, chi, seed=31 + L + chi, decay=True)
    res = _even_odd_dense_check(A, B, chi_max, 3, sketch_p)
    P = mpo.dense(A) @ mpo.dense(B)
    assert mpo.fit_error_dense(A, B, res.C) > 1e-6  # truncation really happens


def test_even_odd_dense_pin_catches_planted_mistakes(monkeypatch):
    """The dense half-step pin fails for the two plausible slips in the
    inverse-gauge bookkeeping: environments built from Psi = U S instead of
    U, and the bond matrix Y = S instead of S^-1."""
    A, B = make_pair(6, 2, 3, seed=40, decay=True)
    orig = fit.canon.truncate_inverse

    def env_from_psi(U, S, Vt, thresh=canon.INV_TRUNC):
        U2, S2, V2, Y, n = orig(U, S, Vt, thresh)
        return U2 * S2[None, :], S2, V2, Y, n

    def y_not_inverted(U, S, Vt, thresh=canon.INV_TRUNC):
        U2, S2, V2, Y, n = orig(U, S, Vt, thresh)
        return U2, S2, V2, S2.copy(), n

    for plant in (env_from_psi, y_not_inverted):
        monkeypatch.setattr(fit.canon, "truncate_inverse", plant)
        with pytest.raises(AssertionError):
            _even_odd_dense_check(A, B, 4, 2)
        monkeypatch.setattr(fit.canon, "truncate_inverse", orig)
    _even_odd_dense_check(A, B, 4, 2)


def test_drop_rule_on_rank_deficient_product():
    """A B with bond rank below chi_C at interior bonds (B the identity MPO
    on a doubled bond, so A B = A but chi^A chi^B = 2 chi^A): the singular
    values beyond A's rank are dropped (zero padding), the fit reproduces A
    exactly in both schedules, and the count of dropped values is reported."""
    L, d, chi = 6, 2, 3
    rng = np.random.default_rng(50)
    A = gaussian_mpo(rng, L, d, chi)
    Bid = []
    for l in range(L):
        cl = 1 if l == 0 else 2
        cr = 1 if l == L - 1 else 2
        core = np.zeros((cl, d, d, cr))
        for i in range(d):
            core[0, i, i, 0] = 1.0
        Bid.append(core)
    for run in (fit.fit_serial, fit.fit_even_odd):
        res = run(A, Bid, 6, 3)
        assert mpo.fit_error_dense(A, Bid, res.C) < 1e-12
        assert res.n_guard > 0


@pytest.mark.parametrize("s,b", [(0, 1), (0, 4), (1, 2), (1, 6), (2, 3)])
@pytest.mark.parametrize("sketch_p", [-1, 3])
def test_resume_at_bond_continues_the_fit(s, b, sketch_p):
    """first_bond = b inside sweep s, started from the fit's state after its
    first b updates of that sweep: one update reproduces the uninterrupted
    fit's next state (the mixed-canonical start leaves every orthogonal core
    in place, R = I), and so does running to the end of the sweep."""
    A, B = make_pair(9, 2, 4, seed=23, decay=True)
    states = []

    def on_update(sweep, l, Cs):
        states.append((sweep, l, [c.copy() for c in Cs]))

    fit.fit_serial(A, B, 6, s + 1, sketch_p=sketch_p, seed=5, on_update=on_update)
    in_sweep = [st for st in states if st[0] == s]
    before, after = in_sweep[b - 1][2], in_sweep[b][2]
    r1 = fit.fit_serial(A, B, 6, 1, sketch_p=sketch_p, seed=5, C_init=before, first_sweep=s, first_bond=b,
                        n_updates=1)
    assert mpo.bond_dims(r1.C) == mpo.bond_dims(after)
    assert mpo.rel_diff(r1.C, after) < 1e-12
    r_end = fit.fit_serial(A, B, 6, 1, sketch_p=sketch_p, seed=5, C_init=before, first_sweep=s, first_bond=b)
    assert mpo.rel_diff(r_end.C, in_sweep[-1][2]) < 1e-12


@pytest.mark.parametrize("sketch_p", [-1, 2])
def test_even_odd_first_half_against_dense_projection(sketch_p):
    """first_half = 1 from a given guess: half-step 1 runs first, from the
    guess's inverse canonical form, and every update still equals the dense
    projection onto its light-cone isometries."""
    A, B = make_pair(7, 2, 3, seed=41, decay=True)
    G = fit.fit_even_odd(A, B, 5, 1, sketch_p=sketch_p, n_half_steps=1).C
    _even_odd_dense_check(A, B, 5, 2, sketch_p, C_init=G, first_half=1)
