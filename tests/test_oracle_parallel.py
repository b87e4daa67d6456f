"""Pins of the site-canonical parallel fit (oracle/parallel.py, Sec. 4
variant II) against the exact product, dense projections and the canonical
form the merge promises."""
import numpy as np
import pytest

from oracle import fit, mpo, parallel
from synth import make_pair


def test_partition():
    for L in (4, 9, 16, 40):
        for n in (2, 4, 8):
            if L < 2 * n:
                with pytest.raises(ValueError):
                    parallel.partition(L, n)
                continue
            parts = parallel.partition(L, n)
            assert parts[0][0] == 0 and parts[-1][1] == L - 1
            assert all(b[0] == a[1] + 1 for a, b in zip(parts, parts[1:]))
            sizes = [e - s + 1 for s, e in parts]
            assert max(sizes) - min(sizes) <= 1 and min(sizes) >= 2
    with pytest.raises(ValueError):
        parallel.partition(12, 6)


@pytest.mark.parametrize("n_parts", [2, 4, 8])
@pytest.mark.parametrize("sketch_p", [-1, 3])
def test_exact_rank_regime_reproduces_the_product(n_parts, sketch_p):
    A, B = make_pair(16, 2, 3, seed=4, decay=True)
    r = parallel.fit_parallel_site(A, B, 9, 2, n_parts, sketch_p=sketch_p, seed=1)
    assert mpo.rel_diff(r.C, mpo.naive_product(A, B)) < 1e-12


def _isometries(C, m):
    """T[x, y, c] of cores 0..m-1 and V[c'', x, y] of cores m+2..L-1."""
    L, d = len(C), C[0].shape[1]
    T = np.ones((1, 1, 1))
    for j in range(m):
        T = np.einsum("xyc,csuC->xsyuC", T, C[j]).reshape(T.shape[0] * d, T.shape[1] * d, -1)
    V = np.ones((1, 1, 1))
    for j in range(L - 1, m + 1, -1):
        V = np.einsum("csuC,Cxy->csxuy", C[j], V).reshape(C[j].shape[0], d * V.shape[1], d * V.shape[2])
    return T, V


def _check_canonical(C, m):
    for j in range(m + 1):
        X = C[j].reshape(-1, C[j].shape[3])
        G = X.T @ X
        assert np.allclose(G, np.eye(G.shape[0]), atol=1e-12), j
    for j in range(m + 2, len(C)):
        X = C[j].reshape(C[j].shape[0], -1)
        G = X @ X.T
        assert np.allclose(G, np.eye(G.shape[0]), atol=1e-12), j


@pytest.mark.parametrize("n_parts", [2, 4])
@pytest.mark.parametrize("n_sets", [1, 2])
def test_merge_leaves_one_canonical_train_and_a_variational_last_update(n_parts, n_sets):
    """After the merge the train is site-canonical around the last merge
    boundary (sites m, m+1), and its two centre sites hold the best rank-r
    approximation (Eckart-Young, LAPACK's SVD) of A B projected densely onto
    the isometries on either side, i.e. the final update is the variational
    update of Alg. 3 with the merged environments."""
    L, d, chi = 8, 2, 4
    A, B = make_pair(L, d, 3, seed=6, decay=True)
    res = parallel.fit_parallel_site(A, B, chi, n_sets, n_parts)
    parts = parallel.partition(L, n_parts)
    m = parts[n_parts // 2 - 1][1]
    Cn = res.C_norm
    _check_canonical(Cn, m)
    A1, B1, nu, _ = fit._preprocess(A, B)
    P = mpo.dense(A1) @ mpo.dense(B1)
    T, V = _isometries(Cn, m)
    nl, nr = d ** m, d ** (L - m - 2)
    P8 = P.reshape(nl, d, d, nr, nl, d, d, nr)
    Th = np.einsum("xyc,xabXyefY,FXY->caebfF", T, P8, V)
    M = Th.reshape(Th.shape[0] * d * d, -1)
    W = np.tensordot(Cn[m], Cn[m + 1], axes=(3, 0)).reshape(M.shape)
    sv = np.linalg.svd(M, compute_uv=False)
    r = Cn[m].shape[3]
    assert r == min(chi, M.shape[0], M.shape[1], A1[m].shape[3] * B1[m].shape[3])
    tail = np.sqrt(np.sum(sv[r:] ** 2))
    assert abs(np.linalg.norm(M - W) - tail) <= 1e-10 * sv[0]
    # and the full train is that two-site tensor between the isometries
    D = mpo.dense(Cn)
    Dw = np.einsum("xyc,caebfF,FXY->xabXyefY", T, W.reshape(Th.shape), V).reshape(D.shape)
    assert np.allclose(D, Dw, atol=1e-12 * np.abs(D).max())


def test_error_bounded_below_and_close_to_the_serial_fit():
    """The merged fit's error is at least the dense tail at every cut
    (Eckart-Young) and, after several sets, within 1% of the serial fit's
    converged error on the same problem."""
    L, d, chi = 8, 2, 5
    A, B = make_pair(L, d, 4, seed=2, decay=True)
    D = mpo.dense(mpo.naive_product(A, B))
    res = parallel.fit_parallel_site(A, B, chi, 4, 4)
    err = np.linalg.norm(mpo.dense(res.C) - D)
    T = D.reshape([d] * (2 * L))
    for cut in range(1, L):
        rows = list(range(cut)) + [L + i for i in range(cut)]
        cols = [i for i in range(2 * L) if i not in rows]
        s = np.linalg.svd(np.transpose(T, rows + cols).reshape(d ** (2 * cut), -1), compute_uv=False)
        assert err >= np.sqrt(np.sum(s[chi:] ** 2)) * (1 - 1e-10)
    ser = fit.fit_serial(A, B, chi, 8)
    e_ser = np.linalg.norm(mpo.dense(ser.C) - D)
    assert err <= 1.01 * e_ser


def test_connection_keeps_both_gauges():
    """A set ends with the B|F connections: before the merge their two sites
    hold U S and S V^T (each side's centre), while the merge leaves U and
    S V^T there."""
    L = 8
    A, B = make_pair(L, 2, 3, seed=3, decay=True)
    parts = parallel.partition(L, 4)
    m = parts[1][1]
    raw = parallel.fit_parallel_site(A, B, 6, 1, 4, merge=False).C_norm
    U_S = raw[m].reshape(-1, raw[m].shape[3])
    S_Vt = raw[m + 1].reshape(raw[m + 1].shape[0], -1)
    # columns of U S are orthogonal with norms S, rows of S V^T orthogonal with the same norms
    G1, G2 = U_S.T @ U_S, S_Vt @ S_Vt.T
    assert np.allclose(G1, np.diag(np.diag(G1)), atol=1e-12 * G1.max())
    assert np.allclose(np.diag(G1), np.diag(G2), rtol=1e-10)
    merged = parallel.fit_parallel_site(A, B, 6, 1, 4).C_norm
    X = merged[m].reshape(-1, merged[m].shape[3])
    assert np.allclose(X.T @ X, np.eye(X.shape[1]), atol=1e-12)


@pytest.mark.parametrize("mistake", ["connection_one_env", "short_merge_qr"])
def test_pins_catch_planted_mistakes(monkeypatch, mistake):
    """A connection that rebuilds only the left environment, or a merge that
    leaves one site of the left group unorthogonalized, fails the pins."""
    orig_update, orig_qr = parallel._State.update, parallel._State.qr_sweep
    if mistake == "connection_one_env":
        monkeypatch.setattr(parallel._State, "update",
                            lambda self, i, mode, st: orig_update(self, i, "fwd" if mode == "both" else mode, st))
    else:
        monkeypatch.setattr(parallel._State, "qr_sweep",
                            lambda self, a, b: orig_qr(self, a, max(a, b - 1)))
    failed = False
    tests = [lambda n=n: test_exact_rank_regime_reproduces_the_product(n, -1) for n in (2, 4, 8)]
    tests += [lambda n=n, s=s: test_merge_leaves_one_canonical_train_and_a_variational_last_update(n, s)
              for n in (2, 4) for s in (1, 2)]
    for test in tests:
        try:
            test()
        except (AssertionError, ValueError):  # a wrong result, or shapes that no longer fit
            failed = True
    assert failed
