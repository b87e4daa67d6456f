"""Kernel-level checks of libmpofit on the GPU against NumPy (float64)."""
import numpy as np
import pytest
import torch

from oracle.canon import qr_pos
from oracle.philox import gaussian_matrix
from paper_2606_23274_amd import _lib

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def hooks():
    from tests.gpu_util import Hooks
    return Hooks()


# (mode, ta, tb, tc): 0 = FP64, 1 = FP32; mode 2 = BF16 (FP32 accumulate)
KINDS = [(0, 0, 0, 0), (0, 1, 0, 0), (0, 0, 1, 0), (0, 1, 1, 0), (1, 1, 1, 1), (1, 0, 1, 1),
         (2, 1, 1, 1), (2, 0, 1, 1)]
TOL = {0: 1e-13, 1: 2e-5, 2: 2e-2}


@pytest.mark.parametrize("kind", KINDS)
@pytest.mark.parametrize("akc,bkc", [(1, 1), (1, 0), (0, 1), (0, 0)])
@pytest.mark.parametrize("M,N,K,tile,splits", [(64, 64, 64, 0, 1), (77, 45, 53, 0, 1),
                                               (200, 136, 300, 1, 1), (130, 70, 1000, 0, 4),
                                               (77, 45, 53, 2, 1), (130, 70, 1000, 2, 4),
                                               (77, 45, 53, 3, 1), (130, 70, 1000, 3, 4),
                                               (77, 45, 53, 4, 1), (144, 144, 300, 4, 2),
                                               (77, 45, 53, 5, 1), (144, 144, 512, 5, 1),
                                               (513, 145, 143, 5, 1)])
def test_gemm_against_numpy(hooks, kind, akc, bkc, M, N, K, tile, splits):
    from tests.gpu_util import dev, ptr
    mode, ta, tb, tc = kind
    if mode == 0 and tile in (1, 2):
        tile = 0  # (FP32/BF16 tiles)
    if mode != 0 and tile == 5:
        pytest.skip("FP64 tile")  # (3 and 4 serve every mode)
    rng = np.random.default_rng(M * 7 + N * 3 + K)
    A = rng.standard_normal((M, K))
    B = rng.standard_normal((K, N))
    Cin = rng.standard_normal((M, N))
    tA = torch.float64 if ta == 0 else torch.float32
    tB = torch.float64 if tb == 0 else torch.float32
    tC = torch.float64 if tc == 0 else torch.float32
    # storage: A K-contiguous = row-major M x K; M-contiguous = row-major K x M
    Ad = dev(A if akc else A.T.copy(), tA)
    Bd = dev(B.T.copy() if bkc else B, tB)
    Cd = dev(Cin, tC)
    lda = K if akc else M
    ldb = K if bkc else N
    Ar = Ad.double().cpu().numpy()
    Br = Bd.double().cpu().numpy()
    Aref = Ar if akc else Ar.T
    Bref = Br.T if bkc else Br
    ref = 0.5 * Aref @ Bref + Cd.double().cpu().numpy()
    st = hooks.lib.mpo_test_gemm(mode, ta, tb, tc, akc, bkc, tile, M, N, K, ptr(Ad), lda, ptr(Bd),
                                 ldb, ptr(Cd), N, 0.5, 1, splits, *hooks.args())
    _lib.check(st)
    got = Cd.double().cpu().numpy()
    err = np.linalg.norm(got - ref) / np.linalg.norm(ref)
    assert err < TOL[mode], err


# sizes on both sides of every register-kernel boundary (k = 32, 64, 96,
# 128, 144, 160, 176), of every panel width of the global-memory reduction
# (32 up to k = 290, 16 up to 570, then 8, unblocked beyond 1100) and of the
# one-wave twisted-vector kernel (k <= 1600; one thread per vector beyond)
@pytest.mark.parametrize("k,r", [(1, 1), (2, 2), (5, 3), (17, 17), (32, 20), (33, 33), (64, 64),
                                 (65, 40), (96, 96), (97, 90), (128, 128), (129, 100), (144, 128),
                                 (145, 145), (160, 128), (161, 150), (176, 176), (177, 160),
                                 (199, 199), (200, 150), (201, 180),
                                 (272, 256), (290, 256), (300, 200), (301, 250), (600, 100),
                                 (1200, 64), (1700, 48)])
def test_eig_against_numpy(hooks, k, r):
    from tests.gpu_util import dev, ptr
    rng = np.random.default_rng(k)
    X = rng.standard_normal((k, 3 * k)) * np.exp(-np.arange(3 * k) / 40.0)
    H = X @ X.T
    w, V = np.linalg.eigh(H)
    w, V = w[::-1][:r], V[:, ::-1][:, :r]
    Hd = dev(H)
    ev = torch.zeros(r, dtype=torch.float64, device="cuda:0")
    Z = torch.zeros((k, r), dtype=torch.float64, device="cuda:0")
    _lib.check(hooks.lib.mpo_test_eig(ptr(Hd), k, r, ptr(ev), ptr(Z), *hooks.args()))
    ev, Z = ev.cpu().numpy(), Z.cpu().numpy()
    nrm = np.abs(w).max()
    assert np.abs(ev - w).max() <= 1e-13 * nrm
    res = np.linalg.norm(H @ Z - Z * ev) / nrm
    assert res < 1e-12
    assert np.abs(Z.T @ Z - np.eye(r)).max() < 1e-9
    # same vectors up to sign
    assert np.abs(np.abs(np.sum(Z * V, axis=0)) - 1).max() < 1e-8


# spectra of either sign: the multisection's first round is geometric below a
# positive upper bound (with a point at 0 when the lower bound is negative)
# and uniform when the upper bound is not positive
@pytest.mark.parametrize("k,kind", [(40, "mixed"), (144, "mixed"), (40, "negative"), (144, "negative"),
                                    (300, "mixed")])
def test_eig_indefinite(hooks, k, kind):
    from tests.gpu_util import dev, ptr
    rng = np.random.default_rng(7 + k)
    Q, _ = np.linalg.qr(rng.standard_normal((k, k)))
    lam = np.linspace(-1.0, 1.0, k) if kind == "mixed" else -np.linspace(1.0, 10.0, k)
    H = (Q * lam) @ Q.T
    H = 0.5 * (H + H.T)
    r = k // 2
    w, V = np.linalg.eigh(H)
    w, V = w[::-1][:r], V[:, ::-1][:, :r]
    Hd = dev(H)
    ev = torch.zeros(r, dtype=torch.float64, device="cuda:0")
    Z = torch.zeros((k, r), dtype=torch.float64, device="cuda:0")
    _lib.check(hooks.lib.mpo_test_eig(ptr(Hd), k, r, ptr(ev), ptr(Z), *hooks.args()))
    ev, Z = ev.cpu().numpy(), Z.cpu().numpy()
    nrm = np.abs(lam).max()
    assert np.abs(ev - w).max() <= 1e-13 * nrm
    assert np.linalg.norm(H @ Z - Z * ev) / nrm < 1e-12
    assert np.abs(Z.T @ Z - np.eye(r)).max() < 1e-10
    assert np.abs(np.abs(np.sum(Z * V, axis=0)) - 1).max() < 1e-8


# several problems per launch: the batched configuration of the eigen
# kernels (eight-lane multisection once problems x eigenvalues >= 2048, the
# register or the global-memory tridiagonalization by size), including a
# partly filled last workgroup of eigenvalues
@pytest.mark.parametrize("n,k,r", [(3, 100, 90), (24, 90, 90), (16, 144, 128), (32, 272, 256)])
def test_eig_batch_against_numpy(hooks, n, k, r):
    from tests.gpu_util import dev, ptr
    Hs, refs = [], []
    for i in range(n):
        rng = np.random.default_rng(1000 * k + i)
        X = rng.standard_normal((k, 3 * k)) * np.exp(-np.arange(3 * k) / (40.0 + 3 * i))
        H = X @ X.T
        w, V = np.linalg.eigh(H)
        Hs.append(H)
        refs.append((w[::-1][:r], V[:, ::-1][:, :r]))
    Hd = dev(np.stack(Hs))
    ev = torch.zeros((n, r), dtype=torch.float64, device="cuda:0")
    Z = torch.zeros((n, k, r), dtype=torch.float64, device="cuda:0")
    _lib.check(hooks.lib.mpo_test_eig_batch(ptr(Hd), n, k, r, ptr(ev), ptr(Z), *hooks.args()))
    ev, Z = ev.cpu().numpy(), Z.cpu().numpy()
    for i, (w, V) in enumerate(refs):
        nrm = np.abs(w).max()
        assert np.abs(ev[i] - w).max() <= 1e-13 * nrm, i
        assert np.linalg.norm(Hs[i] @ Z[i] - Z[i] * ev[i]) / nrm < 1e-12, i
        assert np.abs(Z[i].T @ Z[i] - np.eye(r)).max() < 1e-9, i
        assert np.abs(np.abs(np.sum(Z[i] * V, axis=0)) - 1).max() < 1e-8, i


@pytest.mark.parametrize("n,k", [(40, 12), (90, 32), (200, 33), (300, 64), (400, 96), (400, 97),
                                 (500, 128), (512, 144), (520, 145), (600, 160), (600, 161),
                                 (600, 176), (600, 177), (300, 300), (1024, 272), (900, 321),
                                 (900, 352), (800, 360)])
def test_cholqr2_against_householder(hooks, n, k):
    from tests.gpu_util import dev, ptr
    rng = np.random.default_rng(n + k)
    X = rng.standard_normal((n, k)) @ np.diag(np.exp(-np.arange(k) / 30.0))
    Xd = dev(X)
    _lib.check(hooks.lib.mpo_test_cholqr(ptr(Xd), n, k, *hooks.args()))
    Q = Xd.cpu().numpy()
    Qref, _ = qr_pos(X)
    assert np.abs(Q.T @ Q - np.eye(k)).max() < 1e-13
    assert np.abs(Q - Qref).max() < 1e-9


@pytest.mark.parametrize("chi,dd,k,bond,stream,pair,seed",
                         [(16, 4, 24, 3, 0, 0, 0), (32, 4, 74, 7, 5, 2, 12345), (5, 9, 11, 1, 1, 1, 2**40)])
def test_omega_matches_oracle(hooks, chi, dd, k, bond, stream, pair, seed):
    from tests.gpu_util import ptr
    m = chi * dd
    out = torch.zeros((m, k), dtype=torch.float64, device="cuda:0")
    _lib.check(hooks.lib.mpo_test_omega(ptr(out), chi, dd, k, bond, stream, pair, seed, *hooks.args()))
    got = out.cpu().numpy()
    ref = gaussian_matrix(m, k, seed, pair, stream, bond)  # rows in (su, c'') order
    # the GPU stores row p = c''*dd + su for logical row i = su*chi + c''
    perm = np.array([(p % dd) * chi + p // dd for p in range(m)])
    assert np.abs(got - ref[perm]).max() < 1e-14 * np.abs(ref).max() * 8


# clustered spectra: runs of eigenvalues with relative gaps from exact
# degeneracy to 1e-6; the individual vectors of a tight run are not unique,
# so each run is checked through its invariant-subspace projector
@pytest.mark.parametrize("k,r", [(40, 30), (144, 128), (272, 256), (600, 200)])
@pytest.mark.parametrize("gap", [0.0, 1e-12, 1e-9, 1e-6])
def test_eig_clusters(hooks, k, r, gap):
    from tests.gpu_util import dev, ptr
    rng = np.random.default_rng(k + (0 if gap == 0 else int(-np.log10(gap))))
    lam = np.exp(-np.arange(k) / (k / 6.0))
    # three runs inside the kept range: 2, 3 and 4 (nearly) equal values
    runs = [(1, 2), (7, 3), (r // 2, 4)]
    for start, size in runs:
        lam[start:start + size] = lam[start] * (1.0 - gap * np.arange(size))
    lam = np.sort(lam)[::-1]
    Q, _ = np.linalg.qr(rng.standard_normal((k, k)))
    H = (Q * lam) @ Q.T
    H = 0.5 * (H + H.T)
    Hd = dev(H)
    ev = torch.zeros(r, dtype=torch.float64, device="cuda:0")
    Z = torch.zeros((k, r), dtype=torch.float64, device="cuda:0")
    _lib.check(hooks.lib.mpo_test_eig(ptr(Hd), k, r, ptr(ev), ptr(Z), *hooks.args()))
    ev, Z = ev.cpu().numpy(), Z.cpu().numpy()
    w = np.linalg.eigvalsh(H)[::-1][:r]
    nrm = lam.max()
    assert np.abs(ev - w).max() <= 1e-13 * nrm
    assert np.linalg.norm(H @ Z - Z * ev) / nrm < 1e-12
    assert np.abs(Z.T @ Z - np.eye(r)).max() < 1e-10
    # the span of each run (and of everything up to r) against the exact one
    for start, size in runs:
        idx = [i for i in range(r) if abs(lam[i] - lam[start]) <= 1e-5 * lam[start]]
        idx = list(range(min(idx), max(idx) + 1))
        Pz = Z[:, idx] @ Z[:, idx].T
        w_all, V_all = np.linalg.eigh(H)
        sel = np.abs(w_all - lam[start]) <= 1e-5 * lam[start]
        Pv = V_all[:, sel] @ V_all[:, sel].T
        assert sel.sum() == len(idx)
        assert np.abs(Pz - Pv).max() < 1e-10, (start, size)


@pytest.mark.parametrize("n,k,rank", [(300, 40, 25), (600, 144, 100), (1024, 272, 200)])
def test_cholqr_rank_revealing(hooks, n, k, rank):
    """A rank-deficient sketch (the range finder of a two-site matrix of lower
    rank than the sketch width): the rank-revealing passes leave zero columns
    for the dependent directions and an orthonormal basis of the range in the
    others (checked with the test hook's CholeskyQR2 in rank-revealing mode)."""
    from tests.gpu_util import dev, ptr
    rng = np.random.default_rng(n + k + rank)
    X = rng.standard_normal((n, rank)) @ rng.standard_normal((rank, k))
    Xd = dev(X)
    _lib.check(hooks.lib.mpo_test_cholqr_rr(ptr(Xd), n, k, *hooks.args()))
    Q = Xd.cpu().numpy()
    norms = np.linalg.norm(Q, axis=0)
    nz = norms > 0.5
    assert nz.sum() == rank
    assert np.all(norms[~nz] < 1e-12)
    Qn = Q[:, nz]
    assert np.abs(Qn.T @ Qn - np.eye(rank)).max() < 1e-12
    # same range as X
    U, _, _ = np.linalg.svd(X, full_matrices=False)
    U = U[:, :rank]
    assert np.abs(Qn @ Qn.T - U @ U.T).max() < 1e-10


@pytest.mark.parametrize("q", [1, 7, 64, 130])
def test_jacobi_against_lapack(hooks, q):
    """One-sided Jacobi SVD of a row-graded matrix (rows scaled over ten
    decades, the shape of the canonical forms' R factors) against LAPACK's
    preconditioned Jacobi SVD (dgejsv, relatively accurate for such
    matrices): singular values to 1e-12 relative, left singular vectors to
    1e-12 over the relative gap to the neighbouring values."""
    import scipy.linalg.lapack as lapack
    from tests.gpu_util import dev, ptr
    rng = np.random.default_rng(q)
    W = np.logspace(0, -10, q)[:, None] * rng.standard_normal((q, q))
    sva, U, _, work, _, info = lapack.dgejsv(W, joba=2, jobu=0, jobv=0, jobr=1, jobt=0, jobp=0)
    assert info == 0
    S = sva * (work[0] / work[1])
    Wd = dev(W)
    Ud = torch.zeros((q, q), dtype=torch.float64, device="cuda:0")
    Sd = torch.zeros(q, dtype=torch.float64, device="cuda:0")
    _lib.check(hooks.lib.mpo_test_jacobi(ptr(Wd), q, ptr(Ud), ptr(Sd), *hooks.args()))
    Ug, Sg = Ud.cpu().numpy(), Sd.cpu().numpy()
    assert np.max(np.abs(Sg - S) / S) < 1e-12
    rel = np.abs(np.diff(S)) / S[1:] if q > 1 else np.zeros(0)
    gap = np.minimum(np.r_[rel, np.inf], np.r_[np.inf, rel]) if q > 1 else np.ones(1)
    sg = np.sign(np.sum(Ug * U[:, :q], axis=0))
    dist = np.linalg.norm(Ug * sg[None, :] - U[:, :q], axis=0)
    assert np.all(dist <= 1e-12 / np.minimum(gap, 1.0)), (dist.max(), gap.min())
