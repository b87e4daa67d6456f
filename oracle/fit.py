"""The variational fit of C ~ A B (Sec. 2.3) with the randomized SVD of
Sec. 3.1, in plain FP64 numpy.

Conventions (shared with the GPU path as definitions, not as code):
  * cores (left, out, in, right); C_l carries (c, s = A's out, u = B's in, c');
  * environments L_l[c, a, b] and R_l[c, a, b] are indexed by the C, A and B
    bonds at the open side (Sec. 2.3.3, Fig. envs); L_0 = R_{L+1} = [[[1]]];
  * the two-site tensor of bond l (Sec. 2.3.4, Fig. derivatives (c)) is the
    n x m matrix with rows (c, s1, u1) and columns (s2, u2, c'') row-major;
  * the randomized range finder sketches from the right, M Omega (Sec. 3.1);
  * r = min(chi_max, n, m, chi^A_l chi^B_l): chi_max is the bond cap of Alg. 3,
    n, m bound any SVD of M, and chi^A_l chi^B_l bounds the rank of A B across
    bond l, so no structurally zero singular value is kept; the sketch width
    is k = min(chi_max + p, n, m, chi^A_l chi^B_l) and k = min(n, m) means the
    plain SVD;
  * singular vectors are sign-fixed (largest-magnitude entry of each U column
    positive, Vt rows flipped along), Q of the sketch has R_jj >= 0;
  * of the r kept singular values, those at or below DROP * sigma_1 are
    dropped: the value and its singular vectors become zero and the bond keeps
    its size (zero padding).  Sec. 2.3.4 truncates by a bond cap and a
    tolerance; a relative cut at this level is the reading taken for values the
    GPU's FP64 factorization cannot resolve (its Gram eigenproblem resolves
    sigma down to about 1e-8 sigma_1), and in the inverse gauge it is the
    truncation before inversion that Sec. 2.3.1 allows;
  * tau > 0 truncation keeps the smallest r with
    (sum_{j>r} sigma_j^2)^(1/2) <= (tau / L) ||sigma||_2 (Sec. 2.3.4).

Pins (tests/test_oracle_fit.py): L = 2 reduces to the truncated SVD of the
dense product (Eckart-Young); the exact-rank regime reproduces A B; the error
is bounded below by the dense bond-unfolding tails and never increases from one
update to the next; forward updates leave left-orthogonal cores; the result is
invariant under gauge transforms of A and B; RSVD equals SVD when the sketch
spans the range; the batched inverse-gauge schedule keeps its gauge relations
and reaches the exact product in the exact-rank regime.
"""
from __future__ import annotations

from dataclasses import dataclass, field

import numpy as np

from . import canon
from .philox import gaussian_matrix

DROP = canon.INV_TRUNC


def ext_left(Lprev, A, B):
    """First two diagrams of Fig. envs: contract L_{l-1}[c, a, b] with A_l[a, s, t, a']
    and then with B_l[b, t, u, b'] into XL[c, s, u, a', b']."""
    T = np.tensordot(Lprev, A, axes=([1], [0]))           # [c, b, s, t, a']
    X = np.tensordot(T, B, axes=([1, 3], [0, 1]))          # [c, s, a', u, b']
    return X.transpose(0, 1, 3, 2, 4)


def ext_right(A, B, Rnext):
    """Mirror of ext_left: XR[a, b, s, u, c'] = sum A_l[a, s, t, a'] B_l[b, t, u, b']
    R_{l+1}[c', a', b']."""
    T = np.tensordot(A, Rnext, axes=([3], [1]))            # [a, s, t, c', b']
    X = np.tensordot(T, B, axes=([2, 4], [1, 3]))          # [a, s, c', b, u]
    return X.transpose(0, 3, 1, 4, 2)


def env_left(Lprev, C, A, B):
    """L_l[c', a', b'] = sum L_{l-1}[c, a, b] C_l[c, s, u, c'] A_l[a, s, t, a'] B_l[b, t, u, b']
    (Fig. envs, site-canonical form: no Y tensors; third diagram closes with C)."""
    return np.tensordot(C, ext_left(Lprev, A, B), axes=([0, 1, 2], [0, 1, 2]))


def env_right(Rnext, C, A, B):
    """R_l[c, a, b] = sum C_l[c, s, u, c'] A_l[a, s, t, a'] B_l[b, t, u, b'] R_{l+1}[c', a', b']."""
    X = np.tensordot(ext_right(A, B, Rnext), C, axes=([2, 3, 4], [1, 2, 3]))  # [a, b, c]
    return X.transpose(2, 0, 1)


def two_site_matrix(Lm, A1, B1, A2, B2, Rp):
    """The projected 6-leg tensor of Fig. derivatives (c)/(d):
    Theta[c,s1,u1,s2,u2,c''] = sum L[c,a,b] A1[a,s1,t1,a'] B1[b,t1,u1,b']
                                   A2[a',s2,t2,a''] B2[b',t2,u2,b''] R[c'',a'',b''],
    reshaped to (c s1 u1) x (s2 u2 c'')."""
    XL = ext_left(Lm, A1, B1)                              # [c, s1, u1, a', b']
    XR = ext_right(A2, B2, Rp)                             # [a', b', s2, u2, c'']
    T = np.tensordot(XL, XR, axes=([3, 4], [0, 1]))
    c, s1, u1, s2, u2, cc = T.shape
    return T.reshape(c * s1 * u1, s2 * u2 * cc)


@dataclass
class Factor:
    U: np.ndarray
    S: np.ndarray
    Vt: np.ndarray
    k: int
    gap: float
    n_guard: int
    sigma_all: np.ndarray = field(repr=False, default=None)


def truncation_rank(S, chi_max, cap, tau, L):
    r = min(chi_max, cap, len(S))
    if tau > 0.0:
        tot = float(np.sum(S ** 2))
        thr = (tau / L) ** 2 * tot
        tail = np.concatenate([np.cumsum((S ** 2)[::-1])[::-1][1:], [0.0]])
        ok = np.nonzero(tail <= thr)[0]
        r = min(r, int(ok[0]) + 1 if len(ok) else len(S))
    return max(r, 1)


def factorize(M, chi_max, sketch_p, rank_cap, omega, tau=0.0, L=1):
    """Truncated SVD of the two-site matrix (Alg. 3), optionally through the
    randomized range finder of Sec. 3.1: M Omega = Q R, Q^T M = U_b S V^T,
    U = Q U_b.  ``omega(m, k)`` returns the Gaussian test matrix."""
    n, m = M.shape
    kmax = min(n, m, rank_cap)
    k = min(n, m) if sketch_p < 0 else min(chi_max + sketch_p, kmax)
    if k >= min(n, m):
        U, S, Vt = np.linalg.svd(M, full_matrices=False)
        k = min(n, m)
    else:
        Om = omega(m, k)
        Q, _ = canon.qr_pos(M @ Om)
        Ub, S, Vt = np.linalg.svd(Q.T @ M, full_matrices=False)
        U = Q @ Ub
    r = truncation_rank(S, chi_max, kmax, tau, L)
    gap = float((S[r - 1] - S[r]) / S[r - 1]) if len(S) > r else 1.0
    U, Sr, Vt = U[:, :r], S[:r], Vt[:r]
    s = canon.sign_fix_columns(U)
    U, Vt = U * s[None, :], Vt * s[:, None]
    keep = Sr > DROP * Sr[0]
    U = np.where(keep[None, :], U, 0.0)
    Vt = np.where(keep[:, None], Vt, 0.0)
    Sr = np.where(keep, Sr, 0.0)
    n_drop = int(np.sum(~keep))
    return Factor(U, Sr, Vt, k, gap, n_drop, S)


@dataclass
class FitResult:
    C: list
    nu: float
    bond_dims: list
    min_gap: float
    n_guard: int
    ks: list
    records: list = field(default_factory=list)
    C_norm: list = field(default_factory=list)  # C before the norms are put back
    centre: int = 0  # 0-based site of the orthogonality centre (serial schedule)


def default_guess(A1, B1):
    """The initial guess when none is given (Sec. 2.3.5: one of the two
    inputs): A, whose legs (A's out, A's in) are C's (A's out, B's in) when
    A's and B's input legs agree, as for MPO-MPO products; otherwise B,
    whose legs are then C's: the MPO-MPS variant of Sec. 1, with B an MPS
    (an MPO with a unit input leg)."""
    if A1[0].shape[2] == B1[0].shape[2]:
        return A1
    if B1[0].shape[1] == A1[0].shape[1]:
        return B1
    raise ValueError("neither input has the product's physical legs: pass C_init")


def _preprocess(A, B):
    A1, nuA = canon.left_orthogonalize(A)
    B1, nuB = canon.left_orthogonalize(B)
    caps = [A1[l].shape[3] * B1[l].shape[3] for l in range(len(A1) - 1)]
    return A1, B1, nuA * nuB, caps


def fit_serial(A, B, chi_max, n_sweeps, sketch_p=-1, seed=0, pair=0, tau=0.0,
               on_update=None, C_init=None, first_sweep=0, first_bond=0, n_updates=None):
    """Alg. 5 with the site-canonical update of Alg. 3.

    Preprocessing left-orthogonalizes A and B and splits off their norms; the
    initial guess is (the preprocessed) A, right-orthogonalized; all right
    environments are precomputed; sweeps alternate forward and backward, each a
    pass of L-1 updates (the first backward update repeats the last forward
    bond with a fresh Omega).  Omega of sweep i at bond l (1-based) is the
    Philox stream (pair, i, l).  ``on_update(sweep, l, C_scaled)`` is called
    after each update.

    ``first_sweep`` = s resumes a fit as if s sweeps had been run: the sweep
    indices (direction and Philox stream) are s, s+1, ...; the initial guess
    is right-orthogonalized with all right environments precomputed when
    sweep s runs forward (s even), and left-orthogonalized with all left
    environments precomputed when it runs backward (s odd).  From the result
    of the first s sweeps, which is already in that form up to rounding, this
    continues the same fit.

    ``first_bond`` = b > 0 resumes inside sweep s after its first b updates:
    the guess is brought to the site-canonical form around the two sites of
    the next update (canon.mixed_canonical) and the environments of both
    sides are precomputed; the result of a fit's first b updates of sweep s
    is already in that form up to rounding.  ``n_updates`` stops after that
    many updates (None: the n_sweeps sweeps, the first one partial)."""
    L = len(A)
    A1, B1, nu, caps = _preprocess(A, B)
    guess = default_guess(A1, B1) if C_init is None else C_init
    ones = np.ones((1, 1, 1))
    Lenv = [None] * (L + 1)
    Renv = [None] * (L + 2)
    Lenv[0] = ones
    Renv[L + 1] = ones
    # environments use 1-based site labels: site l is index l-1 in the lists
    if first_bond > 0:
        if not 0 < first_bond < L - 1:
            raise ValueError("first_bond must be in 1 .. L-2")
        l0 = first_bond + 1 if first_sweep % 2 == 0 else L - 1 - first_bond  # 1-based bond
        C = canon.mixed_canonical(guess, l0 - 1)
        for l in range(1, l0):
            Lenv[l] = env_left(Lenv[l - 1], C[l - 1], A1[l - 1], B1[l - 1])
        for l in range(L, l0 + 1, -1):
            Renv[l] = env_right(Renv[l + 1], C[l - 1], A1[l - 1], B1[l - 1])
    elif first_sweep % 2 == 0:
        C = canon.right_orthogonalize(guess)
        for l in range(L, 2, -1):
            Renv[l] = env_right(Renv[l + 1], C[l - 1], A1[l - 1], B1[l - 1])
    else:
        C, cnorm = canon.left_orthogonalize(guess)
        C[-1] = C[-1] * cnorm
        for l in range(1, L - 1):
            Lenv[l] = env_left(Lenv[l - 1], C[l - 1], A1[l - 1], B1[l - 1])
    min_gap, n_guard, ks = 1.0, 0, []
    done = 0
    for sweep in range(first_sweep, first_sweep + n_sweeps):
        fwd = sweep % 2 == 0
        bonds = list(range(1, L) if fwd else range(L - 1, 0, -1))
        if sweep == first_sweep:
            bonds = bonds[first_bond:]
        for l in bonds:
            if n_updates is not None and done >= n_updates:
                break
            done += 1
            if fwd and l >= 2:
                Lenv[l - 1] = env_left(Lenv[l - 2], C[l - 2], A1[l - 2], B1[l - 2])
            if not fwd and l <= L - 2:
                Renv[l + 2] = env_right(Renv[l + 3], C[l + 1], A1[l + 1], B1[l + 1])
            M = two_site_matrix(Lenv[l - 1], A1[l - 1], B1[l - 1], A1[l], B1[l], Renv[l + 2])
            f = factorize(M, chi_max, sketch_p, caps[l - 1],
                          lambda m, k, l=l, sweep=sweep: gaussian_matrix(m, k, seed, pair, sweep, l),
                          tau, L)
            cl = C[l - 1].shape[0]
            cr = C[l].shape[3]
            d1, d2 = A1[l - 1].shape[1], B1[l - 1].shape[2]
            r = len(f.S)
            if fwd:
                C[l - 1] = f.U.reshape(cl, d1, d2, r)
                C[l] = (f.S[:, None] * f.Vt).reshape(r, d1, d2, cr)
            else:
                C[l - 1] = (f.U * f.S[None, :]).reshape(cl, d1, d2, r)
                C[l] = f.Vt.reshape(r, d1, d2, cr)
            min_gap = min(min_gap, f.gap)
            n_guard += f.n_guard
            ks.append(f.k)
            if on_update is not None:
                Cs = [c.copy() for c in C]
                Cs[0] = Cs[0] * nu
                on_update(sweep, l, Cs)
    out = [c.copy() for c in C]
    out[0] = out[0] * nu
    dims = [1] + [c.shape[3] for c in C]
    last = first_sweep + n_sweeps - 1
    centre = (L - 1 if last % 2 == 0 else 0) if n_sweeps > 0 else (0 if first_sweep % 2 == 0 else L - 1)
    if first_bond > 0 or n_updates is not None:
        centre = None  # a partial sweep leaves the centre inside the chain
    return FitResult(out, nu, dims, min_gap, n_guard, ks, C_norm=[c.copy() for c in C], centre=centre)


def fit_even_odd(A, B, chi_max, n_sweeps, sketch_p=-1, seed=0, pair=0, tau=0.0,
                 on_half_step=None, C_init=None, first_sweep=0, on_bond=None, first_half=0,
                 n_half_steps=None):
    """Single-device limit of the parallel fit in inverse canonical form
    (Sec. 4, Alg. 4 and Alg. 6 with every sub-TT two sites long): half-step q
    updates every bond l with l = 1 (mod 2) for q = 0 and l = 0 (mod 2) for
    q = 1, each independently from the environments as they stood at the
    half-step's start.  The initial guess (A, or C_init) is right-
    orthogonalized and brought to inverse canonical form.  An update sets
    Psi_l = U S, Psi_{l+1} = S V^T,
    Y_l = S^{-1} (Alg. 4) and rebuilds L_l from Psi_l Y_l = U and R_{l+1}
    from Y_l Psi_{l+1} = V^T.  Omega of half-step q of sweep i at bond l is the
    Philox stream (pair, 2 i + q, l); ``first_sweep`` offsets i.  The result
    is merged as C_l = Psi_l Y_l, C_L = Psi_L (Sec. 4.7).

    ``on_bond(sweep, q, l, M, factor, Psi0, Y0)`` sees every update: the
    two-site matrix, its factorization and the train (Psi, Y) as it stood at
    the half-step's start.  ``first_half`` = 1 starts with half-step 1 of
    sweep ``first_sweep`` (from the inverse canonical form of the guess and
    its environments); ``n_half_steps`` stops after that many half-steps."""
    L = len(A)
    A1, B1, nu, caps = _preprocess(A, B)
    C0 = canon.right_orthogonalize(default_guess(A1, B1) if C_init is None else C_init)
    # the guess acts only as an operator: its scale (it enters Lambda, hence
    # Y, of the bonds a half-step leaves alone) is set to one
    C0[0] = C0[0] / np.linalg.norm(C0[0])
    Psi, Y, n_guard = canon.inverse_canonical(C0)
    ones = np.ones((1, 1, 1))
    Lenv = [None] * (L + 1)
    Renv = [None] * (L + 2)
    Lenv[0] = ones
    Renv[L + 1] = ones
    for l in range(1, L - 1):  # L_l from C_l = Psi_l Y_l
        Cl = Psi[l - 1] * Y[l - 1][None, None, None, :]
        Lenv[l] = env_left(Lenv[l - 1], Cl, A1[l - 1], B1[l - 1])
    for l in range(L, 2, -1):  # R_l from Y_{l-1} Psi_l
        Cl = Y[l - 2][:, None, None, None] * Psi[l - 1]
        Renv[l] = env_right(Renv[l + 1], Cl, A1[l - 1], B1[l - 1])
    min_gap, ks = 1.0, []
    halves = 0
    for sweep in range(first_sweep, first_sweep + n_sweeps):
        for q in (0, 1):
            if sweep == first_sweep and q < first_half:
                continue
            if n_half_steps is not None and halves >= n_half_steps:
                break
            halves += 1
            bonds = [l for l in range(1, L) if (l % 2 == 1) == (q == 0)]
            if on_bond is not None:
                Psi0 = [p.copy() for p in Psi]
                Y0 = [y.copy() for y in Y]
            facs = {}
            for l in bonds:
                M = two_site_matrix(Lenv[l - 1], A1[l - 1], B1[l - 1], A1[l], B1[l], Renv[l + 2])
                facs[l] = factorize(
                    M, chi_max, sketch_p, caps[l - 1],
                    lambda m, k, l=l, st=2 * sweep + q: gaussian_matrix(m, k, seed, pair, st, l),
                    tau, L)
                if on_bond is not None:
                    on_bond(sweep, q, l, M, facs[l], Psi0, Y0)
            for l in bonds:
                f = facs[l]
                cl = Psi[l - 1].shape[0]
                cr = Psi[l].shape[3]
                d1, d2 = A1[l - 1].shape[1], B1[l - 1].shape[2]
                r = len(f.S)
                U, S, Vt, Yl, nt = canon.truncate_inverse(f.U, f.S, f.Vt)
                U4 = U.reshape(cl, d1, d2, r)
                V4 = Vt.reshape(r, d1, d2, cr)
                Psi[l - 1] = U4 * S[None, None, None, :]
                Psi[l] = S[:, None, None, None] * V4
                Y[l - 1] = Yl
                n_guard += nt
                min_gap = min(min_gap, f.gap)
                ks.append(f.k)
                if l <= L - 2:
                    Lenv[l] = env_left(Lenv[l - 1], U4, A1[l - 1], B1[l - 1])
                if l + 1 >= 3:
                    Renv[l + 1] = env_right(Renv[l + 2], V4, A1[l], B1[l])
            if on_half_step is not None:
                Cm = canon.merge_inverse_canonical(Psi, Y)
                Cm[0] = Cm[0] * nu
                on_half_step(sweep, q, Cm)
    C = canon.merge_inverse_canonical(Psi, Y)
    C[0] = C[0] * nu
    dims = [1] + [c.shape[3] for c in C]
    return FitResult(C, nu, dims, min_gap, n_guard, ks)


def fit_multi_pair(pairs, chi_maxes, n_sweeps, sketch_p=-1, seed=0):
    """Independent even/odd fits of several pairs; pair i uses Philox pair
    index i."""
    return [fit_even_odd(A, B, cm, n_sweeps, sketch_p, seed, pair=i)
            for i, ((A, B), cm) in enumerate(zip(pairs, chi_maxes))]
