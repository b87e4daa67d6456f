"""Parallel fit in site-canonical form (Sec. 4, variant II: sub-TTs swept in
parallel, connections between their orthogonality centres updated, binary
merging at the end), in the single-device form where every sub-TT is one
group of a batched update.  Test infrastructure: only tests/, the package's
smoke check and bench.py's CPU baseline use it.

Readings (the paper describes the scheme in prose; where it is silent the
choices below are taken, by the GPU path too):

  * Partition: N_p (a power of two, >= 2) contiguous sub-TTs as equal as
    possible, the first ones one site longer; each at least two sites.
    Sub-TT n is "odd" in the paper's 1-based count when n (0-based) is even:
    it sweeps forward first ("F"); the others sweep backward first ("B").
  * Initialization: every sub-TT starts from the guess (preprocessed A, or
    C_init) in the mixed canonical form centred on it, so that its
    environments are isometric, as the paper's identities or random
    isometries at the boundaries are: the guess right-orthogonalized, then
    left-orthogonalized (QR sweep, carried to the last site), which gives
    every left environment, then right-orthogonalized again (RQ sweep),
    which gives every right environment.  The local problems are then those
    of the serial fit at the same positions; environments built on the
    guess's own (non-isometric) cores instead would weight each local
    problem by the guess's Schmidt values.
  * One set of local full sweeps (``n_sets`` of them), phases 0..3:
      0: F sub-TTs sweep forward over their inner bonds, B sub-TTs backward
         (each update the serial site-canonical update of Alg. 3);
      1: the F|B connections (last site of an F, first of the next B) are
         updated with the environments both sides just built;
      2: F backward, B forward;
      3: the B|F connections.
    A connection update assigns C_l = U S (the centre of the sub-TT on its
    left, whose next sweep runs backward) and C_{l+1} = S V^T (the centre of
    the one on its right), and rebuilds both L_{l+1} (from U) and R_{l+1}
    (from V^T): each sub-TT keeps its own gauge, as the paper notes.
  * Merge: phase 0 once more, then level 1 updates every F|B connection
    with forward assignment (C_l = U, C_{l+1} = S V^T), which makes each
    pair of sub-TTs one consistent site-canonical train; level t >= 2
    merges adjacent groups of 2^(t-1) sub-TTs: the left group's centre is
    moved to its last site by QR and the environments rebuilt up to the
    boundary, the right group's centre to its first site by RQ and the
    environments rebuilt from its end, then one forward update at the
    boundary.  The result is one site-canonical train.
  * Omega of an update at bond l (1-based) in phase q of set t is the
    Philox stream (pair, 4 t + q, l); the merge uses 4 n_sets (its local
    sweeps) and 4 n_sets + level.
"""
from __future__ import annotations

from dataclasses import dataclass

import numpy as np

from . import canon
from .fit import _preprocess, env_left, env_right, factorize, two_site_matrix
from .philox import gaussian_matrix


def partition(L: int, n_parts: int):
    """[(first, last)] 0-based inclusive site ranges of the sub-TTs."""
    if n_parts < 2 or n_parts & (n_parts - 1):
        raise ValueError("n_parts must be a power of two >= 2")
    if L < 2 * n_parts:
        raise ValueError("every sub-TT needs two sites")
    base, extra = divmod(L, n_parts)
    out, s = [], 0
    for n in range(n_parts):
        ln = base + (1 if n < extra else 0)
        out.append((s, s + ln - 1))
        s += ln
    return out


@dataclass
class ParallelResult:
    C: list
    nu: float
    bond_dims: list
    C_norm: list


class _State:
    """Cores (0-based sites), environments by bond index b (0..L): Lb[b]
    covers sites 0..b-1 and Rb[b] sites b..L-1."""

    def __init__(self, A1, B1, C, chi_max, sketch_p, seed, pair, caps, tau):
        self.A, self.B, self.C = A1, B1, C
        self.L = len(C)
        self.chi_max, self.p, self.seed, self.pair = chi_max, sketch_p, seed, pair
        self.caps, self.tau = caps, tau
        self.Lb = [None] * (self.L + 1)
        self.Rb = [None] * (self.L + 1)
        self.Lb[0] = np.ones((1, 1, 1))
        self.Rb[self.L] = np.ones((1, 1, 1))

    def left_env(self, b):
        """Lb[b + 1] from Lb[b] and core b."""
        self.Lb[b + 1] = env_left(self.Lb[b], self.C[b], self.A[b], self.B[b])

    def right_env(self, b):
        """Rb[b] from Rb[b + 1] and core b."""
        self.Rb[b] = env_right(self.Rb[b + 1], self.C[b], self.A[b], self.B[b])

    def factor(self, i, stream):
        """Two-site matrix of sites i, i+1 from Lb[i], Rb[i+2], and its
        truncated factorization."""
        M = two_site_matrix(self.Lb[i], self.A[i], self.B[i], self.A[i + 1], self.B[i + 1], self.Rb[i + 2])
        return factorize(M, self.chi_max, self.p, self.caps[i],
                         lambda m, k, l=i + 1: gaussian_matrix(m, k, self.seed, self.pair, stream, l),
                         self.tau, self.L)

    def update(self, i, mode, stream):
        """mode 'fwd' (Alg. 3 forward), 'bwd' (backward) or 'both' (a
        connection: U S | S V^T and both environments)."""
        f = self.factor(i, stream)
        cl, cr = self.C[i].shape[0], self.C[i + 1].shape[3]
        d1, d2 = self.A[i].shape[1], self.B[i].shape[2]
        r = len(f.S)
        U4 = f.U.reshape(cl, d1, d2, r)
        V4 = f.Vt.reshape(r, d1, d2, cr)
        US = (f.U * f.S[None, :]).reshape(cl, d1, d2, r)
        SV = (f.S[:, None] * f.Vt).reshape(r, d1, d2, cr)
        if mode == "fwd":
            self.C[i], self.C[i + 1] = U4, SV
            self.left_env(i)
        elif mode == "bwd":
            self.C[i], self.C[i + 1] = US, V4
            self.right_env(i + 1)
        else:
            self.C[i], self.C[i + 1] = U4, V4
            self.left_env(i)
            self.right_env(i + 1)
            self.C[i], self.C[i + 1] = US, SV

    def qr_sweep(self, first, last):
        """Left-orthogonalize sites first..last-1, carrying into `last`."""
        for i in range(first, last):
            cl, d1, d2, cr = self.C[i].shape
            X = self.C[i].reshape(cl * d1 * d2, cr)
            if X.shape[0] >= X.shape[1]:
                Q, R = canon.qr_pos(X)
            else:
                Q, R = np.eye(X.shape[0]), X
            self.C[i] = Q.reshape(cl, d1, d2, Q.shape[1])
            self.C[i + 1] = np.tensordot(R, self.C[i + 1], axes=(1, 0))

    def rq_sweep(self, last, first):
        """Right-orthogonalize sites last..first+1, carrying into `first`."""
        for j in range(last, first, -1):
            cl, d1, d2, cr = self.C[j].shape
            X = self.C[j].reshape(cl, d1 * d2 * cr)
            if X.shape[0] <= X.shape[1]:
                Qt, Rt = canon.qr_pos(X.T)
                core, carry = Qt.T, Rt.T
            else:
                core, carry = np.eye(X.shape[1]), X
            self.C[j] = core.reshape(core.shape[0], d1, d2, cr)
            self.C[j - 1] = np.tensordot(self.C[j - 1], carry, axes=(3, 0))


def _half_sweeps(st, parts, fwd_first, stream):
    """Every F sub-TT sweeps forward and every B one backward when fwd_first,
    the reverse otherwise; sub-TTs do not interact within the phase."""
    for n, (s, e) in enumerate(parts):
        fwd = (n % 2 == 0) == fwd_first
        bonds = range(s, e) if fwd else range(e - 1, s - 1, -1)
        for i in bonds:
            st.update(i, "fwd" if fwd else "bwd", stream)


def fit_parallel_site(A, B, chi_max, n_sets, n_parts, sketch_p=-1, seed=0, pair=0, tau=0.0, C_init=None,
                      merge=True):
    """n_sets sets of local full sweeps on n_parts sub-TTs, then (merge) the
    binary merge.  Returns C scaled back by the norms (only meaningful
    after the merge: before it the sub-TTs' gauges disagree)."""
    L = len(A)
    parts = partition(L, n_parts)
    A1, B1, nu, caps = _preprocess(A, B)
    C = canon.right_orthogonalize(A1 if C_init is None else C_init)
    st = _State(A1, B1, C, chi_max, sketch_p, seed, pair, caps, tau)
    st.qr_sweep(0, L - 1)
    for b in range(0, L - 1):
        st.left_env(b)
    st.rq_sweep(L - 1, 0)
    for b in range(L - 1, 0, -1):
        st.right_env(b)
    for t in range(n_sets):
        _half_sweeps(st, parts, True, 4 * t)
        for n in range(0, n_parts, 2):
            st.update(parts[n][1], "both", 4 * t + 1)
        _half_sweeps(st, parts, False, 4 * t + 2)
        for n in range(1, n_parts - 1, 2):
            st.update(parts[n][1], "both", 4 * t + 3)
    if merge:
        base = 4 * n_sets
        _half_sweeps(st, parts, True, base)
        for n in range(0, n_parts, 2):
            st.update(parts[n][1], "fwd", base + 1)
        size, level = 2, 2
        while size < n_parts:
            for g in range(0, n_parts, 2 * size):
                m = parts[g + size - 1][1]            # boundary: sites m, m+1
                o_left = parts[g + size // 2 - 1][1] + 1   # centre of the left group
                o_right = parts[g + size + size // 2 - 1][1] + 1
                st.qr_sweep(o_left, m)
                for b in range(o_left, m):
                    st.left_env(b)
                st.rq_sweep(o_right, m + 1)
                for b in range(o_right, m + 1, -1):
                    st.right_env(b)
                st.update(m, "fwd", base + level)
            size *= 2
            level += 1
    out = [c.copy() for c in st.C]
    out[0] = out[0] * nu
    dims = [1] + [c.shape[3] for c in st.C]
    return ParallelResult(out, nu, dims, [c.copy() for c in st.C])
