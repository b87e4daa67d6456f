"""Zip-up contraction of two MPOs (Alg. 2, Sec. 2.2), the initial guess of
the fit.  Test infrastructure: only tests/, the package's smoke check and
bench.py's CPU baseline use it.

A and B are first brought to right-canonical form (every core but the first
right-orthogonal, Sec. 2.2), then one left-to-right pass: R_0 = [[[1]]];
at site l the residual R_{l-1} (c, a, b) is contracted with A_l on the A
bond and with B_l on the B bond and the shared physical leg, giving
R''_l (c, s, u, a', b'); its matrix M_l ((c s u) x (a' b')) is factorized
by the truncated SVD of the two-site update (fit.factorize: rank cap
min(chi_max, rows, chi_A chi_B), the randomized range finder of Sec. 3.1
when sketch_p >= 0, the sign rule and the drop rule of the update); C_l = U
and R_l = S V^T.  At the last site M_L has one column and C_L = M_L (the
C_L S V^T of Alg. 2).  The Philox stream of the sketches is ZIP_STREAM at
bond l (reading 27).
"""
from __future__ import annotations

import numpy as np

from . import canon
from .fit import factorize
from .philox import gaussian_matrix

ZIP_STREAM = (1 << 30) + 2


def zipup(A, B, chi_max: int, sketch_p: int = -1, seed: int = 0, pair: int = 0):
    """C ~ A B by Alg. 2 (left to right); returns the list of cores."""
    A1 = canon.right_orthogonalize(A)
    B1 = canon.right_orthogonalize(B)
    L = len(A1)
    R = np.ones((1, 1, 1))
    C = []
    for l in range(L):
        Rp = np.tensordot(R, A1[l], axes=(1, 0))                # (c, b, s, t, a')
        Rpp = np.einsum("cbsta,btux->csuax", Rp, B1[l])          # (c, s, u, a', b')
        c0, d1, d2, a1, b1 = Rpp.shape
        M = Rpp.reshape(c0 * d1 * d2, a1 * b1)
        if l == L - 1:
            C.append(M.reshape(c0, d1, d2, 1))
            break
        f = factorize(M, chi_max, sketch_p, a1 * b1,
                      lambda m, k, l=l: gaussian_matrix(m, k, seed, pair, ZIP_STREAM, l + 1))
        r = len(f.S)
        C.append(f.U.reshape(c0, d1, d2, r))
        R = (f.S[:, None] * f.Vt).reshape(r, a1, b1)
    return C
