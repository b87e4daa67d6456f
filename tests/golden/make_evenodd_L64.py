"""Writes evenodd_L64_chi128.json: functionals of the FP64 oracle's first
even/odd sweep at the batched configuration's full size (L=64, d=2,
chi_A=chi_B=128 with exp(-k/6) bond weights, seed 0, chi_C=256, p=16, Philox
seed 0), small enough to store: the bond dimensions, the number of singular
values truncated before inversion, ||C||^2, <C, A B>, and <C, A B_i> for
three probes B_i: B with the core at site 5, 32 or 58 replaced by a seeded
Gaussian core of the same shape (each probes C around that site).

Run: python tests/golden/make_evenodd_L64.py   (about 4 minutes on 8 cores)
"""
import json
import os
import sys

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
sys.path.insert(0, ROOT)

from oracle import fit as ofit  # noqa: E402
from oracle import mpo  # noqa: E402
from synth import make_pair  # noqa: E402


PROBE_SITES = (5, 32, 58)


def probes(B):
    out = []
    for i, l in enumerate(PROBE_SITES):
        Bi = [c for c in B]
        rng = np.random.default_rng(500 + i)
        Bi[l] = rng.standard_normal(B[l].shape) * np.linalg.norm(B[l]) / np.sqrt(B[l].size)
        out.append(Bi)
    return out


def main():
    A, B = make_pair(64, 2, 128, seed=0, decay=True)
    res = ofit.fit_even_odd(A, B, 256, 1, sketch_p=16, seed=0)
    C = res.C
    out = {
        "config": "L=64 d=2 chi_A=chi_B=128 decay seed 0; chi_C=256 p=16 Philox seed 0; 1 even/odd sweep",
        "bond_dims": res.bond_dims,
        "truncated": res.n_guard,
        "norm2": mpo.left_orth_norm(C) ** 2,
        "inner_ab": mpo.three_layer_inner(C, A, B),
        "probes": [mpo.three_layer_inner(C, A, Bi) for Bi in probes(B)],
    }
    path = os.path.join(os.path.dirname(os.path.abspath(__file__)), "evenodd_L64_chi128.json")
    with open(path, "w") as f:
        json.dump(out, f, indent=1)
    print("wrote", path)


if __name__ == "__main__":
    main()
