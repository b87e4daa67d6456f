"""Writes evenodd_L64_chi128.json: functionals of the FP64 oracle's first
even/odd sweep at the batched configuration's full size (L=64, d=2,
chi_A=chi_B=128 with exp(-k/6) bond weights, seed 0, chi_C=256, p=16, Philox
seed 0), small enough to store: the bond dimensions, the number of singular
values truncated before inversion, the fit functional ||C||^2 - 2 <C, A B>,
and <C, G_i> for three seeded Gaussian MPOs G_i of bond dimension 4.

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
from synth import gaussian_mpo, make_pair  # noqa: E402


def probes(L):
    return [gaussian_mpo(np.random.default_rng(500 + i), L, 2, 4) for i in range(3)]


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
        "probes": [mpo.transfer_inner(C, G) for G in probes(64)],
    }
    path = os.path.join(os.path.dirname(os.path.abspath(__file__)), "evenodd_L64_chi128.json")
    with open(path, "w") as f:
        json.dump(out, f, indent=1)
    print("wrote", path)


if __name__ == "__main__":
    main()
