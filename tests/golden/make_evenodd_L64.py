"""Writes evenodd_L64_chi128.json: the FP64 oracle's first even/odd sweep at
the batched configuration's full size (L=64, d=2, chi_A=chi_B=128 with
exp(-k/6) bond weights, seed 0, chi_C=256, p=16, Philox seed 0), in a form
small enough to store:
  * the bond dimensions and the number of dropped singular values;
  * every bond's singular values from its update in the sweep (normalized
    cores, dropped values zero), 13 significant digits;
  * 64 sampled entries of the merged train C (Sec. 4.7, C_l = Psi_l Y_l,
    scaled by ||A|| ||B||) at each of 9 sites, positions from a seeded
    generator;
  * ||C||^2, <C, A B> and <C, A B_i> for three probes B_i (B with the core
    at site 5, 32 or 58 replaced by a seeded Gaussian core of the same
    shape).

Run: python tests/golden/make_evenodd_L64.py   (about 5 minutes on 8 cores)
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
SAMPLE_SITES = (0, 1, 2, 15, 31, 32, 47, 62, 63)
N_SAMPLES = 64


def probes(B):
    out = []
    for i, l in enumerate(PROBE_SITES):
        Bi = [c for c in B]
        rng = np.random.default_rng(500 + i)
        Bi[l] = rng.standard_normal(B[l].shape) * np.linalg.norm(B[l]) / np.sqrt(B[l].size)
        out.append(Bi)
    return out


def sample_positions(site, shape):
    """Flat indices of the sampled entries of core `site` with this shape."""
    rng = np.random.default_rng(900 + site)
    n = int(np.prod(shape))
    return sorted(int(i) for i in rng.choice(n, size=min(N_SAMPLES, n), replace=False))


def main():
    A, B = make_pair(64, 2, 128, seed=0, decay=True)
    svals = {}

    def on_bond(sweep, q, l, M, f, Psi0, Y0):
        svals[l] = [float(f"{v:.12e}") for v in f.S]

    res = ofit.fit_even_odd(A, B, 256, 1, sketch_p=16, seed=0, on_bond=on_bond)
    C = res.C
    samples = {}
    for l in SAMPLE_SITES:
        pos = sample_positions(l, C[l].shape)
        flat = C[l].reshape(-1)
        samples[str(l)] = {"shape": list(C[l].shape), "index": pos,
                           "value": [float(f"{flat[i]:.12e}") for i in pos]}
    out = {
        "config": "L=64 d=2 chi_A=chi_B=128 decay seed 0; chi_C=256 p=16 Philox seed 0; 1 even/odd sweep",
        "bond_dims": res.bond_dims,
        "dropped": res.n_guard,
        "singular_values": [svals[l] for l in range(1, 64)],
        "samples": samples,
        "norm2": mpo.left_orth_norm(C) ** 2,
        "inner_ab": mpo.three_layer_inner(C, A, B),
        "probes": [mpo.three_layer_inner(C, A, Bi) for Bi in probes(B)],
    }
    path = os.path.join(os.path.dirname(os.path.abspath(__file__)), "evenodd_L64_chi128.json")
    with open(path, "w") as f:
        json.dump(out, f, separators=(",", ":"))
    print("wrote", path)


if __name__ == "__main__":
    main()
