"""The bench's algorithmic flop model (bench.sweep_flops, the MFMA work
credited in `tflops` and the roofline) against the flops the library
credits to each launch from its own GEMM shapes (profiling mode): one fresh
extension, the two-site product and one environment update per bond of a
serial sweep, at the benchmark's workload."""
import os
import sys

import pytest

from synth import make_pair

pytestmark = pytest.mark.gpu

sys.path.insert(0, os.path.dirname(os.path.dirname(os.path.abspath(__file__))))


def test_sweep_flop_model_matches_the_launches():
    import bench
    from paper_2606_23274_amd.api import FitContext
    w = bench.WORKLOAD
    A, B = make_pair(w["L"], w["d"], w["chi"], seed=w["seed"], decay=True)
    ctx = FitContext([(A, B)], w["chi_c"], precision="fp32", sketch_p=w["p"], seed=w["seed"],
                     profile=True, capture_graph=False)
    try:
        ctx.sweep(2)  # bond dims settle
        dims = ctx.bond_dims(0)
        ctx.sweep(2)
        prof = ctx.profile()
    finally:
        ctx.close()
    assert dims == bench.settled_dims(w["L"], w["d"], w["chi"], w["chi_c"])
    credited = sum(prof[c][1] for c in ("theta", "env_update", "env_ext1", "env_ext2") if c in prof) / 2
    model, _ = bench.sweep_flops(w["L"], w["d"], w["chi"], w["chi_c"], w["p"], dims, True)
    print("library", credited / 1e9, "GF per sweep; model", model / 1e9)
    assert abs(credited - model) <= 1e-9 * model


def test_batched_sweep_flop_model_matches_the_launches():
    """The even/odd schedule at L = 64, chi = 128, chi_C = 256: both
    extensions, the two-site product and both environment updates per bond
    (bench.batched_sweep_flops)."""
    import bench
    from paper_2606_23274_amd.api import FitContext
    A, B = make_pair(64, 2, 128, seed=0, decay=True)
    ctx = FitContext([(A, B)], 256, precision="fp32", schedule="even_odd", sketch_p=16, seed=0,
                     profile=True, capture_graph=False)
    try:
        ctx.sweep(2)
        dims = ctx.bond_dims(0)
        ctx.sweep(2)
        prof = ctx.profile()
    finally:
        ctx.close()
    credited = sum(prof[c][1] for c in ("theta", "env_update", "env_ext1", "env_ext2") if c in prof) / 2
    model = bench.batched_sweep_flops(64, 2, 128, dims)
    print("library", credited / 1e12, "TF per sweep; model", model / 1e12)
    assert abs(credited - model) <= 1e-9 * model
