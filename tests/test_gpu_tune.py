"""The GEMM autotuner on the GPU: it returns one winner per launch class,
and a fit run with its table matches the oracle like the built-in choice."""
import numpy as np
import pytest

from oracle import fit as ofit
from oracle import mpo
from synth import make_pair

pytestmark = pytest.mark.gpu


@pytest.mark.parametrize("precision,schedule", [("fp64", "serial"), ("fp32", "even_odd")])
def test_autotune_table_and_fit(tmp_path, precision, schedule):
    from paper_2606_23274_amd import tune
    from paper_2606_23274_amd.api import FitContext, autotune
    A, B = make_pair(12, 2, 8, seed=5, decay=True)
    table = autotune([(A, B)], 16, precision=precision, schedule=schedule, sketch_p=4, seed=1,
                     reps=2)
    assert table
    for e in table:
        assert e["splits"] >= 1 and e["us"] > 0
        if e["mode"] == 0:  # FP64 tiles: 64x64, 32x32, 32x32 deep slabs, 16x16 with K over the waves
            assert e["tile"] in (0, 3, 4, 5)
            assert e["tile"] != 5 or e["splits"] == 1
        else:  # FP32 and BF16 modes: 64x64, 128x128, half-depth 64x64, the 32x32 tiles
            assert e["tile"] in (0, 1, 2, 3, 4)
    path = str(tmp_path / "tune.json")
    tune.save(table, path)
    ctx = FitContext([(A, B)], 16, precision=precision, schedule=schedule, sketch_p=4, seed=1,
                     tuning=path)
    try:
        ctx.sweep(1)
        C = ctx.export_numpy(0)
    finally:
        ctx.close()
    ref_fn = ofit.fit_serial if schedule == "serial" else ofit.fit_even_odd
    ref = ref_fn(A, B, 16, 1, sketch_p=4, seed=1)
    tol = 1e-10 if precision == "fp64" else 1e-5
    assert mpo.rel_diff(C, ref.C) < tol
