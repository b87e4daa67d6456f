"""Failure handling and replay determinism on the GPU: a non-finite input
core is reported as MPO_ERR_NUMERIC (the device flags), and a fit replayed
from captured HIP graphs equals the same fit launched eagerly, bit for bit,
after every sweep."""
import numpy as np
import pytest

from synth import make_pair

pytestmark = pytest.mark.gpu


@pytest.mark.parametrize("schedule", ["serial", "even_odd"])
def test_nan_input_core_is_numeric(schedule):
    from paper_2606_23274_amd import _lib
    from paper_2606_23274_amd.api import FitContext
    A, B = make_pair(8, 2, 8, seed=1, decay=True)
    B = [b.copy() for b in B]
    B[3][0, 1, 0, 2] = np.nan
    with pytest.raises(_lib.MpoError) as e:
        ctx = FitContext([(A, B)], 16, precision="fp64", schedule=schedule, sketch_p=4, seed=0)
        try:
            ctx.sweep(1)
        finally:
            ctx.close()
    assert e.value.status == 5  # MPO_ERR_NUMERIC


@pytest.mark.parametrize("schedule,precision", [("serial", "fp32"), ("serial", "fp64"), ("even_odd", "fp32")])
def test_graph_replay_matches_eager_bitwise(schedule, precision):
    """Sweeps replayed from captured graphs (several replays, host work and
    synchronizations between them) against eager launches of the same
    program: every exported train is identical."""
    from paper_2606_23274_amd.api import FitContext
    A, B = make_pair(12, 2, 16, seed=5, decay=True)
    runs = {}
    for graph in (True, False):
        ctx = FitContext([(A, B)], 32, precision=precision, schedule=schedule, sketch_p=8, seed=3,
                         capture_graph=graph)
        try:
            out = []
            for _ in range(4):
                ctx.sweep(1)
                out.append(ctx.export_numpy(0))
            runs[graph] = out
        finally:
            ctx.close()
    for s, (g, e) in enumerate(zip(runs[True], runs[False])):
        for cg, ce in zip(g, e):
            assert np.array_equal(cg, ce), f"sweep {s + 1} differs"


@pytest.mark.parametrize("kw", [dict(schedule="serial", tau=1.0), dict(schedule="even_odd", tau=2.0),
                                dict(schedule="parallel", n_parts=4)],
                         ids=["serial-tau", "even_odd-tau", "parallel"])
def test_graph_replay_matches_eager_bitwise_tau_and_parallel(kw):
    """The same for the tolerance rule (bond dims on the device, Omega of the
    actual shape drawn into a zero-filled buffer) and for the site-canonical
    parallel schedule (sets replayed, then the merge)."""
    from paper_2606_23274_amd.api import FitContext
    A, B = make_pair(16, 2, 8, seed=7, decay=True)
    runs = {}
    for graph in (True, False):
        ctx = FitContext([(A, B)], 12, precision="fp32", sketch_p=3, seed=4, capture_graph=graph, **kw)
        try:
            out = []
            for _ in range(4):
                ctx.sweep(1)
                if kw["schedule"] != "parallel":
                    out.append((ctx.bond_dims(0), ctx.export_numpy(0)))
            if kw["schedule"] == "parallel":
                ctx.merge()
                out.append((ctx.bond_dims(0), ctx.export_numpy(0)))
            runs[graph] = out
        finally:
            ctx.close()
    for s, ((dg, g), (de, e)) in enumerate(zip(runs[True], runs[False])):
        assert dg == de, f"step {s + 1}: bond dims differ"
        for cg, ce in zip(g, e):
            assert np.array_equal(cg, ce), f"step {s + 1} differs"
