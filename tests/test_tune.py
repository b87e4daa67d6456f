"""GEMM tuning tables on the host: JSON round trip and validation by the
library (bad tables are rejected at the workspace query)."""
import ctypes as C
import os

import pytest

lib_mod = pytest.importorskip("paper_2606_23274_amd._lib")
from paper_2606_23274_amd import tune  # noqa: E402

ENTRY = dict(mode=1, ta=1, tb=1, tc=1, a_kcontig=1, b_kcontig=1, M=512, N=512, K=4096, count=1,
             tile=0, splits=4, us=80.0)


def test_json_round_trip(tmp_path):
    path = str(tmp_path / "t.json")
    tune.save([dict(ENTRY, arch=tune.ARCH)], path)
    got = tune.load(path)
    assert got == [dict(ENTRY, arch=tune.ARCH)]
    arr = tune.to_ctypes(got)
    assert len(arr) == 1 and arr[0].splits == 4 and arr[0].K == 4096
    assert tune.entry_to_dict(arr[0])["splits"] == 4


def test_other_arch_dropped():
    assert tune.load([dict(ENTRY, arch="gfx942")]) == []


def test_incomplete_entry_rejected():
    with pytest.raises(ValueError):
        tune.load([{"mode": 1}])


def _query(opts):
    if not os.path.exists(lib_mod.LIB_PATH):
        pytest.skip("libmpofit.so not built")
    from tests.test_abi import _Pair
    lib = lib_mod.load()
    p = _Pair()
    arr = (lib_mod.MpoPair * 1)(p.pair)
    n = C.c_size_t(0)
    return lib.mpo_fit_workspace_bytes(arr, 1, C.byref(opts), C.byref(n))


def _opts():
    o = lib_mod.MpoFitOpts()
    o.chi_max, o.precision, o.sketch_p = 8, 1, 4
    return o


def test_library_validates_table():
    o = _opts()
    good = tune.to_ctypes([ENTRY])
    o.tune, o.n_tune = good, 1
    assert _query(o) == 0
    bad = tune.to_ctypes([dict(ENTRY, tile=6)])
    o.tune = bad
    assert _query(o) == 1
    o2 = _opts()
    o2.n_tune = 2  # no table pointer
    assert _query(o2) == 1
