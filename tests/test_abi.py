"""The C-ABI library on the host: it loads, exports every function the public
headers declare, and rejects bad arguments with the documented status codes
(mpo_fit_workspace_bytes does all its validation on the host, so these run
without a GPU)."""
import ctypes as C
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))

lib_mod = pytest.importorskip("paper_2606_23274_amd._lib")


def _lib():
    if not os.path.exists(lib_mod.LIB_PATH):
        pytest.skip("libmpofit.so not built")
    return lib_mod.load()


def _declared(header):
    text = open(os.path.join(ROOT, "include", header)).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"^(?:mpo_status|void|const char\*)\s+(mpo_\w+)\s*\(", text, re.M)))


@pytest.mark.parametrize("header", sorted(h for h in os.listdir(os.path.join(ROOT, "include"))
                                          if h.endswith(".h")))
def test_exports_every_declared_symbol(header):
    lib = _lib()
    names = _declared(header)
    assert names, header
    missing = [n for n in names if not hasattr(lib, n)]
    assert not missing, missing


def test_binding_covers_public_header():
    assert set(_declared("mpofit.h")) == set(lib_mod.EXPORTS)


class _Pair:
    """Host-side descriptors with placeholder (never dereferenced) core
    pointers: the workspace query validates shapes and options only."""

    def __init__(self, L=6, d=2, chi_a=4, chi_b=4, chi_max=0):
        self.keep = []
        self.pair = lib_mod.MpoPair(self._tt(L, d, chi_a), self._tt(L, d, chi_b), chi_max)

    def _tt(self, L, d, chi):
        dims = [1] + [chi] * (L - 1) + [1]
        chi_arr = (C.c_int32 * (L + 1))(*dims)
        cores = (C.c_void_p * L)(*([0x1000] * L))
        self.keep += [chi_arr, cores]
        return lib_mod.MpoTT(L, d, chi_arr, cores)


def _opts(**kw):
    o = lib_mod.MpoFitOpts()
    o.chi_max, o.tau, o.precision, o.schedule, o.sketch_p, o.seed = 8, 0.0, 1, 0, 4, 0
    for k, v in kw.items():
        setattr(o, k, v)
    return o


def _query(pairs, opts, n=None):
    lib = _lib()
    arr = (lib_mod.MpoPair * len(pairs))(*[p.pair for p in pairs])
    nbytes = C.c_size_t(0)
    st = lib.mpo_fit_workspace_bytes(arr, len(pairs) if n is None else n, C.byref(opts),
                                     C.byref(nbytes))
    return st, nbytes.value


@pytest.mark.parametrize("schedule", [0, 1])
@pytest.mark.parametrize("precision", [0, 1, 2, 3])
def test_workspace_query_ok(schedule, precision):
    st, n = _query([_Pair()], _opts(schedule=schedule, precision=precision))
    assert st == 0 and n > 0 and n % 256 == 0


@pytest.mark.parametrize("schedule", [0, 1])
def test_tau_workspace_adds_the_rank_slots(schedule):
    """A tolerance keeps the fixed-cap plan's buffers and adds the device
    bond dims and a diagonal per factorization."""
    st0, n0 = _query([_Pair()], _opts(schedule=schedule))
    st1, n1 = _query([_Pair()], _opts(schedule=schedule, tau=0.5))
    assert st0 == 0 and st1 == 0 and n0 < n1 <= n0 + 64 * 1024


@pytest.mark.parametrize("n_parts", [2, 4])
def test_parallel_workspace_query_ok(n_parts):
    st, n = _query([_Pair(L=8)], _opts(schedule=2, n_parts=n_parts))
    assert st == 0 and n > 0 and n % 256 == 0


@pytest.mark.parametrize("kw, pairs, status", [
    (dict(n_parts=0), 1, 1),          # n_parts must be a power of two >= 2
    (dict(n_parts=3), 1, 1),
    (dict(n_parts=4), 2, 6),          # one pair
    (dict(n_parts=2, tau=0.5), 1, 6),
    (dict(n_parts=2, track_error=1), 1, 6),
    (dict(n_parts=2, first_sweep=1), 1, 6),
    (dict(n_parts=4), 1, 2),          # L = 6 < 2 * 4 sites
])
def test_parallel_bad_options(kw, pairs, status):
    st, _ = _query([_Pair() for _ in range(pairs)], _opts(schedule=2, **kw))
    assert st == status
    assert _lib().mpo_last_error()


@pytest.mark.parametrize("schedule", [0, 1])
def test_mps_workspace_is_smaller(schedule):
    """B an MPS (unit input leg): its cores, C's and the extensions shrink."""
    st0, n0 = _query([_Pair()], _opts(schedule=schedule))
    st1, n1 = _query([_Pair()], _opts(schedule=schedule, mps=1))
    assert st0 == 0 and st1 == 0 and 0 < n1 < n0


@pytest.mark.parametrize("kw, status", [
    (dict(mps=2), 1),
    (dict(mps=-1), 1),
    (dict(mps=1, track_error=1), 6),
    (dict(mps=1, schedule=2, n_parts=2), 6),
])
def test_mps_bad_options(kw, status):
    st, _ = _query([_Pair(L=8)], _opts(**kw))
    assert st == status
    assert _lib().mpo_last_error()


def test_workspace_grows_with_pairs_and_bond():
    _, one = _query([_Pair()], _opts())
    _, two = _query([_Pair(), _Pair()], _opts())
    _, big = _query([_Pair(chi_a=16, chi_b=16)], _opts(chi_max=32))
    assert two > one and big > one


@pytest.mark.parametrize("opts, status", [
    (dict(tau=-1e-3), 1),           # tau must be >= 0
    (dict(tau=float("inf")), 1),    # and finite
    (dict(tau=float("nan")), 1),
    (dict(precision=9), 1),
    (dict(schedule=5), 1),
    (dict(schedule=3), 1),
    (dict(chi_max=0), 1),
    (dict(chi_max=500, sketch_p=16), 6),
])
def test_bad_options(opts, status):
    st, _ = _query([_Pair()], _opts(**opts))
    assert st == status
    assert _lib().mpo_last_error()


def test_bad_shapes():
    p = _Pair()
    p.pair.B.L = 5                      # A and B must share L
    assert _query([p], _opts())[0] == 2
    q = _Pair()
    q.keep[0][0] = 2                     # boundary bond must be 1
    assert _query([q], _opts())[0] == 2
    r = _Pair(L=1)
    assert _query([r], _opts())[0] == 2
    assert _query([_Pair()], _opts(), n=0)[0] == 1


def test_null_pointers():
    lib = _lib()
    nbytes = C.c_size_t(0)
    assert lib.mpo_fit_workspace_bytes(None, 1, C.byref(_opts()), C.byref(nbytes)) == 1
    p = _Pair()
    p.pair.A.cores = C.cast(None, C.POINTER(C.c_void_p))
    assert _query([p], _opts())[0] == 1
    assert lib.mpo_fit_sweep(None, 1, None) == 1
    assert lib.mpo_fit_singular_values(None, 0, 1, None, None) == 1
    assert lib.mpo_contract_exact_check_static(None, None, None, None, None, None) == 1


def test_undersized_or_misaligned_workspace():
    """mpo_fit_init checks the workspace before any device call."""
    lib = _lib()
    p = _Pair()
    arr = (lib_mod.MpoPair * 1)(p.pair)
    opts = _opts()
    ctx = C.c_void_p()
    st = lib.mpo_fit_init(C.byref(ctx), arr, 1, C.byref(opts), C.c_void_p(0x100000), 1024, None)
    assert st == 3 and b"small" in lib.mpo_last_error()
    st = lib.mpo_fit_init(C.byref(ctx), arr, 1, C.byref(opts), C.c_void_p(0x100001), 1 << 40, None)
    assert st == 3 and b"aligned" in lib.mpo_last_error()
    assert not ctx.value


@pytest.mark.parametrize("opts, status", [
    (dict(first_sweep=-1), 1),
    (dict(track_error=2), 1),
    (dict(first_sweep=3), 0),
    (dict(first_sweep=3, schedule=1), 0),
])
def test_resume_and_error_options(opts, status):
    st, _ = _query([_Pair()], _opts(**opts))
    assert st == status


def test_error_tracking_reserves_workspace():
    _, plain = _query([_Pair()], _opts())
    _, track = _query([_Pair()], _opts(track_error=1))
    assert track > plain


def test_check_bytes_routes():
    """The exact check's workspace query (host only): small bonds take the
    QR route, whose scratch is much smaller than the four-layer pass's."""
    lib = _lib()
    small, big = _Pair(chi_a=4, chi_b=4), _Pair(chi_a=24, chi_b=24)
    n_small, n_big = C.c_size_t(0), C.c_size_t(0)
    assert lib.mpo_contract_check_bytes(C.byref(small.pair), C.byref(small.pair.A), C.byref(n_small)) == 0
    assert lib.mpo_contract_check_bytes(C.byref(big.pair), C.byref(big.pair.A), C.byref(n_big)) == 0
    assert 0 < n_small.value < n_big.value


def test_initial_guess_validation():
    """An initial guess must match the pair's L and d and have valid bonds."""
    lib = _lib()
    p = _Pair()
    good = _Pair(chi_a=6)   # an MPO of the same L and d
    opts = _opts()
    arr = (lib_mod.MpoTT * 1)(good.pair.A)
    opts.c_init = arr
    assert _query([p], opts)[0] == 0
    bad = _Pair(L=5)
    opts.c_init = (lib_mod.MpoTT * 1)(bad.pair.A)
    assert _query([p], opts)[0] == 2
    nul = _Pair()
    nul.pair.A.cores = C.cast(None, C.POINTER(C.c_void_p))
    opts.c_init = (lib_mod.MpoTT * 1)(nul.pair.A)
    assert _query([p], opts)[0] == 1
    big = _Pair(chi_a=600)
    opts.c_init = (lib_mod.MpoTT * 1)(big.pair.A)
    assert _query([p], opts)[0] == 6


def test_bond_project_queries_and_errors():
    """mpo_bond_project's host-side validation (no device access): the
    workspace grows with the bonds that are cut, k < 1, L < 2, null
    pointers and an output of the wrong bond dims are rejected before any
    launch."""
    lib = _lib()
    p = _Pair(L=6, chi_a=16)
    n4, n8, n64 = C.c_size_t(0), C.c_size_t(0), C.c_size_t(0)
    assert lib.mpo_bond_project_bytes(C.byref(p.pair.A), 4, C.byref(n4)) == 0
    assert lib.mpo_bond_project_bytes(C.byref(p.pair.A), 8, C.byref(n8)) == 0
    assert lib.mpo_bond_project_bytes(C.byref(p.pair.A), 64, C.byref(n64)) == 0
    assert n64.value < n4.value < n8.value
    assert lib.mpo_bond_project_bytes(C.byref(p.pair.A), 0, C.byref(n4)) == 1
    assert lib.mpo_bond_project_bytes(None, 4, C.byref(n4)) == 1
    one = _Pair(L=1)
    assert lib.mpo_bond_project_bytes(C.byref(one.pair.A), 4, C.byref(n4)) == 2
    ws = C.c_void_p(0x100000)
    assert lib.mpo_bond_project(C.byref(p.pair.A), 4, 0, 0, 1 << 30, None, ws, n4.value, None) == 1
    wrong = _Pair(L=6, chi_a=16)  # output dims must be min(k, chi) = 4
    assert lib.mpo_bond_project(C.byref(p.pair.A), 4, 0, 0, 1 << 30, C.byref(wrong.pair.A), ws,
                                1 << 40, None) == 2
    assert lib.mpo_bond_project(C.byref(p.pair.A), 4, 0, 0, -1, C.byref(wrong.pair.A), ws,
                                1 << 40, None) == 1


def test_zipup_dims_and_errors():
    """mpo_zipup_bytes (host only): C's bond dims r_l = min(chi_max, r_{l-1}
    d^2, chi_A chi_B of the right-canonical inputs) and the error codes."""
    lib = _lib()
    p = _Pair(L=6, chi_a=4, chi_b=3)
    dims = (C.c_int32 * 7)()
    n = C.c_size_t(0)
    assert lib.mpo_zipup_bytes(C.byref(p.pair), 10, 4, dims, C.byref(n)) == 0
    # right-canonical dims of A: [1, 4, 4, 4, 4, 4, 1] (4 <= d^2 * 4), of B: [1, 3, ..., 3, 1]
    assert list(dims) == [1, 4, 10, 10, 10, 10, 1]
    assert n.value > 0
    assert lib.mpo_zipup_bytes(C.byref(p.pair), 0, 4, dims, C.byref(n)) == 1
    assert lib.mpo_zipup_bytes(C.byref(p.pair), 600, 4, dims, C.byref(n)) == 6
    assert lib.mpo_zipup_bytes(None, 10, 4, dims, C.byref(n)) == 1
    bad = _Pair(L=6)
    bad.pair.B.L = 5
    assert lib.mpo_zipup_bytes(C.byref(bad.pair), 10, 4, dims, C.byref(n)) == 2
    wrong = _Pair(L=6, chi_a=4)  # C's dims must be the zip-up's
    assert lib.mpo_zipup(C.byref(p.pair), 10, 4, 0, C.byref(wrong.pair.A), C.c_void_p(0x100000), 1 << 40,
                         None) == 2


def test_python_front_end_checks_train_shapes():
    """The front end refuses trains the library would read past: broken bond
    chains, wrong boundary bonds, MPS cores where MPO cores are read."""
    import numpy as np
    from paper_2606_23274_amd.api import check_train
    ok = [np.zeros((1, 2, 2, 3)), np.zeros((3, 2, 2, 1))]
    assert check_train(ok, "A") == 2
    mps = [np.zeros((1, 2, 1, 3)), np.zeros((3, 2, 1, 1))]
    assert check_train(mps, "B", unit_in=True) == 2
    bad = [
        [np.zeros((1, 2, 2, 3)), np.zeros((4, 2, 2, 1))],   # bonds do not chain
        [np.zeros((2, 2, 2, 3)), np.zeros((3, 2, 2, 1))],   # left boundary
        [np.zeros((1, 2, 2, 3)), np.zeros((3, 2, 2, 2))],   # right boundary
        [np.zeros((1, 2, 2, 3)), np.zeros((3, 3, 3, 1))],   # d changes
        mps,                                                  # MPS where an MPO is read
        [np.zeros((1, 2, 2))],                                # not 4-D, one core
    ]
    for t in bad:
        with pytest.raises(ValueError):
            check_train(t, "A")
    with pytest.raises(ValueError):
        check_train(ok, "B", unit_in=True)
