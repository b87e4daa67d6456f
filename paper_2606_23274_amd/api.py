"""Python front end of libmpofit: C ~ A B by the variational fit on one GPU.

PyTorch provides device memory and the stream; every step of the fit runs in
the library's HIP kernels.  Cores are (chi_left, d_out, d_in, chi_right)
float64 arrays (numpy or torch); C = A B contracts A's input leg with B's
output leg.
"""
from __future__ import annotations

import ctypes as C
import ctypes as C_

import numpy as np
import torch

from . import _lib
from . import tune as tune_mod


def check_train(cores, what, unit_in=False):
    """Shapes of a tensor train handed to the library, checked on the host:
    4-D cores (chi_l, d, d_in, chi_r) whose bonds chain up, boundary bonds
    1, one d, and d_in = d (an MPO) or d_in = 1 (unit_in: an MPS stored as
    an MPO).  The C ABI reads cores by these sizes, so a mismatch would read
    past the tensors."""
    if len(cores) < 1:
        raise ValueError(f"{what}: no cores")
    d = int(cores[0].shape[1])
    prev = 1
    for l, c in enumerate(cores):
        sh = tuple(int(x) for x in c.shape)
        if len(sh) != 4:
            raise ValueError(f"{what}: core {l} is not 4-D")
        want_in = 1 if unit_in else d
        if sh[0] != prev or sh[1] != d or sh[2] != want_in:
            raise ValueError(f"{what}: core {l} has shape {sh}, expected ({prev}, {d}, {want_in}, chi)")
        prev = sh[3]
    if prev != 1:
        raise ValueError(f"{what}: the last bond must be 1")
    return d


def _dev_cores(cores, device):
    out = []
    for c in cores:
        t = c if isinstance(c, torch.Tensor) else torch.from_numpy(np.ascontiguousarray(c))
        out.append(t.to(device=device, dtype=torch.float64).contiguous())
    return out


class _TT:
    """Keeps the ctypes view of one MPO and the tensors it points to alive."""

    def __init__(self, cores):
        self.cores = cores
        L = len(cores)
        self.d = int(cores[0].shape[1])
        chi = [int(cores[0].shape[0])] + [int(c.shape[3]) for c in cores]
        self.chi = (C.c_int32 * (L + 1))(*chi)
        self.ptrs = (C.c_void_p * L)(*[c.data_ptr() for c in cores])
        self.tt = _lib.MpoTT(L, self.d, self.chi, self.ptrs)


class _Setup:
    """Device copies of the cores, the ctypes pair array and the options."""

    def __init__(self, pairs, chi_max, precision, schedule, sketch_p, seed, capture_graph, device,
                 profile, pair_chi_max, tuning, c_init=None, first_sweep=0, track_error=False,
                 first_bond=0, first_half=0, tau=0.0, n_parts=0, mps=None):
        self.lib = _lib.load()
        self.device = torch.device(device)
        self.tts = []
        if mps is None:  # B an MPS: its cores have a unit input leg while A's do not
            mps = int(pairs[0][1][0].shape[2]) == 1 and int(pairs[0][0][0].shape[2]) != 1
        self.mps = bool(mps)
        arr = (_lib.MpoPair * len(pairs))()
        for i, (A, B) in enumerate(pairs):
            d = check_train(A, f"pair {i} A")
            if check_train(B, f"pair {i} B", unit_in=self.mps) != d or len(B) != len(A):
                raise ValueError(f"pair {i}: A and B must share L and d")
            ta, tb = _TT(_dev_cores(A, self.device)), _TT(_dev_cores(B, self.device))
            self.tts += [ta, tb]
            cm = 0 if pair_chi_max is None else int(pair_chi_max[i])
            arr[i] = _lib.MpoPair(ta.tt, tb.tt, cm)
        self.pairs = arr
        opts = _lib.MpoFitOpts()
        opts.chi_max = int(chi_max)
        opts.tau = float(tau)
        opts.precision = _lib.PRECISION[precision]
        opts.schedule = _lib.SCHEDULE[schedule]
        opts.sketch_p = int(sketch_p)
        opts.seed = int(seed)
        opts.capture_graph = 1 if capture_graph else 0
        opts.profile = 1 if profile else 0
        opts.first_sweep = int(first_sweep)
        opts.track_error = 1 if track_error else 0
        opts.first_bond = int(first_bond)
        opts.first_half = int(first_half)
        opts.n_parts = int(n_parts)
        opts.mps = 1 if self.mps else 0
        self.tune = tune_mod.to_ctypes(tune_mod.load(tuning)) if tuning is not None else None
        if self.tune is not None and len(self.tune):
            opts.tune = self.tune
            opts.n_tune = len(self.tune)
        if c_init is not None:  # one initial guess (list of FP64 cores) per pair
            if len(c_init) != len(pairs):
                raise ValueError("c_init needs one MPO per pair")
            for i, Cc in enumerate(c_init):
                check_train(Cc, f"c_init {i}", unit_in=self.mps)
            self.c_tts = [_TT(_dev_cores(Cc, self.device)) for Cc in c_init]
            self.c_arr = (_lib.MpoTT * len(pairs))(*[t.tt for t in self.c_tts])
            opts.c_init = self.c_arr
        self.opts = opts
        nbytes = C.c_size_t()
        _lib.check(self.lib.mpo_fit_workspace_bytes(arr, len(pairs), C.byref(opts), C.byref(nbytes)))
        self.workspace_bytes = nbytes.value
        # 256-byte alignment: over-allocate and offset
        self.ws = torch.empty(nbytes.value + 256, dtype=torch.uint8, device=self.device)
        self.ws_ptr = (self.ws.data_ptr() + 255) & ~255


class FitContext:
    """One fit of one or several independent MPO pairs.

    precision: 'fp64' | 'fp32' | 'bf16' | 'bf16x3'; schedule: 'serial' |
    'even_odd'; sketch_p < 0 runs the plain SVD, >= 0 the randomized SVD with
    chi_max + p sketch columns; pair_chi_max optionally sets each pair's cap;
    tuning: a GEMM tuning table (list of entries, or a JSON path) from
    autotune().  c_init: optional initial guess C per pair (lists of
    (chi_l, d, d, chi_r) FP64 cores, e.g. export_numpy() of another fit);
    default: A.  first_sweep: start as if that many sweeps had run (Philox
    stream and direction; with c_init = a fit's result after that many
    sweeps this resumes it).  first_bond (serial, one pair): updates of that
    sweep already done; first_half (even/odd): start with the second
    half-step.  track_error: reserve what sweep(..., errors=True) needs for
    the fit error per sweep.  tau > 0: the truncation tolerance of Sec.
    2.3.4 (bond dims then follow the singular values; bond_dims() reads
    them from the device).  schedule='parallel' with n_parts sub-TTs: the
    site-canonical parallel fit of Sec. 4; sweep(n) runs n sets, merge()
    joins the sub-TTs into one train before export.  mps: the MPO-MPS
    product of Sec. 1, B (and C) with (chi, d, 1, chi) cores; None detects
    it from B's cores.
    """

    def __init__(self, pairs, chi_max, precision="fp32", schedule="serial", sketch_p=-1, seed=0,
                 capture_graph=True, device="cuda:0", profile=False, pair_chi_max=None, tuning=None,
                 c_init=None, first_sweep=0, track_error=False, first_bond=0, first_half=0, tau=0.0,
                 n_parts=0, mps=None):
        su = _Setup(pairs, chi_max, precision, schedule, sketch_p, seed, capture_graph, device,
                    profile, pair_chi_max, tuning, c_init, first_sweep, track_error, first_bond,
                    first_half, tau, n_parts, mps)
        self._setup = su
        self.lib = su.lib
        self.device = su.device
        self.n_pairs = len(pairs)
        self.L = [len(A) for A, _ in pairs]
        self.workspace_bytes = su.workspace_bytes
        # a stream of our own (default priority): the legacy null stream
        # cannot be captured into a graph
        with torch.cuda.device(self.device):
            torch.cuda.current_stream().synchronize()
            self.stream = torch.cuda.Stream(device=self.device)
        ctx = C.c_void_p()
        _lib.check(self.lib.mpo_fit_init(C.byref(ctx), su.pairs, len(pairs), C.byref(su.opts),
                                         C.c_void_p(su.ws_ptr), su.workspace_bytes,
                                         C.c_void_p(self.stream.cuda_stream)))
        self.ctx = ctx

    def sweep(self, n=1, errors=False):
        """Runs n sweeps; with errors=True returns the fit error after each
        sweep as an (n_pairs, n) array (needs track_error)."""
        if not errors:
            _lib.check(self.lib.mpo_fit_sweep(self.ctx, int(n), None))  # synchronizes our stream
            return None
        out = (C.c_double * (self.n_pairs * int(n)))()
        _lib.check(self.lib.mpo_fit_sweep(self.ctx, int(n), out))
        return np.array(out[:], dtype=np.float64).reshape(self.n_pairs, int(n))

    def merge(self):
        """Parallel schedule: the binary merge of the sub-TTs (mpo_fit_merge)."""
        _lib.check(self.lib.mpo_fit_merge(self.ctx))

    def updates(self, n=1):
        """Runs the next n two-site updates (serial) or half-steps (even/odd)."""
        _lib.check(self.lib.mpo_fit_updates(self.ctx, int(n)))

    def position(self):
        """(sweep index, units of it already run)."""
        sw, un = C.c_int32(), C.c_int32()
        _lib.check(self.lib.mpo_fit_position(self.ctx, C.byref(sw), C.byref(un)))
        return sw.value, un.value

    def singular_values(self, bond, pair=0):
        """Singular values of bond `bond` (1..L-1) from its last update, on the
        normalized cores (times norm_factor() for C's own), dropped ones zero."""
        L = self.L[pair]
        out = (C.c_double * 4096)()
        r = C.c_int32()
        dims = self.bond_dims(pair)
        if not 1 <= bond < L or dims[bond] > 4096:
            raise ValueError("bad bond")
        _lib.check(self.lib.mpo_fit_singular_values(self.ctx, pair, int(bond), out, C.byref(r)))
        return np.array(out[:r.value], dtype=np.float64)

    def sweeps_done(self):
        n = C.c_int32()
        _lib.check(self.lib.mpo_fit_sweeps_done(self.ctx, C.byref(n)))
        return n.value

    def norm_factor(self, pair=0):
        """nu = ||A|| ||B|| split off by the preprocessing (export = nu * core 0)."""
        v = C.c_double()
        _lib.check(self.lib.mpo_fit_norm_factor(self.ctx, pair, C.byref(v)))
        return v.value

    def grad(self, W, A=None, B=None, pair=0, recompute_env=False):
        """loss = <W, Pi(A B)> at the frozen truncation bases of the last sweep
        and its gradient (mpo_fit_grad): returns (loss, [dA_l], [dB_l]) with
        float64 device tensors.  A, B default to the fitted pair."""
        su = self._setup
        if A is None:
            A = [t for t in su.tts[2 * pair].cores]
        if B is None:
            B = [t for t in su.tts[2 * pair + 1].cores]
        ta = _TT(_dev_cores(A, self.device))
        tb = _TT(_dev_cores(B, self.device))
        tw = _TT(_dev_cores(W, self.device))
        ab = _lib.MpoPair(ta.tt, tb.tt, 0)
        nbytes = C.c_size_t()
        _lib.check(self.lib.mpo_fit_grad_workspace_bytes(self.ctx, pair, C.byref(tw.tt),
                                                         int(bool(recompute_env)), C.byref(nbytes)))
        ws = torch.empty(nbytes.value + 256, dtype=torch.uint8, device=self.device)
        ws_ptr = (ws.data_ptr() + 255) & ~255
        gA = [torch.empty_like(t) for t in ta.cores]
        gB = [torch.empty_like(t) for t in tb.cores]
        pa = (C.c_void_p * len(gA))(*[g.data_ptr() for g in gA])
        pb = (C.c_void_p * len(gB))(*[g.data_ptr() for g in gB])
        loss = C.c_double()
        self.stream.wait_stream(torch.cuda.current_stream(self.device))
        _lib.check(self.lib.mpo_fit_grad(self.ctx, pair, C.byref(ab), C.byref(tw.tt), pa, pb,
                                         C.byref(loss), int(bool(recompute_env)), C.c_void_p(ws_ptr),
                                         nbytes.value))  # synchronizes our stream
        self.last_grad_workspace_bytes = nbytes.value
        return loss.value, gA, gB

    def truncations(self):
        """Singular values truncated before inversion so far (even/odd)."""
        v = C.c_int64()
        _lib.check(self.lib.mpo_fit_truncations(self.ctx, C.byref(v)))
        return v.value

    def last_sweep_ms(self):
        v = C.c_double()
        _lib.check(self.lib.mpo_fit_last_sweep_ms(self.ctx, C.byref(v)))
        return v.value

    def bond_dims(self, pair=0):
        L = self.L[pair]
        out = (C.c_int32 * (L + 1))()
        _lib.check(self.lib.mpo_fit_bond_dims(self.ctx, pair, out))
        return list(out)

    def export(self, pair=0):
        """C of one pair (scaled so that C ~ A B) as float64 device tensors."""
        dims = self.bond_dims(pair)
        L = self.L[pair]
        d = self._setup.tts[2 * pair].d
        du = 1 if self._setup.mps else d
        cores = [torch.empty((dims[i], d, du, dims[i + 1]), dtype=torch.float64, device=self.device)
                 for i in range(L)]
        ptrs = (C.c_void_p * L)(*[c.data_ptr() for c in cores])
        torch.cuda.current_stream(self.device).synchronize()  # allocations visible to our stream
        _lib.check(self.lib.mpo_fit_export_c(self.ctx, pair, ptrs))  # synchronizes our stream
        return cores

    def export_psi(self, pair=0):
        """Even/odd: the Psi_l of the inverse canonical form (normalized cores,
        no norm factor) as numpy arrays."""
        dims = self.bond_dims(pair)
        L = self.L[pair]
        d = self._setup.tts[2 * pair].d
        du = 1 if self._setup.mps else d
        cores = [torch.empty((dims[i], d, du, dims[i + 1]), dtype=torch.float64, device=self.device)
                 for i in range(L)]
        ptrs = (C.c_void_p * L)(*[c.data_ptr() for c in cores])
        torch.cuda.current_stream(self.device).synchronize()
        _lib.check(self.lib.mpo_fit_export_psi(self.ctx, pair, ptrs))
        return [c.cpu().numpy() for c in cores]

    def export_numpy(self, pair=0):
        return [c.cpu().numpy() for c in self.export(pair)]

    def profile(self):
        """Per kernel class of the last sweep() call (profiling contexts):
        {class: (device ms, algorithmic flops, launches)}, summed over its sweeps."""
        n = C.c_int32()
        _lib.check(self.lib.mpo_fit_profile(self.ctx, 0, None, None, None, None, C.byref(n)))
        ms = (C.c_double * n.value)()
        fl = (C.c_double * n.value)()
        nl = (C.c_int32 * n.value)()
        names = (C.c_char_p * n.value)()
        _lib.check(self.lib.mpo_fit_profile(self.ctx, n.value, ms, names, fl, nl, C.byref(n)))
        return {names[i].decode(): (ms[i], fl[i], nl[i]) for i in range(n.value)}

    def close(self):
        if getattr(self, "ctx", None):
            self.lib.mpo_fit_destroy(self.ctx)
            self.ctx = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def fit(A, B, chi_max, sweeps, **kw):
    """Convenience: fit one pair and return C's cores as numpy arrays."""
    ctx = FitContext([(A, B)], chi_max, **kw)
    try:
        ctx.sweep(sweeps)
        return ctx.export_numpy(0)
    finally:
        ctx.close()


def autotune(pairs, chi_max, precision="fp32", schedule="serial", sketch_p=-1, seed=0,
             device="cuda:0", pair_chi_max=None, reps=5):
    """Times the GEMM launch classes of one sweep of this fit under every
    tile / split-K candidate (mpo_gemm_autotune) and returns the table of
    winners (list of dicts, see tune.py)."""
    su = _Setup(pairs, chi_max, precision, schedule, sketch_p, seed, False, device, False,
                pair_chi_max, None)
    with torch.cuda.device(su.device):
        torch.cuda.current_stream().synchronize()
        stream = torch.cuda.Stream(device=su.device)
    cap = 256
    out = (_lib.MpoGemmTune * cap)()
    n = C.c_int32()
    _lib.check(su.lib.mpo_gemm_autotune(su.pairs, len(pairs), C.byref(su.opts), C.c_void_p(su.ws_ptr),
                                        su.workspace_bytes, C.c_void_p(stream.cuda_stream), int(reps),
                                        out, cap, C.byref(n)))
    return [tune_mod.entry_to_dict(out[i]) for i in range(n.value)]


class FitContract(torch.autograd.Function):
    """loss = <W, Pi(A B)>_F at the frozen truncation bases of a fit (the
    state of `fit_ctx` after its last sweep), differentiable in every core of
    A and B through the library's adjoint (mpo_fit_grad):

        loss = FitContract.apply(fit_ctx, W, *A_cores, *B_cores)
        loss.backward()
    """

    @staticmethod
    def forward(ctx, fit_ctx, W, *cores):
        L = len(cores) // 2
        loss, gA, gB = fit_ctx.grad(W, list(cores[:L]), list(cores[L:]),
                                    recompute_env=getattr(fit_ctx, "recompute_env", False))
        ctx.save_for_backward(*gA, *gB)
        return torch.tensor(loss, dtype=torch.float64, device=cores[0].device)

    @staticmethod
    def backward(ctx, g):
        return (None, None, *[g * t for t in ctx.saved_tensors])


def zipup(A, B, chi_max, sketch_p=-1, seed=0, device="cuda:0", numpy=True):
    """Zip-up contraction C ~ A B on the GPU (mpo_zipup, Alg. 2): the fit's
    initial guess (FitContext(..., c_init=[zipup(A, B, chi)])).  Returns
    numpy arrays (or device tensors with numpy=False)."""
    check_train(A, "A")
    check_train(B, "B")
    lib = _lib.load()
    dev = torch.device(device)
    ta, tb = _TT(_dev_cores(A, dev)), _TT(_dev_cores(B, dev))
    pair = _lib.MpoPair(ta.tt, tb.tt, 0)
    L = len(A)
    dims = (C.c_int32 * (L + 1))()
    nbytes = C.c_size_t()
    _lib.check(lib.mpo_zipup_bytes(C.byref(pair), int(chi_max), int(sketch_p), dims, C.byref(nbytes)))
    d = ta.d
    outs = [torch.empty((dims[i], d, d, dims[i + 1]), dtype=torch.float64, device=dev) for i in range(L)]
    tc = _TT(outs)
    with torch.cuda.device(dev):
        stream = torch.cuda.current_stream(dev)
        ws = torch.empty(nbytes.value + 256, dtype=torch.uint8, device=dev)
        ws_ptr = (ws.data_ptr() + 255) & ~255
        _lib.check(lib.mpo_zipup(C.byref(pair), int(chi_max), int(sketch_p), int(seed), C.byref(tc.tt),
                                 C.c_void_p(ws_ptr), nbytes.value, C.c_void_p(stream.cuda_stream)))
    return [o.cpu().numpy() for o in outs] if numpy else outs


def project_bonds(cores, k, seed=0, pair=0, which="A", device="cuda:0", numpy=True):
    """Randomized bond projection of one MPO on the GPU (mpo_bond_project,
    Sec. 3.2): every inner bond l with k < chi_l becomes min(k, chi_l) by
    Q_{l-1}^T A_l Q_l, Q_l from the Gaussian range finder on core l-1's
    right bond.  `which` picks the conventional Philox stream of A or B.
    Returns numpy arrays (or device tensors with numpy=False)."""
    check_train(cores, "cores")
    lib = _lib.load()
    dev = torch.device(device)
    tin = _TT(_dev_cores(cores, dev))
    L = len(cores)
    dims = [1] + [min(int(k), int(tin.chi[l])) for l in range(1, L)] + [1]
    d = tin.d
    outs = [torch.empty((dims[i], d, d, dims[i + 1]), dtype=torch.float64, device=dev) for i in range(L)]
    tout = _TT(outs)
    nbytes = C.c_size_t()
    _lib.check(lib.mpo_bond_project_bytes(C.byref(tin.tt), int(k), C.byref(nbytes)))
    with torch.cuda.device(dev):
        stream = torch.cuda.current_stream(dev)
        ws = torch.empty(nbytes.value + 256, dtype=torch.uint8, device=dev)
        ws_ptr = (ws.data_ptr() + 255) & ~255
        _lib.check(lib.mpo_bond_project(C.byref(tin.tt), int(k), int(seed), int(pair),
                                        int(_lib.PROJ_STREAM[which]), C.byref(tout.tt), C.c_void_p(ws_ptr),
                                        nbytes.value, C.c_void_p(stream.cuda_stream)))
    return [o.cpu().numpy() for o in outs] if numpy else outs


def fit_error(A, B, C, device="cuda:0", with_method=False, static=False):
    """||A B - C||_F / ||A B||_F and ||A B||_F^2 in FP64 on the GPU
    (mpo_contract_exact_check): Householder-QR sweeps of the naive product
    and the difference MPO when every chi_A chi_B + chi_C <= 512 (method 0,
    accurate far below sqrt(eps)), else transfer passes (method 1, floors
    near 1e-8 relative).  static=True uses mpo_contract_exact_check_static
    (the library's static scratch, no workspace)."""
    for X, what in ((A, "A"), (B, "B"), (C, "C")):
        check_train(X, what)
    lib = _lib.load()
    dev = torch.device(device)
    ta, tb, tc = (_TT(_dev_cores(X, dev)) for X in (A, B, C))
    pair = _lib.MpoPair(ta.tt, tb.tt, 0)
    err, n2, meth = C_.c_double(), C_.c_double(), C_.c_int32()
    with torch.cuda.device(dev):
        stream = torch.cuda.current_stream(dev)
        if static:
            _lib.check(lib.mpo_contract_exact_check_static(C_.byref(pair), C_.byref(tc.tt),
                                                           C_.byref(err), C_.byref(n2), C_.byref(meth),
                                                           C_.c_void_p(stream.cuda_stream)))
        else:
            nbytes = C_.c_size_t()
            _lib.check(lib.mpo_contract_check_bytes(C_.byref(pair), C_.byref(tc.tt), C_.byref(nbytes)))
            ws = torch.empty(nbytes.value + 256, dtype=torch.uint8, device=dev)
            ws_ptr = (ws.data_ptr() + 255) & ~255
            _lib.check(lib.mpo_contract_exact_check(C_.byref(pair), C_.byref(tc.tt), C_.byref(err),
                                                    C_.byref(n2), C_.byref(meth), C_.c_void_p(ws_ptr),
                                                    nbytes.value, C_.c_void_p(stream.cuda_stream)))
    if with_method:
        return err.value, n2.value, meth.value
    return err.value, n2.value
