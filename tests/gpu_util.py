"""Helpers shared by the GPU tests (device buffers for the test hooks)."""
import ctypes as C

import numpy as np
import torch

from paper_2606_23274_amd import _lib

WS_BYTES = 96 << 20


class Hooks:
    def __init__(self):
        self.lib = _lib.load_test_hooks()
        self.ws = torch.empty(WS_BYTES + 256, dtype=torch.uint8, device="cuda:0")
        self.ws_ptr = (self.ws.data_ptr() + 255) & ~255
        self.stream = torch.cuda.current_stream().cuda_stream

    def args(self):
        return C.c_void_p(self.ws_ptr), WS_BYTES, C.c_void_p(self.stream)


def dev(x, dtype=torch.float64):
    return torch.from_numpy(np.ascontiguousarray(x)).to("cuda:0", dtype=dtype)


def ptr(t):
    return C.c_void_p(t.data_ptr())


def device_blocks(ctx, pair, bonds):
    """Two-site blocks Psi_{l} Y_l Psi_{l+1} (= U S V^T of bond l's last
    update) of an even/odd fit, as (chi_{l-1} d^2) x (d^2 chi_{l+1}) matrices
    with rows (c, s1, u1) and columns (s2, u2, c''); 1-based bonds."""
    psi = ctx.export_psi(pair)
    out = {}
    for l in bonds:
        S = ctx.singular_values(l, pair)
        Y = np.where(S > 0, 1.0 / np.where(S > 0, S, 1.0), 0.0)
        a, b = psi[l - 1], psi[l]
        r = a.shape[3]
        out[l] = (a.reshape(-1, r) * Y[None, :]) @ b.reshape(r, -1)
    return out


def oracle_block(f):
    """U S V^T of an oracle factorization (fit.Factor)."""
    return (f.U * f.S[None, :]) @ f.Vt


def block_dist(Bd, Bo):
    return float(np.linalg.norm(Bd - Bo) / np.linalg.norm(Bo))
