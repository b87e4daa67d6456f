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
