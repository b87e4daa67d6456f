"""GEMM tuning tables: the autotuner's output as JSON and back.

A table is a list of entries, one per class of grouped GEMM launches of a fit
(keyed by the operand kind, the largest problem's M, N, K, the problem count
and the GPU architecture), each with the chosen output tile and split-K count
and the measured launch time.  ``paper_2606_23274_amd.api.autotune`` produces
one; ``FitContext(tuning=...)`` consumes it.
"""
from __future__ import annotations

import ctypes as C
import json
import os

from . import _lib

ARCH = os.environ.get("MPOFIT_ARCH", "gfx950")
_INT_FIELDS = ("mode", "ta", "tb", "tc", "a_kcontig", "b_kcontig", "M", "N", "K", "count", "tile",
               "splits")
_MODES = {0: "fp64", 1: "fp32", 2: "bf16", 3: "bf16x3"}


def entry_to_dict(e) -> dict:
    d = {f: int(getattr(e, f)) for f in _INT_FIELDS}
    d["us"] = round(float(e.us), 3)
    d["dtype"] = _MODES.get(d["mode"], str(d["mode"]))
    d["arch"] = ARCH
    return d


def to_ctypes(entries):
    arr = (_lib.MpoGemmTune * len(entries))()
    for i, d in enumerate(entries):
        for f in _INT_FIELDS:
            setattr(arr[i], f, int(d[f]))
        arr[i].us = float(d.get("us", 0.0))
    return arr


def save(entries, path: str) -> None:
    with open(path, "w") as f:
        json.dump({"arch": ARCH, "entries": list(entries)}, f, indent=1)


def load(tuning):
    """A table from a list of entries or a JSON file written by save();
    entries for another architecture are dropped."""
    if isinstance(tuning, (str, os.PathLike)):
        with open(tuning) as f:
            doc = json.load(f)
        entries = doc["entries"] if isinstance(doc, dict) else doc
    else:
        entries = list(tuning)
    for d in entries:
        missing = [f for f in _INT_FIELDS if f not in d]
        if missing:
            raise ValueError(f"tuning entry lacks {missing}")
    return [d for d in entries if d.get("arch", ARCH) == ARCH]
