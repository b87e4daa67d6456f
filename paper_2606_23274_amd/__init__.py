"""MI355X-native randomized variational fit of MPO-MPO products (libmpofit).

The compute path is the HIP library ``libmpofit.so`` built from ``csrc/``
(``python -m paper_2606_23274_amd.build``); this package only marshals
arguments to its C ABI (``include/mpofit.h``).
"""
from . import _lib  # noqa: F401


def __getattr__(name):
    if name in ("FitContext", "fit"):
        from . import api
        return getattr(api, name)
    raise AttributeError(name)
