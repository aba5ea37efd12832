"""MI355X-native time-stepping resolvent analysis (hot path of Martini, Rodriguez, Towne & Cavalieri,
"Efficient computation of global resolvent modes").

The computation lives in the HIP library ``libresolvent.so`` (C ABI in ``include/resolvent.h``); this package
is its thin Python binding.  Importing the package does not touch the GPU; the first call does.
"""
from . import operators  # noqa: F401


def __getattr__(name):
    if name in ("ResolventOp",):
        from .api import ResolventOp
        return ResolventOp
    if name in ("ResolventApply", "resolvent_apply"):
        from . import autograd
        return getattr(autograd, name)
    if name in ("ResolventError",):
        from ._lib import ResolventError
        return ResolventError
    raise AttributeError(name)
