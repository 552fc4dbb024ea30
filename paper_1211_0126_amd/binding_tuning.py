"""Binding of the graph-capture switch (tm_set_graphs); argument marshalling
only."""

from __future__ import annotations

import ctypes

from .binding import Context, EXPORTS

EXPORTS += ["tm_set_graphs"]


def tm_set_graphs(ctx: Context, on=None):
    """Enable/disable graph capture of CG chunks (None: leave); returns the
    number of graph replays so far."""
    ctx.lib.tm_set_graphs.argtypes = [ctypes.c_void_p, ctypes.c_int32, ctypes.POINTER(ctypes.c_int64)]
    ctx.lib.tm_set_graphs.restype = ctypes.c_int32
    n = ctypes.c_int64()
    ctx.check(ctx.lib.tm_set_graphs(ctx.h, -1 if on is None else int(bool(on)), ctypes.byref(n)))
    return int(n.value)
