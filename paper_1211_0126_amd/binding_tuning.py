"""Bindings of the graph-capture switch (tm_set_graphs) and the per-variant
profile (tm_profile_entries); argument marshalling
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


class ProfileEntry(ctypes.Structure):
    _fields_ = [("kc", ctypes.c_int32), ("prec", ctypes.c_int32), ("lane_rhs", ctypes.c_int32),
                ("solver", ctypes.c_int32), ("launches", ctypes.c_int64), ("ms", ctypes.c_double),
                ("bytes", ctypes.c_double)]


EXPORTS += ["tm_profile_entries"]


def tm_profile_entries(ctx: Context, cap=256):
    """Per-variant profile: list of dicts with kc (class name), prec,
    lane_rhs, solver, launches, ms, bytes."""
    from .binding import KC_NAMES
    ctx.lib.tm_profile_entries.argtypes = [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_int32,
                                           ctypes.POINTER(ctypes.c_int32)]
    ctx.lib.tm_profile_entries.restype = ctypes.c_int32
    buf = (ProfileEntry * cap)()
    n = ctypes.c_int32()
    ctx.check(ctx.lib.tm_profile_entries(ctx.h, buf, int(cap), ctypes.byref(n)))
    return [{"kc": KC_NAMES[e.kc], "prec": e.prec, "lane_rhs": e.lane_rhs, "solver": e.solver,
             "launches": int(e.launches), "ms": float(e.ms), "bytes": float(e.bytes)} for e in buf[:n.value]]
