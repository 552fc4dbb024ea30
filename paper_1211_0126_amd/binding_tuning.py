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
                ("solver", ctypes.c_int32), ("tseg", ctypes.c_int32), ("reliable", ctypes.c_int32),
                ("launches", ctypes.c_int64), ("ms", ctypes.c_double), ("bytes", ctypes.c_double)]


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
    return [{"kc": KC_NAMES[e.kc], "prec": e.prec, "lane_rhs": e.lane_rhs, "solver": e.solver, "tseg": e.tseg,
             "reliable": e.reliable, "launches": int(e.launches), "ms": float(e.ms), "bytes": float(e.bytes)} for e in buf[:n.value]]


EXPORTS += ["tm_set_march"]


def tm_set_march(ctx: Context, prec, tseg):
    """Time slices per lane of the CG stencils in storage precision prec
    (0: one lane per site)."""
    ctx.lib.tm_set_march.argtypes = [ctypes.c_void_p, ctypes.c_int32, ctypes.c_int32]
    ctx.lib.tm_set_march.restype = ctypes.c_int32
    ctx.check(ctx.lib.tm_set_march(ctx.h, int(prec), int(tseg)))


EXPORTS += ["tm_autotune_cg"]
TUNE_CANDIDATES = [(1, 0), (2, 0), (4, 0), (1, 4), (1, 8), (1, 16), (2, 4), (2, 8)]


def tm_autotune_cg(ctx: Context, prec, nrhs):
    """Returns (right-hand sides per lane, time slices per lane, {candidate:
    ms per CG iteration}) and keeps the choice for later solves."""
    import numpy as np
    ctx.lib.tm_autotune_cg.argtypes = [ctypes.c_void_p, ctypes.c_int32, ctypes.c_int32,
                                       ctypes.POINTER(ctypes.c_int32), ctypes.POINTER(ctypes.c_int32), ctypes.c_void_p]
    ctx.lib.tm_autotune_cg.restype = ctypes.c_int32
    nr, ts = ctypes.c_int32(), ctypes.c_int32()
    ms = np.zeros(len(TUNE_CANDIDATES), dtype=np.float64)
    ctx.check(ctx.lib.tm_autotune_cg(ctx.h, int(prec), int(nrhs), ctypes.byref(nr), ctypes.byref(ts),
                                     ms.ctypes.data_as(ctypes.c_void_p)))
    return int(nr.value), int(ts.value), {c: float(m) for c, m in zip(TUNE_CANDIDATES, ms) if m >= 0}


EXPORTS += ["tm_set_eo_tiles"]


def tm_set_eo_tiles(ctx: Context, prec, on):
    """Even-odd half-hops: 1 = LDS-staged link tiles shared by all right-hand
    sides, 0 = one lane per half-site (the default)."""
    ctx.lib.tm_set_eo_tiles.argtypes = [ctypes.c_void_p, ctypes.c_int32, ctypes.c_int32]
    ctx.lib.tm_set_eo_tiles.restype = ctypes.c_int32
    ctx.check(ctx.lib.tm_set_eo_tiles(ctx.h, int(prec), int(on)))


EXPORTS += ["tm_autotune_eo"]

EO_TUNE_CANDIDATES = [(1, 0), (2, 0), (4, 0), (1, 1), (2, 1), (4, 1)]


def tm_autotune_eo(ctx: Context, prec, nrhs):
    """Even-odd solver: returns (right-hand sides per lane, tiles 0/1,
    {(nr, tiles): ms per Schur-CG iteration}) and keeps the choice."""
    import numpy as np
    ctx.lib.tm_autotune_eo.argtypes = [ctypes.c_void_p, ctypes.c_int32, ctypes.c_int32,
                                       ctypes.POINTER(ctypes.c_int32), ctypes.POINTER(ctypes.c_int32), ctypes.c_void_p]
    ctx.lib.tm_autotune_eo.restype = ctypes.c_int32
    nr, tl = ctypes.c_int32(), ctypes.c_int32()
    ms = np.zeros(len(EO_TUNE_CANDIDATES), dtype=np.float64)
    ctx.check(ctx.lib.tm_autotune_eo(ctx.h, int(prec), int(nrhs), ctypes.byref(nr), ctypes.byref(tl),
                                     ms.ctypes.data_as(ctypes.c_void_p)))
    return int(nr.value), int(tl.value), {c: float(m) for c, m in zip(EO_TUNE_CANDIDATES, ms) if m >= 0}
