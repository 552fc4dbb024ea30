"""Persisted autotuner choices (JSON).

The choice of the CG kernels' traversal (right-hand sides per lane, time
segments or LDS tiles) depends on the device, the lattice, the storage
precision, the solver and the block of sources; the autotuners of the
library measure it (tm_autotune_cg, tm_autotune_eo).  This module keeps their
results in a JSON file, so that later runs on the same device apply the
choice without measuring again.  The file is $TMQCD_TUNE_CACHE, else
~/.cache/tmqcd/autotune.json.
"""

from __future__ import annotations

import json
import os

from .binding import PREC_F64, SOLVER_CG_EO, tm_set_lane_rhs
from .binding_tuning import tm_autotune_cg, tm_autotune_eo, tm_set_eo_tiles, tm_set_march


def cache_path() -> str:
    p = os.environ.get("TMQCD_TUNE_CACHE")
    if p:
        return p
    return os.path.join(os.path.expanduser("~"), ".cache", "tmqcd", "autotune.json")


def load(path: str | None = None) -> dict:
    path = path or cache_path()
    try:
        with open(path) as fh:
            d = json.load(fh)
        return d if isinstance(d, dict) else {}
    except (OSError, ValueError):
        return {}


def save(entries: dict, path: str | None = None) -> None:
    path = path or cache_path()
    os.makedirs(os.path.dirname(path) or ".", exist_ok=True)
    tmp = path + ".tmp%d" % os.getpid()
    with open(tmp, "w") as fh:
        json.dump(entries, fh, indent=1, sort_keys=True)
    os.replace(tmp, path)


def key(device: str, dims, kappa: float, mu: float, prec: int, solver: int, block: int) -> str:
    return "%s|%s|k%.6g|m%.6g|p%d|s%d|b%d" % (device, "x".join(str(int(d)) for d in dims), kappa, mu, prec, solver,
                                            block)


def device_name() -> str:
    import torch
    return torch.cuda.get_device_name(0) if torch.cuda.is_available() else "none"


def apply(ctx, prec: int, solver: int, rec: dict) -> None:
    """Install a recorded choice in the context."""
    tm_set_lane_rhs(ctx, prec, int(rec["lane_rhs"]))
    if solver == SOLVER_CG_EO:
        tm_set_eo_tiles(ctx, prec, int(rec.get("tiles", 0)))
    else:
        tm_set_march(ctx, prec, int(rec.get("tseg", 0)))


def tune(ctx, prec: int, solver: int, block: int, path: str | None = None, use_cache: bool = True) -> dict:
    """The traversal for (prec, solver, block) on this context: from the
    cache if recorded for this device and lattice, else measured by the
    library's autotuner and recorded.  The choice is installed in ctx.
    Returns {lane_rhs, tseg or tiles, ms_per_cg_iteration, cached}."""
    k = key(device_name(), ctx.dims, ctx.kappa, ctx.mu, prec, solver, block)
    entries = load(path) if use_cache else {}
    if k in entries:
        rec = dict(entries[k])
        apply(ctx, prec, solver, rec)
        rec["cached"] = True
        return rec
    if solver == SOLVER_CG_EO and prec != PREC_F64:
        nr, tiles, ms = tm_autotune_eo(ctx, prec, block)
        rec = {"lane_rhs": nr, "tiles": tiles, "ms_per_cg_iteration": ms[(nr, tiles)],
               "candidates": {"%d,%d" % c: m for c, m in ms.items()}}
    else:
        nr, ts, ms = tm_autotune_cg(ctx, prec, block)
        rec = {"lane_rhs": nr, "tseg": ts, "ms_per_cg_iteration": ms[(nr, ts)],
               "candidates": {"%d,%d" % c: m for c, m in ms.items()}}
    if use_cache:
        entries = load(path)
        entries[k] = rec
        save(entries, path)
    out = dict(rec)
    out["cached"] = False
    return out
