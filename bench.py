"""Benchmark: one TSM estimate of the disconnected loops per step on one GPU.

A step is the whole path (Z4 sources, N_HP high- and N_HP + N_LP
low-precision CG solves of M^dag M, loop contractions for 16 Gamma and 27
momenta per timeslice, the Eq. 4 combination) over one synthetic gauge
field, by default the 32^3x64 workload (N_HP = 32, N_LP = 2048).

value = N_LP / (wall time of the whole step): LP TSM sources per second,
HP correction included.  Per-kernel durations come from HIP events recorded
on the library's stream around every launch during the timed steps; the
roofline entry is for the kernel class with the largest total time.

Prints one JSON line.
"""

from __future__ import annotations

import argparse
import hashlib
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "LP TSM sources/s + Dslash HBM GB/s, learned/mixed vs plain CG at equal residual"
HBM_PEAK_GBS = 8000.0
PREC_NAMES = {"f64": 0, "f32": 1, "f16": 2, "bf16": 3}


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=1)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--workload", default="c3")
    ap.add_argument("--lp-prec", default="f16", choices=list(PREC_NAMES))
    ap.add_argument("--lp-block", type=int, default=16)
    ap.add_argument("--hp-block", type=int, default=8)
    ap.add_argument("--n-lp", type=int, default=None, help="override N_LP (default: the workload's)")
    ap.add_argument("--n-hp", type=int, default=None)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-fp32-reference", action="store_true")
    ap.add_argument("--cpu-threads", type=int, default=0)
    return ap.parse_args()


def log(msg):
    print("[bench] " + msg, file=sys.stderr, flush=True)


def main():
    args = parse()
    if args.gpus != 1:
        print("bench.py runs on one GPU only (--gpus 1); the path shards by source, see the design notes",
              file=sys.stderr)
        sys.exit(2)

    import torch
    import paper_1211_0126_amd as tq
    from lattice_inputs import make_gauge, get_workload

    wl = get_workload(args.workload)
    n_lp = wl.n_lp if args.n_lp is None else args.n_lp
    n_hp = wl.n_hp if args.n_hp is None else args.n_hp
    torch.cuda.set_device(0)
    log("generating gauge field %s" % (wl.dims,))
    t0 = time.time()
    U = make_gauge(wl.dims, wl.eps, wl.gauge_seed)
    log("gauge generated in %.1f s" % (time.time() - t0))
    ctx = tq.tm_create(wl.dims, wl.kappa, wl.mu, wl.t_bc)
    tq.tm_gauge_load(ctx, U)
    mom = wl.momenta()
    lp_prec = PREC_NAMES[args.lp_prec]
    lp = tq.solve_params(prec=lp_prec, tol=wl.lp_tol, max_iter=wl.lp_maxit, rhs_block=args.lp_block, true_resid=1)
    hp = tq.solve_params(prec=tq.PREC_F32, tol=wl.hp_tol, max_iter=-1, reliable=1, delta=0.1,
                         rhs_block=args.hp_block, true_resid=1)

    def step():
        return tq.tsm_loops(ctx, wl.noise_seed, n_hp, n_lp, lp, hp, mom, stats=True)

    for w in range(args.warmup):
        t0 = time.time()
        r = step()
        log("warmup step %d: %.1f ms (LP iters %d, HP iters %d)" % (w, 1e3 * (time.time() - t0),
                                                                      r["run"]["lp_iters"], r["run"]["hp_iters"]))

    tq.tm_profile_enable(ctx, True)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    res = None
    for k in range(args.steps):
        res = step()
        log("timed step %d done" % k)
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    prof = tq.tm_profile_read(ctx)
    tq.tm_profile_enable(ctx, False)
    ms_per_step = 1e3 * (t1 - t0) / args.steps
    value = n_lp / (ms_per_step / 1e3)

    # dominant kernel class
    dom = max(prof, key=lambda k: prof[k]["ms"])
    d = prof[dom]
    avg_ms = d["ms"] / max(d["launches"], 1)
    avg_bytes = d["bytes"] / max(d["launches"], 1)
    achieved = avg_bytes / (avg_ms * 1e-3) / 1e9
    roofline = {"bound": "hbm", "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
                "frac": round(achieved / HBM_PEAK_GBS, 4), "traffic": None, "kernel": dom,
                "avg_launch_us": round(avg_ms * 1e3, 2), "algorithmic_bytes_per_launch": avg_bytes}
    per_class = {k: {"launches": v["launches"], "avg_us": round(1e3 * v["ms"] / max(v["launches"], 1), 2),
                     "GBps": round(v["bytes"] / max(v["ms"], 1e-9) / 1e6, 1) if v["bytes"] > 0 else None,
                     "total_ms": round(v["ms"], 1)} for k, v in prof.items()}

    st = res["stats"]
    lp_true = [s[0]["resid_true"] for s in st]
    lp_iters = [s[0]["iters"] for s in st]
    hp_iters = [s[1]["iters"] for s in st[:n_hp]]
    run = res["run"]

    out = {
        "metric": METRIC,
        "value": round(value, 2),
        "unit": "LP sources/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(ms_per_step, 1),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {
            "workload": "%s: %dx%dx%dx%d twisted-mass Wilson, kappa %.4f, a*mu %.4f, N_HP %d (FP32 + FP64 reliable "
                        "updates to %.0e), N_LP %d (%s storage, FP32 arithmetic, to %.0e), 16 Gamma x %d momenta"
                        % (wl.name, *wl.dims, wl.kappa, wl.mu, n_hp, wl.hp_tol, n_lp, args.lp_prec, wl.lp_tol,
                           len(mom)),
            "lattice": "x".join(str(d) for d in wl.dims),
            "n_hp": n_hp, "n_lp": n_lp, "lp_storage": args.lp_prec, "lp_rhs_block": args.lp_block,
            "hp_rhs_block": args.hp_block,
        },
        "lp_phase_sources_per_s": round(n_lp / (run["ms_lp_phase"] / 1e3), 2),
        "hp_phase_ms": round(run["ms_hp_phase"], 1),
        "lp_iters_mean": round(float(np.mean(lp_iters)), 2),
        "hp_iters_mean": round(float(np.mean(hp_iters)), 2) if hp_iters else None,
        "lp_true_resid_median": float(np.median(lp_true)),
        "lp_true_resid_max": float(np.max(lp_true)),
        "hp_true_resid_max": run["max_hp_resid_true"],
        "kernels": per_class,
        "roofline": roofline,
    }

    # plain FP32 single-RHS CG on the same GPU, same sources, same stop
    if not args.no_fp32_reference:
        ns = 64
        ids = list(range(n_hp, n_hp + ns))
        ref_p = tq.solve_params(prec=tq.PREC_F32, tol=wl.lp_tol, max_iter=wl.lp_maxit, rhs_block=1, true_resid=1)
        cand_p = tq.solve_params(prec=lp_prec, tol=wl.lp_tol, max_iter=wl.lp_maxit, rhs_block=args.lp_block,
                                 true_resid=1)
        tq.tsm_solve_batch(ctx, ref_p, wl.noise_seed, ids[:4], want_solutions=False)  # warm
        torch.cuda.synchronize()
        ta = time.perf_counter()
        _, st_ref, _ = tq.tsm_solve_batch(ctx, ref_p, wl.noise_seed, ids, want_solutions=False)
        torch.cuda.synchronize()
        tb = time.perf_counter()
        _, st_c, _ = tq.tsm_solve_batch(ctx, cand_p, wl.noise_seed, ids, want_solutions=False)
        torch.cuda.synchronize()
        tc = time.perf_counter()
        out["fp32_1rhs_reference"] = {
            "sources": ns,
            "solve_sources_per_s": round(ns / (tb - ta), 2),
            "true_resid_median": float(np.median([s["resid_true"] for s in st_ref])),
            "iters_mean": float(np.mean([s["iters"] for s in st_ref])),
            "candidate_solve_sources_per_s": round(ns / (tc - tb), 2),
            "candidate_true_resid_median": float(np.median([s["resid_true"] for s in st_c])),
            "speedup": round((tb - ta) / (tc - tb), 3),
        }
        log("fp32 1-rhs reference: %s" % out["fp32_1rhs_reference"])

    ctx.close()

    if not args.no_cpu_baseline:
        out["cpu_baseline"] = cpu_baseline(wl, U, args.cpu_threads)

    print(json.dumps(out), flush=True)


def cpu_baseline(wl, U, threads):
    """The FP64 oracle on the host cores: one LP source (CG to the LP
    tolerance on the normal equations) plus its loop contraction on the
    same lattice, scaled to LP sources/s."""
    import oracle
    n = threads or min(16, os.cpu_count() or 1)
    oracle.set_threads(n)
    used = oracle.get_threads()
    t0 = time.perf_counter()
    eta = oracle.noise_z4(wl.dims, wl.noise_seed, wl.n_hp)
    x, st = oracle.cgnr(wl.dims, wl.t_bc, wl.kappa, wl.mu, U, eta, wl.lp_tol, wl.lp_maxit)
    oracle.loops(wl.dims, eta, x, wl.momenta())
    dt = time.perf_counter() - t0
    log("cpu baseline: one LP source in %.1f s (%d iterations, %d threads)" % (dt, st["iters"], used))
    return {"value": round(1.0 / dt, 5), "unit": "LP sources/s", "cores": used, "kind": "oracle",
            "sample": "1 LP source (FP64 CG on M^dag M to %.0e, %d iterations) + 16x%d-momentum loop contraction "
                      "on the %s lattice; %.1f s" % (wl.lp_tol, st["iters"], len(wl.momenta()),
                                                       "x".join(str(d) for d in wl.dims), dt)}


if __name__ == "__main__":
    main()
