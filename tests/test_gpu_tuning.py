"""Autotuner: picks one of the right-hand-side-per-lane variants by timing,
and solves with the tuned choice give the same per-source results."""

import numpy as np
import torch
import pytest

from lattice_inputs import make_gauge

pytestmark = pytest.mark.gpu


def test_autotune_choice_and_solve():
    import torch
    import paper_1211_0126_amd as tq
    dims = (8, 8, 8, 16)
    U = make_gauge(dims, 0.25, 5)
    ctx = tq.tm_create(dims, 0.1632, 0.004, -1)
    tq.tm_gauge_load(ctx, U)
    p = tq.solve_params(prec=tq.PREC_BF16, tol=1e-2, max_iter=-1, rhs_block=8)
    ref, st_ref, _ = tq.tsm_solve_batch(ctx, p, 3, list(range(8)))
    best, ms = tq.tm_autotune(ctx, tq.PREC_BF16, 8)
    assert best in (1, 2, 4)
    assert np.all(ms > 0) and ms[[1, 2, 4].index(best)] == ms.min()
    for nr in (1, 2, 4):
        tq.tm_set_lane_rhs(ctx, tq.PREC_BF16, nr)
        sol, st, _ = tq.tsm_solve_batch(ctx, p, 3, list(range(8)))
        # the per-lane width only regroups independent work (rounding may
        # differ between the compiled variants)
        assert all(abs(a["iters"] - b["iters"]) <= 1 for a, b in zip(st, st_ref))
        rel = (torch.linalg.vector_norm(sol - ref) / torch.linalg.vector_norm(ref)).item()
        assert rel < 1e-5
    # FP64 has the one-per-lane variant only
    best64, ms64 = tq.tm_autotune(ctx, tq.PREC_F64, 4)
    assert best64 == 1 and ms64[1] < 0 and ms64[2] < 0
    with pytest.raises(tq.TmError):
        tq.tm_set_lane_rhs(ctx, tq.PREC_F32, 3)
    ctx.close()


def test_autotune_cg_choice_and_solve():
    """tm_autotune_cg returns one of its candidates, keeps it for later
    solves, and those solves take the iterations of the untuned kernels."""
    import paper_1211_0126_amd as tq
    dims = (8, 8, 8, 16)
    U = make_gauge(dims, 0.25, 1002)
    ctx = tq.tm_create(dims, 0.1632, 0.004, -1)
    tq.tm_gauge_load(ctx, U)
    p = tq.solve_params(prec=tq.PREC_F16, tol=1e-2, max_iter=-1, rhs_block=8)
    ref, st_ref, _ = tq.tsm_solve_batch(ctx, p, 3, list(range(8)))
    nr, ts, ms = tq.tm_autotune_cg(ctx, tq.PREC_F16, 8)
    assert (nr, ts) in tq.binding_tuning.TUNE_CANDIDATES
    assert (nr, ts) in ms and ms[(nr, ts)] == min(ms.values())
    assert (4, 0) in ms and (1, 8) in ms
    sol, st, _ = tq.tsm_solve_batch(ctx, p, 3, list(range(8)))
    for a, b in zip(st, st_ref):
        assert abs(a["iters"] - b["iters"]) <= 1
    rel = (torch.linalg.vector_norm(sol - ref) / torch.linalg.vector_norm(ref)).item()
    assert rel < 2e-2
    with pytest.raises(tq.TmError):
        tq.tm_autotune_cg(ctx, tq.PREC_F16, 33)
    ctx.close()
