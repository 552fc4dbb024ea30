"""Time-marching CG stencils (tm_set_march) against the one-lane-per-site
kernels and the FP64 oracle: same iterates up to rounding, on lattices
whose spatial volume is or is not a multiple of the 256-lane tile, with
segment lengths that do and do not divide the time extent."""

import numpy as np
import pytest
import torch

from lattice_inputs import make_gauge

pytestmark = pytest.mark.gpu


def _solve(tq, ctx, prec, blk, nr, tseg, tol=1e-30, maxit=12, reliable=0, stop=0):
    tq.tm_set_lane_rhs(ctx, prec, nr)
    tq.tm_set_march(ctx, prec, tseg)
    p = tq.solve_params(prec=prec, tol=tol, max_iter=maxit, rhs_block=blk, reliable=reliable, stop=stop)
    sol, st, _ = tq.tsm_solve_batch(ctx, p, 77, list(range(blk)))
    tq.tm_set_march(ctx, prec, 0)
    tq.tm_set_lane_rhs(ctx, prec, 0)
    return sol, st


def _rel(a, b):
    return (torch.linalg.vector_norm(a - b) / torch.linalg.vector_norm(b)).item()


@pytest.mark.parametrize("dims", [(8, 8, 8, 8), (6, 4, 4, 10), (16, 16, 16, 8)])
@pytest.mark.parametrize("prec,nr", [(1, 1), (1, 2), (2, 1), (2, 2), (3, 2)])
@pytest.mark.parametrize("tseg", [1, 3, 64])
def test_march_matches_lane_per_site(dims, prec, nr, tseg):
    import paper_1211_0126_amd as tq
    U = make_gauge(dims, 0.25, 31)
    ctx = tq.tm_create(dims, 0.1632, 0.004, -1)
    tq.tm_gauge_load(ctx, U)
    ref, st_ref = _solve(tq, ctx, prec, 4, nr, 0)
    sol, st = _solve(tq, ctx, prec, 4, nr, tseg)
    assert [s["iters"] for s in st] == [s["iters"] for s in st_ref]
    # 12 truncated iterations; FP32 arithmetic summed in another order, and
    # for FP16 / BF16 storage rounding of intermediate fields
    tol = {1: 1e-5, 2: 2e-3, 3: 2e-2}[prec]
    for i in range(4):
        assert _rel(sol[i], ref[i]) < tol, (i, _rel(sol[i], ref[i]))
    ctx.close()


def test_march_fp64_matches_oracle(orc):
    import paper_1211_0126_amd as tq
    dims = (4, 4, 6, 8)
    U = make_gauge(dims, 0.3, 5)
    ctx = tq.tm_create(dims, 0.16, 0.03125, -1)
    tq.tm_gauge_load(ctx, U)
    sol, st = _solve(tq, ctx, 0, 2, 1, 3, tol=1e-12, maxit=-1)
    sol = sol.cpu().numpy()
    for j in range(2):
        eta = orc.noise_z4(dims, 77, j)
        x, so = orc.cgnr(dims, -1, 0.16, 0.03125, U, eta, 1e-12)
        assert st[j]["converged"]
        assert abs(st[j]["iters"] - so["iters"]) <= 1
        assert np.linalg.norm(sol[j] - x) / np.linalg.norm(x) < 1e-9
    ctx.close()


def test_march_reliable_and_true_residual_stop():
    """The marching kernels serve the reliable-update HP path and the
    recursive true-residual stop as well."""
    import paper_1211_0126_amd as tq
    dims = (8, 8, 8, 8)
    U = make_gauge(dims, 0.25, 1002)
    ctx = tq.tm_create(dims, 0.1632, 0.004, -1)
    tq.tm_gauge_load(ctx, U)
    ref, st_ref = _solve(tq, ctx, 1, 4, 1, 0, tol=1e-10, maxit=-1, reliable=1)
    sol, st = _solve(tq, ctx, 1, 4, 1, 5, tol=1e-10, maxit=-1, reliable=1)
    for i in range(4):
        assert st[i]["converged"] and st[i]["resid_iterated"] <= 1e-10
        assert _rel(sol[i], ref[i]) < 1e-8
    ref, st_ref = _solve(tq, ctx, 1, 4, 1, 0, tol=1e-2, maxit=-1, stop=tq.STOP_TRUE)
    sol, st = _solve(tq, ctx, 1, 4, 1, 2, tol=1e-2, maxit=-1, stop=tq.STOP_TRUE)
    assert [s["iters"] for s in st] == [s["iters"] for s in st_ref]
    ctx.close()


def test_set_march_rejects_bad_arguments():
    import paper_1211_0126_amd as tq
    ctx = tq.tm_create((4, 4, 4, 4), 0.16, 0.03, -1)
    for prec, tseg in ((4, 1), (-1, 1), (1, -1), (1, 70000)):
        with pytest.raises(tq.TmError):
            tq.tm_set_march(ctx, prec, tseg)
    ctx.close()
