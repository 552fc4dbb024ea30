"""The benchmark's own launch shape at its full size: 32^3x64, FP16 storage,
blocks of 16 sources, two right-hand sides per lane and time segments of 8
slices.  Three CG iterations (truncation by iteration count) are compared
element by element with the one-lane-per-site kernels (pinned to the oracle
on smaller lattices) and, for two of the sources, with the FP64 oracle."""

import numpy as np
import pytest

from lattice_inputs import make_gauge
from lattice_inputs.workloads import get_workload

pytestmark = pytest.mark.gpu

C3 = get_workload("c3")


def test_bench_launch_shape_full_lattice(orc):
    import torch
    import paper_1211_0126_amd as tq
    print("generating the 32^3x64 gauge field", flush=True)
    U = make_gauge(C3.dims, C3.eps, C3.gauge_seed)
    caps = tq.caps([tq.solve_params(prec=tq.PREC_F16, rhs_block=16)], max_sources=16)
    ctx = tq.tm_create(C3.dims, C3.kappa, C3.mu, -1, caps=caps)
    tq.tm_gauge_load(ctx, U)
    ids = list(range(100, 116))
    p = tq.solve_params(prec=tq.PREC_F16, tol=0.0, max_iter=3, rhs_block=16, true_resid=1)
    tq.tm_set_lane_rhs(ctx, tq.PREC_F16, 2)
    tq.tm_set_march(ctx, tq.PREC_F16, 8)
    print("FP16 CG, NR 2, tseg 8, 16 sources", flush=True)
    a, st_a, _ = tq.tsm_solve_batch(ctx, p, C3.noise_seed, ids)
    tq.tm_set_lane_rhs(ctx, tq.PREC_F16, 1)
    tq.tm_set_march(ctx, tq.PREC_F16, 0)
    print("FP16 CG, lane per site", flush=True)
    b, st_b, _ = tq.tsm_solve_batch(ctx, p, C3.noise_seed, ids)
    ctx.close()
    for sa, sb in zip(st_a, st_b):
        assert sa["iters"] == sb["iters"] == 3
        assert abs(sa["resid_true"] / sb["resid_true"] - 1) < 1e-2
    # element by element, each source against its own largest component
    d = (a - b).abs().amax(dim=(1, 2, 3)) / b.abs().amax(dim=(1, 2, 3))
    dn = torch.linalg.vector_norm((a - b).reshape(16, -1), dim=1) / torch.linalg.vector_norm(b.reshape(16, -1), dim=1)
    print("marching vs lane per site: elementwise max %.3g, normwise max %.3g" % (d.max().item(), dn.max().item()))
    assert d.max().item() < 5e-3 and dn.max().item() < 2e-3
    for i in (0, 15):
        eta = orc.noise_z4(C3.dims, C3.noise_seed, ids[i])
        print("oracle CG source %d" % ids[i], flush=True)
        x, so = orc.cgnr(C3.dims, -1, C3.kappa, C3.mu, U, eta, 0.0, 3)
        got = a[i].cpu().numpy()
        rel = np.linalg.norm((got - x).ravel()) / np.linalg.norm(x.ravel())
        print("source %d: FP16 marching vs FP64 oracle, normwise %.3g" % (ids[i], rel))
        assert rel < 5e-3
        assert abs(st_a[i]["resid_true"] / so["resid_true"] - 1) < 1e-2
    del a, b
    torch.cuda.empty_cache()


def test_evenodd_blocks_of_32_full_lattice(orc):
    """The even-odd solver at 32^3x64 with blocks of 32 FP16 sources: the
    split and merge of a block move fields larger than 4 GiB, the solution
    of each source is bitwise that of blocks of 16, and three Schur-CG
    iterations agree with the FP64 oracle's for two sources."""
    import torch
    import paper_1211_0126_amd as tq
    print("generating the 32^3x64 gauge field", flush=True)
    U = make_gauge(C3.dims, C3.eps, C3.gauge_seed)
    caps = tq.caps([tq.solve_params(prec=tq.PREC_F16, rhs_block=32, solver=tq.SOLVER_CG_EO)], max_sources=32)
    ctx = tq.tm_create(C3.dims, C3.kappa, C3.mu, -1, caps=caps)
    tq.tm_gauge_load(ctx, U)
    ids = list(range(200, 232))
    tq.tm_set_lane_rhs(ctx, tq.PREC_F16, 2)
    out = []
    for blk, tiles in ((32, 0), (16, 0), (32, 1)):
        tq.tm_set_eo_tiles(ctx, tq.PREC_F16, tiles)
        p = tq.solve_params(prec=tq.PREC_F16, tol=0.0, max_iter=3, rhs_block=blk, true_resid=1,
                            solver=tq.SOLVER_CG_EO)
        print("even-odd FP16 CG, blocks of %d, tiles %d" % (blk, tiles), flush=True)
        sol, st, _ = tq.tsm_solve_batch(ctx, p, C3.noise_seed, ids)
        out.append((sol, st))
    ctx.close()
    (a, sa), (b, sb), (c, sc) = out
    assert torch.equal(a, b)
    # the tile kernels hash the sources in FP32 where the others store them
    # in FP16 first: the same iterate up to FP16 rounding
    d = torch.linalg.vector_norm((c - a).reshape(32, -1), dim=1) / torch.linalg.vector_norm(a.reshape(32, -1), dim=1)
    print("tiles vs lane per half-site: normwise max %.3g" % d.max().item())
    assert d.max().item() < 2e-3
    del c
    for s in sa:
        assert s["iters"] == 3 and 0.01 < s["resid_true"] < 0.5, s
    for i in (0, 31):
        eta = orc.noise_z4(C3.dims, C3.noise_seed, ids[i])
        print("oracle even-odd CG source %d" % ids[i], flush=True)
        x, so = orc.cgnr_eo(C3.dims, -1, C3.kappa, C3.mu, U, eta, 0.0, 3)
        got = a[i].cpu().numpy()
        rel = np.linalg.norm((got - x).ravel()) / np.linalg.norm(x.ravel())
        print("source %d: FP16 even-odd vs FP64 oracle, normwise %.3g, true residual %.4g vs %.4g"
              % (ids[i], rel, sa[i]["resid_true"], so["resid_true"]))
        assert rel < 5e-3
        assert abs(sa[i]["resid_true"] / so["resid_true"] - 1) < 1e-2
    del a, b
    torch.cuda.empty_cache()
