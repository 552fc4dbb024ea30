"""GPU parity of the even-odd (Schur complement) solver against the FP64
oracle's even-odd CG, through the C ABI: truncated FP64 iterates, converged
solves, the tracked true-residual stop, FP32 iterations with FP64 reliable
updates, reduced-precision LP solves, the right-hand sides per lane, block
independence and the 4^4 TSM estimate with even-odd LP and HP solves."""

import numpy as np
import pytest

from lattice_inputs import make_gauge
from lattice_inputs.workloads import get_workload, momenta_27

pytestmark = pytest.mark.gpu

# (dims, kappa, a*mu, eps): single partial block of half sites (2x4x6x8:
# 192 per parity), ragged (6x4x8x10: 960), the 4^4 workload, several tiles,
# and a lattice whose half-site blocks run in the brick order (Lx/2 = 8: a
# wave is 8 rows, a block 4 z planes; 2 x 2 bricks per time slice)
LATTICES = [
    ((2, 4, 6, 8), 0.1632, 0.004, 0.3),
    ((6, 4, 8, 10), 0.1632, 0.003, 0.25),
    ((4, 4, 4, 4), 0.160, 0.03125, 0.3),
    ((8, 8, 8, 8), 0.1632, 0.004, 0.25),
    ((16, 16, 8, 4), 0.1632, 0.004, 0.25),
]


def _ctx(dims, kappa, mu, U):
    import paper_1211_0126_amd as tq
    ctx = tq.tm_create(dims, kappa, mu, -1)
    tq.tm_gauge_load(ctx, U)
    return ctx


def _rel(a, b):
    return np.linalg.norm((a - b).ravel()) / np.linalg.norm(b.ravel())


@pytest.mark.parametrize("lat", LATTICES)
def test_eo_fp64_truncated_iterates_match_oracle(orc, lat):
    """Truncation by iteration count: the same Schur-CG iterate (and its
    reconstructed even half) on both sides, to 1e-12."""
    import paper_1211_0126_amd as tq
    dims, kappa, mu, eps = lat
    U = make_gauge(dims, eps, 41)
    ctx = _ctx(dims, kappa, mu, U)
    ids = [0, 3, 7]
    for k in (1, 2, 6):
        p = tq.solve_params(prec=tq.PREC_F64, tol=0.0, max_iter=k, rhs_block=2, solver=tq.SOLVER_CG_EO)
        sol, st, _ = tq.tsm_solve_batch(ctx, p, 13, ids)
        sol = sol.cpu().numpy()
        for i, j in enumerate(ids):
            eta = orc.noise_z4(dims, 13, j)
            x, so = orc.cgnr_eo(dims, -1, kappa, mu, U, eta, 0.0, k)
            assert st[i]["iters"] == k and st[i]["truncated"]
            assert _rel(sol[i], x) < 1e-12, (dims, k, j, _rel(sol[i], x))
            assert abs(st[i]["resid_true"] - so["resid_true"]) < 1e-10 * max(1.0, so["resid_true"])
    ctx.close()


def test_eo_fp64_converged_and_true_stop(orc):
    import paper_1211_0126_amd as tq
    dims, kappa, mu, eps = LATTICES[3]
    U = make_gauge(dims, eps, 43)
    ctx = _ctx(dims, kappa, mu, U)
    ids = [0, 1, 2, 5]
    for tol, stop in ((1e-2, tq.STOP_NORMAL), (1e-11, tq.STOP_NORMAL), (1e-2, tq.STOP_TRUE)):
        p = tq.solve_params(prec=tq.PREC_F64, tol=tol, max_iter=-1, rhs_block=4, stop=stop,
                            solver=tq.SOLVER_CG_EO)
        sol, st, _ = tq.tsm_solve_batch(ctx, p, 17, ids)
        sol = sol.cpu().numpy()
        for i, j in enumerate(ids):
            eta = orc.noise_z4(dims, 17, j)
            x, so = orc.cgnr_eo(dims, -1, kappa, mu, U, eta, tol, -1, stop)
            assert st[i]["converged"] and st[i]["iters"] == so["iters"], (tol, stop, st[i], so)
            assert _rel(sol[i], x) < 1e-10
            if stop == tq.STOP_TRUE:
                assert st[i]["resid_true"] <= tol and abs(st[i]["resid_iterated"] - st[i]["resid_true"]) < 1e-9
    # the converged solution solves the whole system
    eta = orc.noise_z4(dims, 17, 0)
    p = tq.solve_params(prec=tq.PREC_F64, tol=1e-11, max_iter=-1, rhs_block=1, solver=tq.SOLVER_CG_EO)
    sol, st, _ = tq.tsm_solve_batch(ctx, p, 17, [0])
    mx = orc.apply_op(dims, -1, kappa, mu, orc.OP_M, U, sol.cpu().numpy()[0])
    assert np.linalg.norm((eta - mx).ravel()) / np.linalg.norm(eta.ravel()) < 1e-9
    ctx.close()


@pytest.mark.parametrize("delta", [0.1, 1e-4])
def test_eo_fp32_reliable_hp(orc, delta):
    """FP32 iterations with FP64 reliable updates on the Schur system, to
    1e-10 on the normal equations and on the true residual, with updates
    every decade of the residual or every four decades."""
    import paper_1211_0126_amd as tq
    dims, kappa, mu, eps = LATTICES[3]
    U = make_gauge(dims, eps, 1002)
    ctx = _ctx(dims, kappa, mu, U)
    ids = [0, 1, 2, 3]
    for stop in (tq.STOP_NORMAL, tq.STOP_TRUE):
        p = tq.solve_params(prec=tq.PREC_F32, tol=1e-10, max_iter=-1, reliable=1, delta=delta, rhs_block=4,
                            stop=stop, solver=tq.SOLVER_CG_EO)
        sol, st, _ = tq.tsm_solve_batch(ctx, p, 9, ids)
        sol = sol.cpu().numpy()
        for i, j in enumerate(ids):
            eta = orc.noise_z4(dims, 9, j)
            x, so = orc.cgnr_eo(dims, -1, kappa, mu, U, eta, 1e-10, -1, stop)
            mx = orc.apply_op(dims, -1, kappa, mu, orc.OP_M, U, sol[i])
            true = np.linalg.norm((eta - mx).ravel()) / np.linalg.norm(eta.ravel())
            print("stop %d source %d: iters %d (oracle %d), true residual %.3g (reported %.3g)"
                  % (stop, j, st[i]["iters"], so["iters"], true, st[i]["resid_true"]))
            assert st[i]["converged"], st[i]
            assert abs(st[i]["iters"] - so["iters"]) <= 3
            assert _rel(sol[i], x) < 1e-8
            if stop == tq.STOP_TRUE:
                assert st[i]["resid_true"] <= 1e-10 and true <= 1.01e-10
    ctx.close()


@pytest.mark.parametrize("delta", [0.1, 1e-2])
@pytest.mark.parametrize("prec", [2, 3])
def test_eo_half_storage_reliable_hp(orc, prec, delta):
    """FP16 / BF16 storage of the iteration vectors (FP32 arithmetic) with
    FP64 reliable updates, stopped on the FP64 true residual: converged to
    1e-10 (checked with the oracle's operator), the oracle's solution to
    1e-8, at most half again the oracle's iterations."""
    import paper_1211_0126_amd as tq
    dims, kappa, mu, eps = LATTICES[3]
    U = make_gauge(dims, eps, 1002)
    ctx = _ctx(dims, kappa, mu, U)
    ids = [0, 1, 2, 3]
    p = tq.solve_params(prec=prec, tol=1e-10, max_iter=400, reliable=1, delta=delta, rhs_block=4,
                        stop=tq.STOP_TRUE, solver=tq.SOLVER_CG_EO)
    sol, st, _ = tq.tsm_solve_batch(ctx, p, 9, ids)
    sol = sol.cpu().numpy()
    for i, j in enumerate(ids):
        eta = orc.noise_z4(dims, 9, j)
        x, so = orc.cgnr_eo(dims, -1, kappa, mu, U, eta, 1e-10, -1, tq.STOP_TRUE)
        mx = orc.apply_op(dims, -1, kappa, mu, orc.OP_M, U, sol[i])
        true = np.linalg.norm((eta - mx).ravel()) / np.linalg.norm(eta.ravel())
        print("prec %d delta %g source %d: iters %d (oracle %d), true residual %.3g (reported %.3g)"
              % (prec, delta, j, st[i]["iters"], so["iters"], true, st[i]["resid_true"]))
        assert st[i]["converged"], st[i]
        assert st[i]["iters"] <= 1.5 * so["iters"] + 2
        assert st[i]["resid_true"] <= 1e-10 and true <= 1.01e-10
        assert _rel(sol[i], x) < 1e-8
    ctx.close()


@pytest.mark.parametrize("tiles", [0, 1])
@pytest.mark.parametrize("prec", [1, 2, 3])
def test_eo_reduced_precision_lp(orc, prec, tiles):
    """FP32 / FP16 / BF16 storage on the Schur system, both traversals of
    the half-hops: converged at the LP tolerance within an iteration of the
    FP64 oracle, with an FP64 true residual close to the oracle's."""
    import paper_1211_0126_amd as tq
    dims, kappa, mu, eps = LATTICES[3]
    U = make_gauge(dims, eps, 1002)
    ctx = _ctx(dims, kappa, mu, U)
    tq.tm_set_eo_tiles(ctx, prec, tiles)
    ids = list(range(8))
    p = tq.solve_params(prec=prec, tol=1e-2, max_iter=-1, rhs_block=8, solver=tq.SOLVER_CG_EO)
    sol, st, _ = tq.tsm_solve_batch(ctx, p, 7, ids)
    for i, j in enumerate(ids):
        eta = orc.noise_z4(dims, 7, j)
        x, so = orc.cgnr_eo(dims, -1, kappa, mu, U, eta, 1e-2)
        assert st[i]["converged"]
        assert abs(st[i]["iters"] - so["iters"]) <= 1, (st[i], so)
        assert abs(st[i]["resid_true"] - so["resid_true"]) < 0.05 * so["resid_true"] + 1e-3
    ctx.close()


@pytest.mark.parametrize("prec", [1, 2])
def test_eo_brick_order_lp_and_reliable_hp(orc, prec):
    """On the brick-order lattice: reduced-precision LP solves (the ring of
    directions) within an iteration of the FP64 oracle, and FP32 HP solves
    with FP64 reliable updates to 1e-8 of the oracle's solution."""
    import paper_1211_0126_amd as tq
    dims, kappa, mu, eps = LATTICES[4]
    U = make_gauge(dims, eps, 47)
    ctx = _ctx(dims, kappa, mu, U)
    ids = list(range(4))
    p = tq.solve_params(prec=prec, tol=1e-2, max_iter=-1, rhs_block=4, solver=tq.SOLVER_CG_EO)
    _, st, _ = tq.tsm_solve_batch(ctx, p, 5, ids)
    hp = tq.solve_params(prec=tq.PREC_F32, tol=1e-10, max_iter=-1, reliable=1, delta=0.1, rhs_block=2,
                         stop=tq.STOP_TRUE, solver=tq.SOLVER_CG_EO)
    sol, sth, _ = tq.tsm_solve_batch(ctx, hp, 5, ids[:2])
    sol = sol.cpu().numpy()
    ctx.close()
    for i, j in enumerate(ids):
        eta = orc.noise_z4(dims, 5, j)
        x, so = orc.cgnr_eo(dims, -1, kappa, mu, U, eta, 1e-2)
        assert st[i]["converged"] and abs(st[i]["iters"] - so["iters"]) <= 1, (st[i], so)
        assert abs(st[i]["resid_true"] - so["resid_true"]) < 0.05 * so["resid_true"] + 1e-3
        if i < 2:
            x, so = orc.cgnr_eo(dims, -1, kappa, mu, U, eta, 1e-10, -1, tq.STOP_TRUE)
            assert sth[i]["converged"] and sth[i]["resid_true"] <= 1e-10
            assert _rel(sol[i], x) < 1e-8, _rel(sol[i], x)


@pytest.mark.parametrize("prec", [1, 2])
def test_eo_lane_rhs_variants_agree(prec):
    """1, 2 and 4 right-hand sides per lane, a lane per half-site or tiles
    with LDS-staged links: the same solutions."""
    import paper_1211_0126_amd as tq
    dims, kappa, mu, eps = LATTICES[1]
    U = make_gauge(dims, eps, 5)
    ctx = _ctx(dims, kappa, mu, U)
    p = tq.solve_params(prec=prec, tol=0.0, max_iter=5, rhs_block=8, solver=tq.SOLVER_CG_EO)
    out = []
    for tiles in (0, 1):
        tq.tm_set_eo_tiles(ctx, prec, tiles)
        for nr in (1, 2, 4):
            tq.tm_set_lane_rhs(ctx, prec, nr)
            sol, _, _ = tq.tsm_solve_batch(ctx, p, 3, list(range(8)))
            out.append(sol.cpu().numpy())
    for o in out[1:]:
        assert _rel(o, out[0]) < (1e-6 if prec == 1 else 1e-3)
    ctx.close()


@pytest.mark.parametrize("tiles", [0, 1])
def test_eo_batching_does_not_change_a_source(tiles):
    import torch
    import paper_1211_0126_amd as tq
    dims = (4, 4, 4, 8)
    U = make_gauge(dims, 0.25, 77)
    ctx = _ctx(dims, 0.1632, 0.004, U)
    tq.tm_set_eo_tiles(ctx, tq.PREC_F16, tiles)
    p = tq.solve_params(prec=tq.PREC_F16, tol=1e-2, max_iter=-1, rhs_block=8, solver=tq.SOLVER_CG_EO)
    a, _, _ = tq.tsm_solve_batch(ctx, p, 3, list(range(8)))
    b, _, _ = tq.tsm_solve_batch(ctx, p, 3, [4, 5, 6, 7, 0, 1, 2, 3])
    assert torch.equal(a[:4], b[4:]) and torch.equal(a[4:], b[:4])
    ctx.close()


def test_eo_odd_extent_refused():
    import paper_1211_0126_amd as tq
    dims = (4, 4, 4, 6)
    U = make_gauge((3, 4, 4, 6), 0.25, 1)
    ctx = _ctx((3, 4, 4, 6), 0.1632, 0.004, U)
    p = tq.solve_params(prec=tq.PREC_F32, tol=1e-2, max_iter=-1, solver=tq.SOLVER_CG_EO)
    with pytest.raises(tq.TmError) as ei:
        tq.tsm_solve_batch(ctx, p, 1, [0])
    assert ei.value.code == -5
    ctx.close()


def test_eo_tsm_config0_matches_oracle(orc):
    """The 4^4 estimate of Eq. 4 with even-odd LP and HP solves in FP64."""
    import paper_1211_0126_amd as tq
    C0 = get_workload("c0")
    U = make_gauge(C0.dims, C0.eps, C0.gauge_seed)
    ctx = _ctx(C0.dims, C0.kappa, C0.mu, U)
    lp = tq.solve_params(prec=tq.PREC_F64, tol=C0.lp_tol, max_iter=C0.lp_maxit, rhs_block=4,
                         solver=tq.SOLVER_CG_EO)
    hp = tq.solve_params(prec=tq.PREC_F64, tol=C0.hp_tol, max_iter=-1, rhs_block=4, solver=tq.SOLVER_CG_EO)
    mom = C0.momenta()
    res = tq.tsm_loops(ctx, C0.noise_seed, C0.n_hp, C0.n_lp, lp, hp, mom, per_source=True)
    ref = orc.tsm(C0.dims, -1, C0.kappa, C0.mu, U, C0.noise_seed, C0.n_hp, C0.n_lp, C0.lp_tol, C0.lp_maxit,
                  C0.hp_tol, -1, mom, per_source=True, lp_eo=True, hp_eo=True)
    scale = np.max(np.abs(ref["loops"]))
    assert np.max(np.abs(res["loops"] - ref["loops"])) < 1e-10 * scale
    assert np.max(np.abs(res["per_source"] - ref["per_source"])) < 1e-10 * np.max(np.abs(ref["per_source"]))
    for j in range(C0.n_hp + C0.n_lp):
        assert res["stats"][j][0]["iters"] == int(ref["stats"][j][0][0])
    ctx.close()


@pytest.mark.parametrize("tiles", [0, 1])
def test_eo_tsm_27_momenta_fp32(orc, tiles):
    """Even-odd FP32 LP and reliable HP solves through the whole estimate on
    an anisotropic lattice at 27 momenta, against the oracle's even-odd
    FP64 TSM (LP truncated by iteration count, so both sides take the same
    iterate up to FP32 rounding)."""
    import paper_1211_0126_amd as tq
    dims, kappa, mu = (4, 6, 4, 8), 0.1632, 0.004
    U = make_gauge(dims, 0.25, 88)
    ctx = _ctx(dims, kappa, mu, U)
    tq.tm_set_eo_tiles(ctx, tq.PREC_F32, tiles)
    lp = tq.solve_params(prec=tq.PREC_F32, tol=0.0, max_iter=6, rhs_block=4, solver=tq.SOLVER_CG_EO)
    hp = tq.solve_params(prec=tq.PREC_F32, tol=1e-10, max_iter=-1, reliable=1, delta=0.1, rhs_block=4,
                         solver=tq.SOLVER_CG_EO)
    mom = momenta_27()
    res = tq.tsm_loops(ctx, 5, 2, 6, lp, hp, mom, per_source=True)
    ref = orc.tsm(dims, -1, kappa, mu, U, 5, 2, 6, 0.0, 6, 1e-10, -1, mom, per_source=True, lp_eo=True,
                  hp_eo=True)
    scale = np.max(np.abs(ref["per_source"]))
    assert np.max(np.abs(res["per_source"] - ref["per_source"])) < 1e-4 * scale
    assert np.max(np.abs(res["loops"] - ref["loops"])) < 1e-4 * np.max(np.abs(ref["loops"]))
    ctx.close()


@pytest.mark.parametrize("lp_iters", [6, 20])
def test_eo_tsm_fp16_lp_brick_lattice(orc, lp_iters):
    """FP16 LP solves on the brick-order lattice through the whole estimate:
    the standard loop then contracts the two FP16 halves of each LP solution
    (no full field is formed; with 20 iterations the solution is formed from
    the kept directions twice in FP32 before the last pass writes it in
    FP16); against the oracle's even-odd FP64 TSM with the same truncation,
    to FP16 storage rounding."""
    import paper_1211_0126_amd as tq
    dims, kappa, mu, eps = LATTICES[4]
    U = make_gauge(dims, eps, 91)
    ctx = _ctx(dims, kappa, mu, U)
    lp = tq.solve_params(prec=tq.PREC_F16, tol=0.0, max_iter=lp_iters, rhs_block=4, solver=tq.SOLVER_CG_EO)
    hp = tq.solve_params(prec=tq.PREC_F16, tol=1e-10, max_iter=-1, reliable=1, delta=1e-2, rhs_block=2,
                         solver=tq.SOLVER_CG_EO)
    mom = momenta_27()
    res = tq.tsm_loops(ctx, 7, 2, 6, lp, hp, mom, per_source=True)
    ref = orc.tsm(dims, -1, kappa, mu, U, 7, 2, 6, 0.0, lp_iters, 1e-10, -1, mom, per_source=True, lp_eo=True,
                  hp_eo=True)
    scale = np.max(np.abs(ref["per_source"]))
    dev = np.max(np.abs(res["per_source"] - ref["per_source"])) / scale
    print("FP16 LP per-source loops: max deviation %.3g of the largest" % dev)
    assert dev < 2e-2
    ctx.close()


@pytest.mark.parametrize("prec", [1, 2])
def test_eo_long_truncated_solve_ring_flushes(orc, prec):
    """FP32 / FP16 Schur CG truncated at 20 iterations (the search
    directions sit in a ring of 8 and the solution is formed from them every
    7 iterations): the same iterate as the FP64 oracle's to FP32 / FP16
    rounding, for sources of a block that stop at different counts."""
    import paper_1211_0126_amd as tq
    dims, kappa, mu, eps = LATTICES[1]
    U = make_gauge(dims, eps, 61)
    ctx = _ctx(dims, kappa, mu, U)
    ids = [0, 1, 2, 3]
    p = tq.solve_params(prec=prec, tol=0.0, max_iter=20, rhs_block=4, solver=tq.SOLVER_CG_EO)
    sol, st, _ = tq.tsm_solve_batch(ctx, p, 23, ids)
    sol = sol.cpu().numpy()
    for i, j in enumerate(ids):
        eta = orc.noise_z4(dims, 23, j)
        x, so = orc.cgnr_eo(dims, -1, kappa, mu, U, eta, 0.0, 20)
        assert st[i]["iters"] == 20
        assert _rel(sol[i], x) < (1e-4 if prec == 1 else 2e-2), (prec, j, _rel(sol[i], x))
    # sources that stop early (tolerance) next to ones that run on
    p2 = tq.solve_params(prec=prec, tol=1e-4, max_iter=-1, rhs_block=4, solver=tq.SOLVER_CG_EO)
    sol2, st2, _ = tq.tsm_solve_batch(ctx, p2, 23, ids)
    sol2 = sol2.cpu().numpy()
    for i, j in enumerate(ids):
        eta = orc.noise_z4(dims, 23, j)
        x, so = orc.cgnr_eo(dims, -1, kappa, mu, U, eta, 1e-4)
        assert st2[i]["converged"] and abs(st2[i]["iters"] - so["iters"]) <= 1
        assert st2[i]["resid_true"] < 2 * so["resid_true"] + (0 if prec == 1 else 1e-3)
    ctx.close()
