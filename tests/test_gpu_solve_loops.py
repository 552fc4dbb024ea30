"""GPU parity: CG solves, loop contractions and the TSM estimate of Eq. 4
against the FP64 CPU oracle, through the C ABI."""

import numpy as np
import pytest

from lattice_inputs import make_gauge
from lattice_inputs.workloads import momenta_27, get_workload

pytestmark = pytest.mark.gpu


def _ctx(dims, kappa, mu, U):
    import paper_1211_0126_amd as tq
    ctx = tq.tm_create(dims, kappa, mu, -1)
    tq.tm_gauge_load(ctx, U)
    return ctx


def _rel(a, b):
    return np.linalg.norm((a - b).ravel()) / np.linalg.norm(b.ravel())


C0 = get_workload("c0")


@pytest.fixture(scope="module")
def c0():
    U = make_gauge(C0.dims, C0.eps, C0.gauge_seed)
    return U


def test_fp64_truncated_solve_matches_oracle(orc, c0):
    """Truncation by iteration count: the same iterate on both sides."""
    import paper_1211_0126_amd as tq
    ctx = _ctx(C0.dims, C0.kappa, C0.mu, c0)
    ids = [0, 3, 5]
    for k in (0, 1, 5, 17):
        p = tq.solve_params(prec=tq.PREC_F64, tol=0.0, max_iter=k, rhs_block=2)
        sol, st, rc = tq.tsm_solve_batch(ctx, p, C0.noise_seed, ids)
        sol = sol.cpu().numpy()
        for i, j in enumerate(ids):
            eta = orc.noise_z4(C0.dims, C0.noise_seed, j)
            x, so = orc.cgnr(C0.dims, -1, C0.kappa, C0.mu, c0, eta, 0.0, k)
            assert st[i]["iters"] == k and st[i]["truncated"] == (True)
            if k == 0:
                assert np.all(sol[i] == 0)
            else:
                assert _rel(sol[i], x) < 1e-12, (k, j, _rel(sol[i], x))
            assert abs(st[i]["resid_true"] - so["resid_true"]) < 1e-10
    ctx.close()


def test_fp64_converged_solves(orc, c0):
    import paper_1211_0126_amd as tq
    ctx = _ctx(C0.dims, C0.kappa, C0.mu, c0)
    ids = list(range(5))
    for tol in (1e-2, 1e-12):
        p = tq.solve_params(prec=tq.PREC_F64, tol=tol, max_iter=-1, rhs_block=4)
        sol, st, rc = tq.tsm_solve_batch(ctx, p, C0.noise_seed, ids)
        sol = sol.cpu().numpy()
        for i, j in enumerate(ids):
            eta = orc.noise_z4(C0.dims, C0.noise_seed, j)
            x, so = orc.cgnr(C0.dims, -1, C0.kappa, C0.mu, c0, eta, tol)
            assert st[i]["converged"] and abs(st[i]["iters"] - so["iters"]) <= 1
            assert st[i]["resid_iterated"] <= tol
            if st[i]["iters"] == so["iters"]:
                assert _rel(sol[i], x) < 1e-10
    ctx.close()


def test_true_residual_stop(orc, c0):
    import paper_1211_0126_amd as tq
    ctx = _ctx(C0.dims, C0.kappa, C0.mu, c0)
    p = tq.solve_params(prec=tq.PREC_F64, tol=1e-2, max_iter=-1, stop=tq.STOP_TRUE)
    sol, st, rc = tq.tsm_solve_batch(ctx, p, C0.noise_seed, [2])
    eta = orc.noise_z4(C0.dims, C0.noise_seed, 2)
    x, so = orc.cgnr(C0.dims, -1, C0.kappa, C0.mu, c0, eta, 1e-2, -1, orc.STOP_TRUE)
    assert st[0]["iters"] == so["iters"] and st[0]["resid_true"] <= 1e-2
    assert _rel(sol.cpu().numpy()[0], x) < 1e-12
    ctx.close()


@pytest.mark.parametrize("prec", [1, 2, 3])
def test_reduced_precision_lp_solve(orc, prec):
    """LP solves with FP32 / FP16 / BF16 storage reach the LP tolerance; the
    FP64 true residual is close to the FP64 oracle's at the same stop."""
    import paper_1211_0126_amd as tq
    dims = (8, 8, 8, 8)
    U = make_gauge(dims, 0.25, 1002)
    ctx = _ctx(dims, 0.1632, 0.004, U)
    ids = list(range(8))
    p = tq.solve_params(prec=prec, tol=1e-2, max_iter=-1, rhs_block=8)
    sol, st, rc = tq.tsm_solve_batch(ctx, p, 7, ids)
    for i, j in enumerate(ids):
        eta = orc.noise_z4(dims, 7, j)
        x, so = orc.cgnr(dims, -1, 0.1632, 0.004, U, eta, 1e-2)
        assert st[i]["converged"]
        assert abs(st[i]["iters"] - so["iters"]) <= 2
        assert st[i]["resid_true"] < 2 * so["resid_true"] + 1e-2
    ctx.close()


def test_fp32_reliable_hp_solve(orc):
    """FP32 iterations with FP64 reliable updates reach 1e-10 (normal
    equations) and agree with the FP64 oracle solution."""
    import paper_1211_0126_amd as tq
    dims = (8, 8, 8, 8)
    U = make_gauge(dims, 0.25, 1002)
    ctx = _ctx(dims, 0.1632, 0.004, U)
    ids = [0, 1, 2, 3]
    p = tq.solve_params(prec=tq.PREC_F32, tol=1e-10, max_iter=-1, reliable=1, delta=0.1, rhs_block=4)
    sol, st, rc = tq.tsm_solve_batch(ctx, p, 9, ids)
    sol = sol.cpu().numpy()
    for i, j in enumerate(ids):
        eta = orc.noise_z4(dims, 9, j)
        x, so = orc.cgnr(dims, -1, 0.1632, 0.004, U, eta, 1e-12)
        assert st[i]["converged"], st[i]
        assert st[i]["resid_iterated"] <= 1e-10
        assert _rel(sol[i], x) < 1e-8, _rel(sol[i], x)
    ctx.close()


def test_fp32_reliable_hp_true_residual_stop(orc):
    """FP32 iterations with FP64 reliable updates stopping on the FP64 true
    residual |eta - M x| / |eta| <= 1e-10 (taken at the updates): the
    reported and the independently recomputed true residuals meet the
    target, and the iteration count is the FP64 oracle's with the same stop
    to within a few iterations."""
    import paper_1211_0126_amd as tq
    dims = (8, 8, 8, 8)
    U = make_gauge(dims, 0.25, 1002)
    ctx = _ctx(dims, 0.1632, 0.004, U)
    ids = [0, 1, 2, 3]
    p = tq.solve_params(prec=tq.PREC_F32, tol=1e-10, max_iter=-1, reliable=1, delta=0.1, rhs_block=4,
                        stop=tq.STOP_TRUE)
    sol, st, rc = tq.tsm_solve_batch(ctx, p, 9, ids)
    sol = sol.cpu().numpy()
    for i, j in enumerate(ids):
        eta = orc.noise_z4(dims, 9, j)
        x, so = orc.cgnr(dims, -1, 0.1632, 0.004, U, eta, 1e-10, -1, orc.STOP_TRUE)
        mx = orc.apply_op(dims, -1, 0.1632, 0.004, orc.OP_M, U, sol[i])
        true = np.linalg.norm((eta - mx).ravel()) / np.linalg.norm(eta.ravel())
        print("source %d: iters %d (oracle %d), true residual %.3g (reported %.3g)"
              % (j, st[i]["iters"], so["iters"], true, st[i]["resid_true"]))
        assert st[i]["converged"], st[i]
        assert st[i]["resid_iterated"] <= 1e-10 and st[i]["resid_true"] <= 1e-10 and true <= 1.01e-10
        assert abs(st[i]["iters"] - so["iters"]) <= 3
    ctx.close()


def test_batching_does_not_change_a_source(c0):
    """Per-source arithmetic is independent of the other sources of a block:
    the same source solved in different blocks is bitwise identical."""
    import paper_1211_0126_amd as tq
    import torch
    dims = (4, 4, 4, 8)
    U = make_gauge(dims, 0.25, 77)
    ctx = _ctx(dims, 0.1632, 0.004, U)
    p = tq.solve_params(prec=tq.PREC_BF16, tol=1e-2, max_iter=-1, rhs_block=8)
    a, _, _ = tq.tsm_solve_batch(ctx, p, 3, list(range(8)))
    b, _, _ = tq.tsm_solve_batch(ctx, p, 3, [4, 5, 6, 7, 0, 1, 2, 3])
    assert torch.equal(a[:4], b[4:]) and torch.equal(a[4:], b[:4])
    ctx.close()


@pytest.mark.parametrize("dims,mom", [((4, 4, 4, 4), "p0"), ((2, 4, 6, 8), "p27"), ((8, 6, 4, 6), "p27")])
def test_contract_matches_oracle(orc, dims, mom):
    """Identical sources and solutions: loops agree to 1e-8 (normwise max)."""
    import torch
    import paper_1211_0126_amd as tq
    U = make_gauge(dims, 0.3, 21)
    ctx = _ctx(dims, 0.1632, 0.004, U)
    moms = np.zeros((1, 3), np.int32) if mom == "p0" else momenta_27()
    ids = [0, 1, 9]
    sols = []
    for j in ids:
        eta = orc.noise_z4(dims, 5, j)
        x, _ = orc.cgnr(dims, -1, 0.1632, 0.004, U, eta, 1e-3)
        sols.append(x)
    sol = torch.from_numpy(np.stack(sols)).cuda()
    got = tq.tsm_contract(ctx, 5, ids, sol, moms)
    for i, j in enumerate(ids):
        ref = orc.loops(dims, orc.noise_z4(dims, 5, j), sols[i], moms)
        assert np.max(np.abs(got[i] - ref)) <= 1e-8 * np.max(np.abs(ref))
    ctx.close()


def test_tsm_config0_matches_oracle(orc, c0):
    """The whole estimate of Eq. 4 at the 4^4 workload in FP64."""
    import paper_1211_0126_amd as tq
    ctx = _ctx(C0.dims, C0.kappa, C0.mu, c0)
    lp = tq.solve_params(prec=tq.PREC_F64, tol=C0.lp_tol, max_iter=C0.lp_maxit, rhs_block=4)
    hp = tq.solve_params(prec=tq.PREC_F64, tol=C0.hp_tol, max_iter=-1, rhs_block=4)
    mom = C0.momenta()
    res = tq.tsm_loops(ctx, C0.noise_seed, C0.n_hp, C0.n_lp, lp, hp, mom, per_source=True)
    ref = orc.tsm(C0.dims, -1, C0.kappa, C0.mu, c0, C0.noise_seed, C0.n_hp, C0.n_lp, C0.lp_tol, C0.lp_maxit,
                  C0.hp_tol, -1, mom, per_source=True)
    scale = np.max(np.abs(ref["loops"]))
    assert np.max(np.abs(res["loops"] - ref["loops"])) < 1e-10 * scale
    assert np.max(np.abs(res["err"] - ref["err"])) < 1e-8 * np.max(np.abs(ref["err"]))
    assert np.max(np.abs(res["per_source"] - ref["per_source"])) < 1e-10 * np.max(np.abs(ref["per_source"]))
    for j in range(C0.n_hp + C0.n_lp):
        assert res["stats"][j][0]["iters"] == int(ref["stats"][j][0][0])
    ctx.close()


def test_tsm_edge_cases(orc, c0):
    import paper_1211_0126_amd as tq
    ctx = _ctx(C0.dims, C0.kappa, C0.mu, c0)
    lp = tq.solve_params(prec=tq.PREC_F64, tol=0.0, max_iter=3, rhs_block=4)
    hp = tq.solve_params(prec=tq.PREC_F64, tol=1e-12, max_iter=-1, rhs_block=4)
    mom = np.zeros((1, 3), np.int32)
    for n_hp, n_lp in ((0, 5), (3, 0), (1, 1), (5, 7)):
        res = tq.tsm_loops(ctx, 11, n_hp, n_lp, lp, hp, mom)
        ref = orc.tsm(C0.dims, -1, C0.kappa, C0.mu, c0, 11, n_hp, n_lp, 0.0, 3, 1e-12, -1, mom)
        assert np.max(np.abs(res["loops"] - ref["loops"])) < 1e-10 * max(1.0, np.max(np.abs(ref["loops"])))
    # nothing at all
    res = tq.tsm_loops(ctx, 11, 0, 0, lp, hp, mom)
    assert np.all(res["loops"] == 0)
    ctx.close()
