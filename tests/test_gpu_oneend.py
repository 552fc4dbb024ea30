"""GPU parity of the one-end-trick loops (section 2.3, Eqs. 5 and 6) against
the FP64 CPU oracle, through the C ABI: the contraction of given solutions,
the whole TSM estimate of Eq. 4 with each estimator, the FP32-solution path
and the argument checks."""

import numpy as np
import pytest

from lattice_inputs import make_gauge
from lattice_inputs.workloads import momenta_27, get_workload

pytestmark = pytest.mark.gpu

C0 = get_workload("c0")
ESTS = [1, 2]


def _ctx(dims, kappa, mu, U):
    import paper_1211_0126_amd as tq
    ctx = tq.tm_create(dims, kappa, mu, -1)
    tq.tm_gauge_load(ctx, U)
    return ctx


def _spinors(dims, n, seed):
    rng = np.random.default_rng(seed)
    v = int(np.prod(dims))
    return (rng.standard_normal((n, v, 4, 3)) + 1j * rng.standard_normal((n, v, 4, 3))).astype(np.complex128)


@pytest.mark.parametrize("est", ESTS)
@pytest.mark.parametrize("dims,mom,kind", [((4, 4, 4, 4), "p0", "cg"), ((2, 4, 6, 8), "p27", "cg"),
                                           ((8, 6, 4, 6), "p27", "rand"), ((16, 8, 8, 16), "p27", "rand")])
def test_oneend_contract_matches_oracle(orc, est, dims, mom, kind):
    """Same solutions on both sides: the one-end loops agree to 1e-8 of their
    largest element.  Lattices from one to several contraction blocks with a
    ragged last block; CG solutions and arbitrary spinors (the estimator is a
    bilinear of any field)."""
    import torch
    import paper_1211_0126_amd as tq
    kappa, mu = 0.1632, 0.004
    U = make_gauge(dims, 0.3, 21)
    ctx = _ctx(dims, kappa, mu, U)
    moms = np.zeros((1, 3), np.int32) if mom == "p0" else momenta_27()
    if kind == "cg":
        sols = np.stack([orc.cgnr(dims, -1, kappa, mu, U, orc.noise_z4(dims, 5, j), 1e-3)[0] for j in (0, 1, 9)])
    else:
        sols = _spinors(dims, 3, 1234 + est)
    print("one-end contract est=%d dims=%s mom=%s kind=%s" % (est, dims, mom, kind), flush=True)
    got = tq.tsm_contract(ctx, 0, None, torch.from_numpy(sols).cuda(), moms, estimator=est)
    for i in range(len(sols)):
        ref = orc.loops_est(dims, -1, kappa, mu, U, est, sols[i], moms)
        assert np.max(np.abs(got[i] - ref)) <= 1e-8 * np.max(np.abs(ref)), i
    ctx.close()


@pytest.mark.parametrize("est", ESTS)
def test_oneend_tsm_config0_matches_oracle(orc, est):
    """The TSM estimate of Eq. 4 with a one-end estimator at the 4^4 workload
    in FP64: totals, errors and every per-source loop."""
    import paper_1211_0126_amd as tq
    U = make_gauge(C0.dims, C0.eps, C0.gauge_seed)
    ctx = _ctx(C0.dims, C0.kappa, C0.mu, U)
    lp = tq.solve_params(prec=tq.PREC_F64, tol=C0.lp_tol, max_iter=C0.lp_maxit, rhs_block=4)
    hp = tq.solve_params(prec=tq.PREC_F64, tol=C0.hp_tol, max_iter=-1, rhs_block=4)
    mom = C0.momenta()
    print("one-end tsm c0 est=%d" % est, flush=True)
    res = tq.tsm_loops(ctx, C0.noise_seed, C0.n_hp, C0.n_lp, lp, hp, mom, per_source=True, estimator=est)
    ref = orc.tsm(C0.dims, -1, C0.kappa, C0.mu, U, C0.noise_seed, C0.n_hp, C0.n_lp, C0.lp_tol, C0.lp_maxit,
                  C0.hp_tol, -1, mom, per_source=True, estimator=est)
    scale = np.max(np.abs(ref["loops"]))
    assert np.max(np.abs(res["loops"] - ref["loops"])) < 1e-10 * scale
    assert np.max(np.abs(res["err"] - ref["err"])) < 1e-8 * np.max(np.abs(ref["err"]))
    assert np.max(np.abs(res["per_source"] - ref["per_source"])) < 1e-10 * np.max(np.abs(ref["per_source"]))
    ctx.close()


@pytest.mark.parametrize("est", ESTS)
def test_oneend_fp32_solutions(orc, est):
    """LP solves in FP32 storage and arithmetic, stopped after a fixed number
    of iterations, contracted from their FP32 solutions (the generalized loop
    forms D s in FP32 on the FP32 links).  FP32 CG iterates differ from the
    FP64 ones by about k * 1e-7 * cond, so the per-source loops agree to
    1e-4."""
    import paper_1211_0126_amd as tq
    dims = (8, 8, 8, 8)
    kappa, mu = 0.1632, 0.004
    U = make_gauge(dims, 0.25, 5)
    ctx = _ctx(dims, kappa, mu, U)
    k = 12
    lp = tq.solve_params(prec=tq.PREC_F32, tol=0.0, max_iter=k, rhs_block=4)
    hp = tq.solve_params(prec=tq.PREC_F64, tol=1e-10, max_iter=-1, rhs_block=4)
    mom = momenta_27()
    print("one-end fp32 solutions est=%d" % est, flush=True)
    res = tq.tsm_loops(ctx, 77, 0, 6, lp, hp, mom, per_source=True, estimator=est)
    for j in range(6):
        x, _ = orc.cgnr(dims, -1, kappa, mu, U, orc.noise_z4(dims, 77, j), 0.0, k)
        ref = orc.loops_est(dims, -1, kappa, mu, U, est, x, mom)
        got = res["per_source"][j, 0]
        assert np.max(np.abs(got - ref)) < 1e-4 * np.max(np.abs(ref)), j
    ctx.close()


def test_oneend_argument_checks():
    import torch
    import paper_1211_0126_amd as tq
    dims = (4, 4, 4, 4)
    ctx = tq.tm_create(dims, 0.16, 0.03, -1)
    sol = torch.zeros((1, 256, 4, 3), dtype=torch.complex128, device="cuda")
    mom = np.zeros((1, 3), np.int32)
    with pytest.raises(tq.TmError) as e:
        tq.tsm_contract(ctx, 0, None, sol, mom, estimator=3)
    assert e.value.code == -1
    with pytest.raises(tq.TmError) as e:
        tq.tsm_contract(ctx, 0, None, sol, mom, estimator=0)   # the standard loop needs ids
    assert e.value.code == -1
    with pytest.raises(tq.TmError) as e:
        tq.tsm_contract(ctx, 0, None, sol, mom, estimator=2)   # no gauge field yet
    assert e.value.code == -4
    # the isovector loop of a zero field is zero, with or without links
    out = tq.tsm_contract(ctx, 0, None, sol, mom, estimator=1)
    assert np.all(out == 0)
    ctx.close()
