"""GPU parity of the one-derivative loops psibar Gamma Dsym_mu psi against the
FP64 CPU oracle, through the C ABI: the contraction of given solutions on
lattices of one to several contraction blocks, the TSM estimate of Eq. 4
with the derivative estimator, FP32 solutions and the argument checks."""

import numpy as np
import pytest

from lattice_inputs import make_gauge
from lattice_inputs.workloads import momenta_27, get_workload

pytestmark = pytest.mark.gpu

C0 = get_workload("c0")


def _ctx(dims, kappa, mu, U):
    import paper_1211_0126_amd as tq
    ctx = tq.tm_create(dims, kappa, mu, -1)
    tq.tm_gauge_load(ctx, U)
    return ctx


@pytest.mark.parametrize("dims,mom,kind", [((4, 4, 4, 4), "p0", "cg"), ((2, 4, 6, 8), "p27", "cg"),
                                           ((4, 6, 4, 8), "p27", "rand"), ((16, 8, 8, 16), "p27", "rand")])
def test_deriv_contract_matches_oracle(orc, dims, mom, kind):
    """Same sources and solutions: every direction's loops agree to 1e-8 of
    the largest element; an extent of 2 (forward and backward neighbours
    the same site), odd multiples of the block size and a ragged last
    block."""
    import torch
    import paper_1211_0126_amd as tq
    kappa, mu = 0.1632, 0.004
    U = make_gauge(dims, 0.3, 23)
    ctx = _ctx(dims, kappa, mu, U)
    moms = np.zeros((1, 3), np.int32) if mom == "p0" else momenta_27()
    ids = [0, 1, 9]
    if kind == "cg":
        sols = np.stack([orc.cgnr(dims, -1, kappa, mu, U, orc.noise_z4(dims, 5, j), 1e-3)[0] for j in ids])
    else:
        rng = np.random.default_rng(4321)
        v = int(np.prod(dims))
        sols = rng.standard_normal((3, v, 4, 3)) + 1j * rng.standard_normal((3, v, 4, 3))
    print("deriv contract dims=%s mom=%s kind=%s" % (dims, mom, kind), flush=True)
    got = tq.tsm_contract(ctx, 5, ids, torch.from_numpy(sols).cuda(), moms, estimator=tq.LOOP_DERIVATIVE)
    assert got.shape == (3, 4, 16, len(moms), dims[3])
    for i, j in enumerate(ids):
        ref = orc.loops_deriv(dims, -1, U, orc.noise_z4(dims, 5, j), sols[i], moms)
        assert np.max(np.abs(got[i] - ref)) <= 1e-8 * np.max(np.abs(ref)), i
    ctx.close()


def test_deriv_tsm_config0_matches_oracle(orc):
    import paper_1211_0126_amd as tq
    U = make_gauge(C0.dims, C0.eps, C0.gauge_seed)
    ctx = _ctx(C0.dims, C0.kappa, C0.mu, U)
    lp = tq.solve_params(prec=tq.PREC_F64, tol=C0.lp_tol, max_iter=C0.lp_maxit, rhs_block=4)
    hp = tq.solve_params(prec=tq.PREC_F64, tol=C0.hp_tol, max_iter=-1, rhs_block=4)
    mom = C0.momenta()
    print("deriv tsm c0", flush=True)
    res = tq.tsm_loops(ctx, C0.noise_seed, C0.n_hp, C0.n_lp, lp, hp, mom, per_source=True,
                       estimator=tq.LOOP_DERIVATIVE)
    ref = orc.tsm(C0.dims, -1, C0.kappa, C0.mu, U, C0.noise_seed, C0.n_hp, C0.n_lp, C0.lp_tol, C0.lp_maxit,
                  C0.hp_tol, -1, mom, per_source=True, estimator=orc.LOOP_DERIV)
    assert res["loops"].shape == ref["loops"].shape
    scale = np.max(np.abs(ref["loops"]))
    assert np.max(np.abs(res["loops"] - ref["loops"])) < 1e-10 * scale
    assert np.max(np.abs(res["err"] - ref["err"])) < 1e-8 * np.max(np.abs(ref["err"]))
    assert np.max(np.abs(res["per_source"] - ref["per_source"])) < 1e-10 * np.max(np.abs(ref["per_source"]))
    ctx.close()


def test_deriv_fp32_solutions(orc):
    """FP32 LP solves with a fixed iteration count, contracted from their
    FP32 solutions: agreement to 1e-4 (FP32 against FP64 CG iterates)."""
    import paper_1211_0126_amd as tq
    dims = (8, 8, 8, 8)
    kappa, mu = 0.1632, 0.004
    U = make_gauge(dims, 0.25, 5)
    ctx = _ctx(dims, kappa, mu, U)
    k = 12
    lp = tq.solve_params(prec=tq.PREC_F32, tol=0.0, max_iter=k, rhs_block=4)
    hp = tq.solve_params(prec=tq.PREC_F64, tol=1e-10, max_iter=-1, rhs_block=4)
    mom = momenta_27()
    print("deriv fp32 solutions", flush=True)
    res = tq.tsm_loops(ctx, 77, 0, 5, lp, hp, mom, per_source=True, estimator=tq.LOOP_DERIVATIVE)
    for j in range(5):
        eta = orc.noise_z4(dims, 77, j)
        x, _ = orc.cgnr(dims, -1, kappa, mu, U, eta, 0.0, k)
        ref = orc.loops_deriv(dims, -1, U, eta, x, mom)
        assert np.max(np.abs(res["per_source"][j, 0] - ref)) < 1e-4 * np.max(np.abs(ref)), j
    ctx.close()


def test_deriv_argument_checks():
    import torch
    import paper_1211_0126_amd as tq
    ctx = tq.tm_create((4, 4, 4, 4), 0.16, 0.03, -1)
    sol = torch.zeros((1, 256, 4, 3), dtype=torch.complex128, device="cuda")
    mom = np.zeros((1, 3), np.int32)
    with pytest.raises(tq.TmError) as e:
        tq.tsm_contract(ctx, 0, None, sol, mom, estimator=tq.LOOP_DERIVATIVE)  # needs the sources
    assert e.value.code == -1
    with pytest.raises(tq.TmError) as e:
        tq.tsm_contract(ctx, 0, [0], sol, mom, estimator=tq.LOOP_DERIVATIVE)   # no gauge field yet
    assert e.value.code == -4
    ctx.close()
