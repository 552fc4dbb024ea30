"""The 16^3x32 workload end to end in FP32 (27 momenta, antiperiodic time),
with the two truncations of the LP solves of section 2.2: by the residual
(1e-2, capped at 50 iterations) and by a fixed number of iterations.  The
FP32 estimate is compared with the FP64 oracle's on the same sources."""

import numpy as np
import pytest

from lattice_inputs import make_gauge
from lattice_inputs.workloads import get_workload

pytestmark = pytest.mark.gpu

C1 = get_workload("c1")
N_HP, N_LP = 1, 4


@pytest.fixture(scope="module")
def gauge():
    return make_gauge(C1.dims, C1.eps, C1.gauge_seed)


@pytest.mark.parametrize("lp_tol,lp_maxit", [(1e-2, 50), (0.0, 12)])
def test_config1_fp32_tsm_matches_oracle(orc, gauge, lp_tol, lp_maxit):
    import paper_1211_0126_amd as tq
    mom = C1.momenta()
    ctx = tq.tm_create(C1.dims, C1.kappa, C1.mu, -1)
    tq.tm_gauge_load(ctx, gauge)
    lp = tq.solve_params(prec=tq.PREC_F32, tol=lp_tol, max_iter=lp_maxit, rhs_block=4)
    hp = tq.solve_params(prec=tq.PREC_F32, tol=C1.hp_tol, max_iter=-1, reliable=1, delta=0.1, rhs_block=1)
    print("config 1 GPU, LP tol %g cap %d" % (lp_tol, lp_maxit), flush=True)
    res = tq.tsm_loops(ctx, C1.noise_seed, N_HP, N_LP, lp, hp, mom, per_source=True)
    ctx.close()
    print("config 1 oracle", flush=True)
    ref = orc.tsm(C1.dims, -1, C1.kappa, C1.mu, gauge, C1.noise_seed, N_HP, N_LP, lp_tol, lp_maxit, C1.hp_tol,
                  -1, mom, per_source=True)
    for j in range(N_HP + N_LP):
        gi, oi = res["stats"][j][0]["iters"], int(ref["stats"][j][0][0])
        assert gi == oi, (j, gi, oi)
        if lp_tol == 0.0:
            assert res["stats"][j][0]["truncated"] and gi == lp_maxit
    dev = np.max(np.abs(res["loops"] - ref["loops"])) / np.max(np.abs(ref["loops"]))
    dps = np.max(np.abs(res["per_source"] - ref["per_source"])) / np.max(np.abs(ref["per_source"]))
    print("config 1 TSM deviation %.3g, per-source %.3g" % (dev, dps))
    assert dev < 1e-4 and dps < 1e-4
