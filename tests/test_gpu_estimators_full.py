"""One-end loops (Eqs. 5 and 6) on the full 32^3 x 64 lattice of the
benchmark, checked against the oracle one timeslice at a time.

A field that vanishes outside one timeslice t0 has one-end loops only at
t0, and there they depend only on the field and the links of that
timeslice (the isovector loop is site-local; the generalized one applies D,
whose time hops from t0 land on zeros).  So the oracle computes the same
numbers on a 32^3 x 2 lattice holding that timeslice, which it finishes in
seconds, while the library contracts on the whole lattice with the grid of
the benchmark size."""

import numpy as np
import pytest

from lattice_inputs import make_gauge
from lattice_inputs.workloads import momenta_27

pytestmark = pytest.mark.gpu

DIMS = (32, 32, 32, 64)
KAPPA, MU = 0.1632, 0.003


@pytest.fixture(scope="module")
def gauge():
    return make_gauge(DIMS, 0.25, 1003)


@pytest.mark.parametrize("est", [1, 2])
def test_one_end_loops_full_lattice(orc, gauge, est):
    import torch
    import paper_1211_0126_amd as tq
    vs = DIMS[0] * DIMS[1] * DIMS[2]
    slices = (0, 37)
    rng = np.random.default_rng(808 + est)
    fields = np.zeros((len(slices), DIMS[3], vs, 4, 3), dtype=np.complex128)
    for i, t0 in enumerate(slices):
        fields[i, t0] = rng.standard_normal((vs, 4, 3)) + 1j * rng.standard_normal((vs, 4, 3))
    ctx = tq.tm_create(DIMS, KAPPA, MU, -1, caps=tq.caps([], max_sources=len(slices), estimators=(est,)))
    tq.tm_gauge_load(ctx, gauge)
    mom = momenta_27()
    print("full-lattice one-end est=%d" % est, flush=True)
    sol = torch.from_numpy(fields.reshape(len(slices), -1, 4, 3)).cuda()
    got = tq.tsm_contract(ctx, 0, None, sol, mom, estimator=est)
    ctx.close()
    del sol
    Ug = np.asarray(gauge).reshape(DIMS[3], vs, 4, 3, 3)
    small = DIMS[:3] + (2,)
    for i, t0 in enumerate(slices):
        Us = np.stack([Ug[t0], Ug[(t0 + 1) % DIMS[3]]]).reshape(-1, 4, 3, 3)
        ss = np.stack([fields[i, t0], np.zeros_like(fields[i, t0])]).reshape(-1, 4, 3)
        ref = orc.loops_est(small, -1, KAPPA, MU, Us, est, ss, mom)[:, :, 0]
        scale = np.max(np.abs(ref))
        assert np.max(np.abs(got[i][:, :, t0] - ref)) <= 1e-8 * scale, t0
        others = np.delete(got[i], t0, axis=2)
        assert np.max(np.abs(others)) <= 1e-12 * scale
