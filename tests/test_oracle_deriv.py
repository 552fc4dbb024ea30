"""Oracle pins for the one-derivative loops psibar Gamma Dsym_mu psi.

The loop of a source is eta^dag K s with
    K = (1/4) (P Gamma F - F^dag P Gamma),   F = U_mu T_{+mu} - U_mu^dag T_{-mu},
P the diagonal timeslice-and-phase projector and T the shifts (with the time
boundary factor).  The pins build K densely here, with numpy, straight from
the link array, and compare
 - the sum over a complete set of unit sources (exact solutions from LAPACK)
   with Tr[K M^{-1}], on lattices whose extents are all >= 3 (forward and
   backward neighbours distinct) and on a 2^4 lattice;
 - the TSM driver with the derivative estimator against the per-source
   loops.
"""

import numpy as np
import pytest

from lattice_inputs import make_gauge
from lattice_inputs.workloads import momenta_27
from dense import coords, dense_op, big_gamma_numpy

KAPPA, MU = 0.16, 0.03125


def dense_shift_covariant(dims, U, mu, t_bc):
    """F = U_mu(x) psi(x+mu) - U_mu(x-mu)^dag psi(x-mu) as a dense matrix."""
    v = int(np.prod(dims))
    x, y, z, t = coords(dims)
    c = np.stack([x, y, z, t], axis=1)
    U = np.asarray(U).reshape(v, 4, 3, 3)
    F = np.zeros((12 * v, 12 * v), dtype=np.complex128)

    def site(cc):
        return cc[0] + dims[0] * (cc[1] + dims[1] * (cc[2] + dims[2] * cc[3]))

    for s in range(v):
        for d in (+1, -1):
            cc = c[s].copy()
            cc[mu] += d
            ph = 1.0
            if cc[mu] == dims[mu] or cc[mu] < 0:
                cc[mu] %= dims[mu]
                if mu == 3:
                    ph = t_bc
            nb = site(cc)
            link = U[s, mu] if d > 0 else U[nb, mu].conj().T
            for a in range(4):
                F[12 * s + 3 * a:12 * s + 3 * a + 3, 12 * nb + 3 * a:12 * nb + 3 * a + 3] += d * ph * link
    return F


def exact_deriv_loops(dims, U, Minv, mom, t_bc=-1):
    """Tr[K M^{-1}] = (1/4) sum_x d_x (tr[Gs (F M^-1)_xx] - tr[Gs (M^-1 F^dag)_xx])
    with Gs = Gamma_n (x) 1_colour and (.)_xx the 12x12 site-diagonal block."""
    v = int(np.prod(dims))
    x, y, z, t = coords(dims)
    mom = np.asarray(mom).reshape(-1, 3)
    out = np.zeros((4, 16, len(mom), dims[3]), dtype=np.complex128)
    idx = np.arange(v)
    for mu in range(4):
        F = dense_shift_covariant(dims, U, mu, t_bc)
        A = (F @ Minv).reshape(v, 12, v, 12)[idx, :, idx, :]            # [x][12][12]
        B = (Minv @ F.conj().T).reshape(v, 12, v, 12)[idx, :, idx, :]
        for n in range(16):
            Gs = np.kron(big_gamma_numpy(n), np.eye(3))
            site = 0.25 * (np.einsum("ij,xji->x", Gs, A) - np.einsum("ij,xji->x", Gs, B))
            for m, (nx, ny, nz) in enumerate(mom):
                ph = np.exp(-2j * np.pi * (nx * x / dims[0] + ny * y / dims[1] + nz * z / dims[2]))
                np.add.at(out[mu, n, m], t, ph * site)
    return out


def unit_sum(orc, dims, U, Minv, mom):
    v = int(np.prod(dims))
    tot = np.zeros((4, 16, len(mom), dims[3]), dtype=np.complex128)
    for i in range(12 * v):
        e = np.zeros(12 * v, dtype=np.complex128)
        e[i] = 1
        tot += orc.loops_deriv(dims, -1, U, e.reshape(v, 4, 3), Minv[:, i].reshape(v, 4, 3), mom)
    return tot


@pytest.mark.parametrize("dims,mom", [((3, 3, 3, 4), [(0, 0, 0), (1, 0, 0), (0, -1, 1)]),
                                      ((2, 2, 2, 2), [(0, 0, 0), (1, 1, 0)])])
def test_unit_sources_give_exact_trace(orc, dims, mom):
    U = make_gauge(dims, 0.3, 91)
    Minv = np.linalg.inv(dense_op(dims, -1, KAPPA, MU, U, orc.OP_M))
    mom = np.asarray(mom, dtype=np.int32)
    ex = exact_deriv_loops(dims, U, Minv, mom)
    tot = unit_sum(orc, dims, U, Minv, mom)
    scale = np.max(np.abs(ex))
    assert scale > 1e-3
    assert np.max(np.abs(tot - ex)) < 1e-12 * scale
    # every direction contributes (a dropped or swapped hop would show here)
    for mu in range(4):
        assert np.max(np.abs(ex[mu])) > 1e-2 * scale


def test_tsm_with_derivative_estimator(orc):
    dims = (2, 2, 2, 4)
    U = make_gauge(dims, 0.3, 1000)
    mom = momenta_27()
    res = orc.tsm(dims, -1, KAPPA, MU, U, 42, 2, 3, 1e-2, -1, 1e-12, -1, mom, per_source=True,
                  estimator=orc.LOOP_DERIV)
    ps = res["per_source"]
    assert ps.shape == (5, 2, 4, 16, 27, 4)
    assert np.allclose(res["loops"][0], (ps[:2, 1] - ps[:2, 0]).mean(axis=0), rtol=1e-13, atol=1e-13)
    assert np.allclose(res["loops"][1], ps[2:, 0].mean(axis=0), rtol=1e-13, atol=1e-13)
    eta = orc.noise_z4(dims, 42, 3)
    s, _ = orc.cgnr(dims, -1, KAPPA, MU, U, eta, 1e-2)
    assert np.allclose(ps[3, 0], orc.loops_deriv(dims, -1, U, eta, s, mom), atol=1e-13)
