"""Oracle pins for the one-end-trick loops (section 2.3, Eqs. 5 and 6).

 - a complete set of unit sources turns the isovector estimator into the exact
   difference Tr[X M_u^{-1}] - Tr[X M_d^{-1}] and the generalized one into the
   exact sum, per timeslice, momentum and Gamma, with M_d the operator at -mu
   and both inverses from LAPACK.  This fixes the overall factor, its sign, the
   gamma_5 placements and the D (not M) of Eq. 6.
 - the same holds on an anisotropic lattice (momentum sign and axis order).
 - with Z4 noise and exact solves both estimators are unbiased within their
   errors, and each isovector per-source value at p = 0 is purely real or
   purely imaginary as the hermiticity of g5 Gamma says.
 - the TSM driver with a one-end estimator combines the per-source one-end
   loops as Eq. 4 says.
"""

import numpy as np
import pytest

from lattice_inputs import make_gauge
from lattice_inputs.workloads import momenta_27
from dense import big_gamma_numpy, coords, dense_op, exact_loops

D2 = (2, 2, 2, 2)
KAPPA, MU = 0.16, 0.03125  # 2 kappa mu = 0.01


@pytest.fixture(scope="module")
def flavours(orc):
    U = make_gauge(D2, 0.3, 1000)
    Mu = dense_op(D2, -1, KAPPA, MU, U, orc.OP_M)
    Md = dense_op(D2, -1, KAPPA, -MU, U, orc.OP_M)
    return U, np.linalg.inv(Mu), np.linalg.inv(Md)


def _unit_sum(orc, dims, U, Minv, est, mom, kappa=KAPPA, mu=MU):
    v = int(np.prod(dims))
    tot = np.zeros((16, len(mom), dims[3]), dtype=np.complex128)
    for i in range(12 * v):
        tot += orc.loops_est(dims, -1, kappa, mu, U, est, Minv[:, i].reshape(v, 4, 3), mom)
    return tot


@pytest.mark.parametrize("est", [1, 2])
def test_unit_sources_give_exact_flavour_combination(orc, flavours, est):
    U, Miu, Mid = flavours
    mom = momenta_27()
    tot = _unit_sum(orc, D2, U, Miu, est, mom)
    eu, ed = exact_loops(D2, Miu, mom), exact_loops(D2, Mid, mom)
    ex = eu - ed if est == 1 else eu + ed
    scale = np.max(np.abs(ex))
    assert scale > 1e-3
    assert np.max(np.abs(tot - ex)) < 1e-12 * scale
    # the opposite sign (the printed one for Eq. 5) is far off
    if est == 1:
        assert np.max(np.abs(-tot - ex)) > 0.5 * scale


def test_unit_sources_anisotropic(orc):
    dims = (2, 4, 2, 4)
    U = make_gauge(dims, 0.3, 77)
    mu = 0.05
    Miu = np.linalg.inv(dense_op(dims, -1, KAPPA, mu, U, orc.OP_M))
    Mid = np.linalg.inv(dense_op(dims, -1, KAPPA, -mu, U, orc.OP_M))
    mom = momenta_27()
    eu, ed = exact_loops(dims, Miu, mom), exact_loops(dims, Mid, mom)
    for est, ex in ((1, eu - ed), (2, eu + ed)):
        tot = _unit_sum(orc, dims, U, Miu, est, mom, mu=mu)
        assert np.max(np.abs(tot - ex)) < 1e-12 * np.max(np.abs(ex))


def test_z4_estimates_unbiased(orc, flavours):
    """With Z4 sources and exact solves both one-end estimators scatter
    around the exact flavour combination; at p = 0 every per-source value of
    a Gamma with hermitian (anti-hermitian) g5 Gamma is purely imaginary
    (real), since s^dag g5 Gamma s is real (imaginary) site by site."""
    U, Miu, Mid = flavours
    mom = [(0, 0, 0)]
    eu, ed = exact_loops(D2, Miu, mom), exact_loops(D2, Mid, mom)
    n = 64
    vals = {1: [], 2: []}
    for j in range(n):
        eta = orc.noise_z4(D2, 5150, j)
        su = (Miu @ eta.reshape(-1)).reshape(eta.shape)
        for est in (1, 2):
            vals[est].append(orc.loops_est(D2, -1, KAPPA, MU, U, est, su, mom)[:, 0])
    g5 = np.diag([1.0, 1.0, -1.0, -1.0])
    herm = [np.allclose(g5 @ orc.gamma(k), (g5 @ orc.gamma(k)).conj().T) for k in range(16)]
    for est, ex in ((1, eu - ed), (2, eu + ed)):
        a = np.array(vals[est])  # [n][16][Lt]
        err = np.abs(a.real.std(axis=0, ddof=1)) + 1j * np.abs(a.imag.std(axis=0, ddof=1))
        err /= np.sqrt(n)
        d = a.mean(axis=0) - ex[:, 0]
        assert np.all(np.abs(d.real) <= 5 * err.real + 1e-12)
        assert np.all(np.abs(d.imag) <= 5 * err.imag + 1e-12)
    a = np.array(vals[1])
    for k in range(16):
        part = a[:, k].real if herm[k] else a[:, k].imag
        assert np.max(np.abs(part)) < 1e-12 * max(1.0, np.max(np.abs(a[:, k])))


def test_generalized_needs_d_not_m(orc, flavours):
    """The exact-sum pin separates Eq. 6 from the slip of using M s (= the
    source) in place of D s: that variant, written out here with numpy over
    the same unit sources, misses the exact sum by percents."""
    U, Miu, Mid = flavours
    mom = momenta_27()
    v = int(np.prod(D2))
    x, y, z, t = coords(D2)
    g5 = np.diag([1.0, 1.0, -1.0, -1.0]).astype(complex)
    ex = exact_loops(D2, Miu, mom) + exact_loops(D2, Mid, mom)
    wrong = np.zeros_like(ex)
    for i in range(12 * v):
        s = Miu[:, i].reshape(v, 4, 3)
        e = np.zeros(12 * v, complex)
        e[i] = 1
        for n in range(16):
            site = 2 * np.einsum("xac,ab,xbc->x", s.conj(), g5 @ big_gamma_numpy(n) @ g5, e.reshape(v, 4, 3))
            for m, (a, b, c) in enumerate(mom):
                ph = np.exp(-2j * np.pi * (a * x / D2[0] + b * y / D2[1] + c * z / D2[2]))
                np.add.at(wrong[n, m], t, ph * site)
    right = _unit_sum(orc, D2, U, Miu, 2, mom)
    scale = np.max(np.abs(ex))
    assert np.max(np.abs(right - ex)) < 1e-12 * scale
    assert np.max(np.abs(wrong - ex)) > 1e-2 * scale


@pytest.mark.parametrize("est", [1, 2])
def test_tsm_with_one_end_estimator(orc, flavours, est):
    U, Miu, _ = flavours
    mom = momenta_27()
    res = orc.tsm(D2, -1, KAPPA, MU, U, 42, 2, 3, 1e-2, -1, 1e-12, -1, mom, per_source=True, estimator=est)
    ps = res["per_source"]
    assert np.allclose(res["loops"][0], (ps[:2, 1] - ps[:2, 0]).mean(axis=0), rtol=1e-13, atol=1e-13)
    assert np.allclose(res["loops"][1], ps[2:, 0].mean(axis=0), rtol=1e-13, atol=1e-13)
    eta = orc.noise_z4(D2, 42, 3)
    s, _ = orc.cgnr(D2, -1, KAPPA, MU, U, eta, 1e-2)
    assert np.allclose(ps[3, 0], orc.loops_est(D2, -1, KAPPA, MU, U, est, s, mom), atol=1e-13)
    eta0 = orc.noise_z4(D2, 42, 0)
    s_ex = (Miu @ eta0.reshape(-1)).reshape(eta0.shape)
    ref = orc.loops_est(D2, -1, KAPPA, MU, U, est, s_ex, mom)
    assert np.max(np.abs(ps[0, 1] - ref)) < 1e-9 * np.max(np.abs(ref))
