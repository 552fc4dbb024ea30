"""Oracle pins for the solver, the loop contraction and the estimators.

 - CG iterates are the Krylov-optimal (A-norm minimising) approximations of
   A x = b, A = M^dag M, checked against a projection onto an explicitly built
   Krylov basis; the converged solve against LAPACK.
 - the free propagator's local traces against the momentum-space closed form.
 - loops from a complete set of unit sources reproduce the exact traces of
   M^{-1} per timeslice and momentum (Eq. 2 with an orthonormal basis).
 - Eq. 3 holds exactly for exact solves; the stochastic error falls as
   1/sqrt(N); the Z4 variance closed form; and the TSM of Eq. 4 removes the
   bias of a deliberately crude truncated solver.
"""

import numpy as np
import pytest

from lattice_inputs import make_gauge, unit_gauge
from lattice_inputs.workloads import momenta_27
from dense import dense_op, exact_loops

D2 = (2, 2, 2, 2)
KAPPA, MU = 0.16, 0.03125  # 2 kappa mu = 0.01


@pytest.fixture(scope="module")
def setup2(orc):
    U = make_gauge(D2, 0.3, 1000)
    M = dense_op(D2, -1, KAPPA, MU, U, orc.OP_M)
    Minv = np.linalg.inv(M)
    return U, M, Minv


def test_cg_converged_matches_dense(orc, setup2):
    U, M, Minv = setup2
    eta = orc.noise_z4(D2, 2000, 0)
    x, st = orc.cgnr(D2, -1, KAPPA, MU, U, eta, 1e-12)
    exact = (Minv @ eta.reshape(-1)).reshape(x.shape)
    cond = np.linalg.cond(M)
    assert st["converged"] and not st["truncated"]
    assert np.linalg.norm(x - exact) / np.linalg.norm(exact) < 1e-12 * cond ** 2
    assert st["resid_true"] < 1e-10


def test_cg_iterates_are_krylov_optimal(orc, setup2):
    U, M, _ = setup2
    A = M.conj().T @ M
    eta = orc.noise_z4(D2, 2000, 1).reshape(-1)
    b = M.conj().T @ eta
    for k in range(1, 7):
        x, st = orc.cgnr(D2, -1, KAPPA, MU, U, eta.reshape(-1, 4, 3), 0.0, k)
        assert st["iters"] == k and st["truncated"]
        # orthonormal Krylov basis of span{b, Ab, ..., A^{k-1} b}
        K = np.stack([np.linalg.matrix_power(A, i) @ b for i in range(k)], axis=1)
        Q, _ = np.linalg.qr(K)
        y = np.linalg.solve(Q.conj().T @ A @ Q, Q.conj().T @ b)
        xk = Q @ y
        assert np.linalg.norm(x.reshape(-1) - xk) / np.linalg.norm(xk) < 1e-10


def test_cg_truncation_rules(orc, setup2):
    U, _, _ = setup2
    eta = orc.noise_z4(D2, 2000, 2)
    x, st = orc.cgnr(D2, -1, KAPPA, MU, U, eta, 1e-2, 0)
    assert st["iters"] == 0 and np.all(x == 0) and st["truncated"]
    x, st = orc.cgnr(D2, -1, KAPPA, MU, U, eta, 2.0)  # initial residual is 1
    assert st["iters"] == 0 and st["converged"]
    x, st = orc.cgnr(D2, -1, KAPPA, MU, U, eta, 1e-2)
    assert st["converged"] and st["resid_normal"] <= 1e-2 and st["iters"] > 3
    x2, st2 = orc.cgnr(D2, -1, KAPPA, MU, U, eta, 1e-2, -1, orc.STOP_TRUE)
    assert st2["converged"] and st2["resid_true"] <= 1e-2 * (1 + 1e-9)


def _free_closed_form(dims, kappa, mu, tbc=-1):
    """Per-site Tr[M^{-1}(x,x)] and Tr[g5 M^{-1}(x,x)] of the free operator:
    M(p)^{-1} = M(p)^dag / (a^2 + sum b^2 + m^2), a = 1 - 2k sum cos p,
    b = 2k sin p, m = 2k mu."""
    ps = [2 * np.pi * np.arange(L) / L for L in dims[:3]]
    pt = (2 * np.pi * np.arange(dims[3]) + (np.pi if tbc == -1 else 0)) / dims[3]
    P = np.meshgrid(*ps, pt, indexing="ij")
    a = 1 - 2 * kappa * sum(np.cos(p) for p in P)
    bsq = sum((2 * kappa * np.sin(p)) ** 2 for p in P)
    m = 2 * kappa * mu
    D = a ** 2 + bsq + m ** 2
    V = np.prod(dims)
    return 12 * np.sum(a / D) / V, -12j * m * np.sum(1 / D) / V


@pytest.mark.parametrize("dims", [(2, 2, 2, 2), (4, 4, 4, 4)])
def test_free_field_local_traces(orc, dims):
    U = unit_gauge(dims)
    M = dense_op(dims, -1, KAPPA, MU, U, orc.OP_M)
    Minv = np.linalg.inv(M)
    ex = exact_loops(dims, Minv, [(0, 0, 0)])
    tr1, tr5 = _free_closed_form(dims, KAPPA, MU)
    V3 = np.prod(dims[:3])
    assert np.allclose(ex[0, 0], V3 * tr1, rtol=1e-12, atol=1e-12)
    assert np.allclose(ex[15, 0], V3 * tr5, rtol=1e-12, atol=1e-12)
    for n in range(1, 15):
        assert np.max(np.abs(ex[n])) < 1e-12


def test_loops_unit_sources_give_exact_trace(orc, setup2):
    """Eq. 2 with the complete orthonormal source set {e_i}: sum_i of the loop
    of (e_i, M^{-1} e_i) is the exact trace of Gamma M^{-1} per timeslice."""
    U, M, Minv = setup2
    dims = D2
    mom = momenta_27()
    v = int(np.prod(dims))
    tot = np.zeros((16, 27, dims[3]), dtype=np.complex128)
    for i in range(12 * v):
        e = np.zeros(12 * v, dtype=np.complex128)
        e[i] = 1
        s = Minv[:, i]
        tot += orc.loops(dims, e.reshape(v, 4, 3), s.reshape(v, 4, 3), mom)
    ex = exact_loops(dims, Minv, mom)
    assert np.max(np.abs(tot - ex)) < 1e-13 * np.max(np.abs(ex))


def test_loops_anisotropic_momenta(orc):
    dims = (2, 4, 6, 2)
    U = make_gauge(dims, 0.3, 31)
    M = dense_op(dims, -1, KAPPA, MU, U, orc.OP_M)
    Minv = np.linalg.inv(M)
    mom = momenta_27()
    v = int(np.prod(dims))
    tot = np.zeros((16, 27, dims[3]), dtype=np.complex128)
    for i in range(12 * v):
        e = np.zeros(12 * v, dtype=np.complex128)
        e[i] = 1
        tot += orc.loops(dims, e.reshape(v, 4, 3), Minv[:, i].reshape(v, 4, 3), mom)
    ex = exact_loops(dims, Minv, mom)
    assert np.max(np.abs(tot - ex)) < 1e-12 * np.max(np.abs(ex))
    # on a random gauge field the traces at n = (0, 1, 0) and (0, -1, 0)
    # differ (L_y = 4), so the sign of the Fourier phase is pinned
    assert np.max(np.abs(ex[:, 16] - ex[:, 10])) > 1e-3


def test_eq3_exact_error_identity(orc, setup2):
    """Eq. 3: M^{-1} - M_E^{-1} = M^{-1} (1 - (1/N) sum eta eta^dag), in trace form."""
    U, M, Minv = setup2
    dims = D2
    N = 8
    mom = [(0, 0, 0)]
    est = np.zeros((16, 1, dims[3]), dtype=np.complex128)
    Pn = np.zeros_like(Minv)
    for j in range(N):
        eta = orc.noise_z4(dims, 5, j)
        s = (Minv @ eta.reshape(-1)).reshape(eta.shape)
        est += orc.loops(dims, eta, s, mom) / N
        Pn += np.outer(eta.reshape(-1), eta.reshape(-1).conj()) / N
    ex = exact_loops(dims, Minv, mom)
    dev = exact_loops(dims, Minv @ (np.eye(Minv.shape[0]) - Pn), mom)
    assert np.max(np.abs((ex - est) - dev)) < 1e-12


def test_z4_variance_closed_form(orc, setup2):
    """For Z4 noise (E eta = 0, E eta^2 = 0, |eta| = 1):
    Var(eta^dag A eta) = sum_{i != j} |A_ij|^2."""
    U, M, Minv = setup2
    dims = D2
    v = int(np.prod(dims))
    # A = P_{t=0} Gamma_0 M^{-1}: only rows on timeslice 0
    t = np.arange(v) // (dims[0] * dims[1] * dims[2])
    rows = np.repeat(t == 0, 12)
    A = Minv * rows[:, None]
    N = 3000
    vals = np.empty(N, dtype=np.complex128)
    for j in range(N):
        eta = orc.noise_z4(dims, 99, j)
        s = (Minv @ eta.reshape(-1)).reshape(eta.shape)
        vals[j] = orc.loops(dims, eta, s, [(0, 0, 0)])[0, 0, 0]
    off = A - np.diag(np.diag(A))
    var_closed = np.sum(np.abs(off) ** 2)
    var_emp = np.var(vals)
    assert abs(np.mean(vals) - np.trace(A)) < 5 * np.sqrt(var_closed / N)
    assert abs(var_emp / var_closed - 1) < 0.1


def test_error_falls_as_inverse_sqrt_n(orc, setup2):
    """Eq. 3 consequence: RMS error of the exact-solve estimator ~ N^{-1/2}."""
    U, M, Minv = setup2
    dims = D2
    ex = exact_loops(dims, Minv, [(0, 0, 0)])
    Ns = [4, 16, 64]
    n_seeds = 60
    rms = []
    for N in Ns:
        errs = []
        for seed in range(n_seeds):
            est = 0
            for j in range(N):
                eta = orc.noise_z4(dims, 10_000 + seed, j)
                s = (Minv @ eta.reshape(-1)).reshape(eta.shape)
                est = est + orc.loops(dims, eta, s, [(0, 0, 0)])
            est = est / N
            errs.append(np.abs(est - ex)[[0, 15]].ravel())
        rms.append(np.sqrt(np.mean(np.concatenate(errs) ** 2)))
    slope = np.polyfit(np.log(Ns), np.log(rms), 1)[0]
    assert -0.6 < slope < -0.4


def test_tsm_oracle_solves_match_manual(orc, setup2):
    """orc_tsm combines per-source loops as Eq. 4 says."""
    U, M, Minv = setup2
    dims = D2
    mom = momenta_27()
    res = orc.tsm(dims, -1, KAPPA, MU, U, 42, 2, 3, 1e-2, -1, 1e-12, -1, mom, per_source=True)
    ps = res["per_source"]
    C = (ps[:2, 1] - ps[:2, 0]).mean(axis=0)
    B = ps[2:, 0].mean(axis=0)
    assert np.allclose(res["loops"][0], C, rtol=1e-13, atol=1e-13)
    assert np.allclose(res["loops"][1], B, rtol=1e-13, atol=1e-13)
    assert np.allclose(res["loops"][2], C + B, rtol=1e-13, atol=1e-13)
    # each per-source LP loop is the loop of that source's truncated solve
    eta = orc.noise_z4(dims, 42, 3)
    s, _ = orc.cgnr(dims, -1, KAPPA, MU, U, eta, 1e-2)
    assert np.allclose(ps[3, 0], orc.loops(dims, eta, s, mom), atol=1e-13)
    # HP loop of an HP source equals the loop of the exact solve within tolerance
    eta0 = orc.noise_z4(dims, 42, 0)
    s_ex = (Minv @ eta0.reshape(-1)).reshape(eta0.shape)
    ref = orc.loops(dims, eta0, s_ex, mom)
    assert np.max(np.abs(ps[0, 1] - ref)) < 1e-9 * np.max(np.abs(ref))
    # standard errors from the per-source spread
    dC = ps[:2, 1] - ps[:2, 0]
    assert np.allclose(res["err"][0].real, np.std(dC.real, axis=0, ddof=1) / np.sqrt(2), atol=1e-14)
    assert np.allclose(res["err"][1].imag, np.std(ps[2:, 0].imag, axis=0, ddof=1) / np.sqrt(3), atol=1e-14)


def test_tsm_removes_truncation_bias(orc, setup2):
    """Eq. 4: with a crude LP solver (2 CG iterations) the LP-only estimate is
    biased by many standard errors, the TSM total is not."""
    U, M, Minv = setup2
    dims = D2
    ex = exact_loops(dims, Minv, [(0, 0, 0)])
    res = orc.tsm(dims, -1, KAPPA, MU, U, 7, 64, 1024, 0.0, 2, 1e-12, -1, [(0, 0, 0)])
    B, T = res["loops"][1], res["loops"][2]
    eB, eT = res["err"][1], res["err"][2]
    # scalar and pseudoscalar loops (the ones with a nonzero expectation)
    for n in (0, 15):
        zB = np.abs(B[n] - ex[n]).max() / np.abs(eB[n]).max()
        zT = np.abs((T[n] - ex[n]).real) / eT[n].real
        assert zB > 10
        assert np.all(zT < 4)
