"""Oracle pins for the even-odd (Schur-complement) reduction of M.

The dense matrix of M comes from the oracle's own operator (pinned in
test_oracle_operator.py); the Schur complement, its inverse relations and
the reconstruction are then checked against numpy block algebra on that
matrix, written here independently of the oracle:
 - the diagonal blocks of M are 1 + i tw gamma_5 on each site and M has no
   even-even or odd-odd hops (the structure the reduction relies on);
 - Mhat, Mhat^dag and Mhat^dag Mhat equal M_oo - M_oe M_ee^{-1} M_eo (and its
   adjoint) from numpy's dense inverse;
 - gamma_5 Mhat(mu) gamma_5 = Mhat(-mu)^dag;
 - the solve reaches M^{-1} eta (LAPACK) and the reconstructed whole-system
   residual equals the Schur residual with a zero even part;
 - CG iterates are A-norm optimal over the Krylov space of Mhat^dag Mhat;
 - with exact solves the TSM loops equal those of the unreduced solver.
"""

import numpy as np
import pytest

from dense import coords, dense_op
from lattice_inputs import make_gauge, random_spinor
from lattice_inputs.workloads import momenta_27

LATS = [((2, 2, 2, 2), 0.3, 0.16, 0.03125), ((2, 2, 4, 2), 0.25, 0.1632, 0.004), ((4, 2, 2, 4), 0.3, 0.15, 0.1)]


def parities(dims):
    x, y, z, t = coords(dims)
    return (x + y + z + t) % 2


def comp_index(sites):
    return (12 * np.asarray(sites)[:, None] + np.arange(12)[None, :]).ravel()


@pytest.mark.parametrize("dims,eps,kappa,mu", LATS)
def test_block_structure(orc, dims, eps, kappa, mu):
    U = make_gauge(dims, eps, 3)
    M = dense_op(dims, -1, kappa, mu, U, orc.OP_M)
    par = parities(dims)
    ev, od = comp_index(np.where(par == 0)[0]), comp_index(np.where(par == 1)[0])
    tw = 2 * kappa * mu
    g5 = np.diag([1, 1, -1, -1]).astype(complex)
    blk = np.kron(np.eye(len(ev) // 12), np.kron(np.eye(4) + 1j * tw * g5, np.eye(3)))
    assert np.max(np.abs(M[np.ix_(ev, ev)] - blk)) < 1e-14
    assert np.max(np.abs(M[np.ix_(od, od)] - blk)) < 1e-14


def dense_schur(orc, dims, U, kappa, mu, op):
    M = dense_op(dims, -1, kappa, mu, U, orc.OP_M)
    par = parities(dims)
    ev, od = comp_index(np.where(par == 0)[0]), comp_index(np.where(par == 1)[0])
    S = M[np.ix_(od, od)] - M[np.ix_(od, ev)] @ np.linalg.inv(M[np.ix_(ev, ev)]) @ M[np.ix_(ev, od)]
    if op == orc.OP_MDAG:
        S = S.conj().T
    elif op == orc.OP_MDAGM:
        S = S.conj().T @ S
    return S, od


def oracle_schur_matrix(orc, dims, U, kappa, mu, op):
    v = int(np.prod(dims))
    par = parities(dims)
    od = comp_index(np.where(par == 1)[0])
    e = np.zeros((v, 4, 3), dtype=np.complex128)
    flat = e.reshape(-1)
    S = np.zeros((len(od), len(od)), dtype=np.complex128)
    for j, i in enumerate(od):
        flat[:] = 0
        flat[i] = 1.0
        out = orc.eo_apply(dims, -1, kappa, mu, op, U, e).reshape(-1)
        # nothing on the even sites
        assert np.max(np.abs(np.delete(out, od))) == 0.0
        S[:, j] = out[od]
    return S


@pytest.mark.parametrize("dims,eps,kappa,mu", LATS)
@pytest.mark.parametrize("op", [0, 1, 2])
def test_schur_complement_matches_dense_blocks(orc, dims, eps, kappa, mu, op):
    U = make_gauge(dims, eps, 5)
    S_ref, _ = dense_schur(orc, dims, U, kappa, mu, op)
    S = oracle_schur_matrix(orc, dims, U, kappa, mu, op)
    assert np.max(np.abs(S - S_ref)) < 1e-13 * np.max(np.abs(S_ref))


def test_even_sites_of_the_input_are_ignored(orc):
    dims = (2, 2, 4, 2)
    U = make_gauge(dims, 0.3, 6)
    psi = random_spinor(dims, 1)
    par = parities(dims)
    odd_only = psi * (par == 1)[:, None, None]
    for op in (0, 1, 2):
        a = orc.eo_apply(dims, -1, 0.16, 0.03, op, U, psi)
        b = orc.eo_apply(dims, -1, 0.16, 0.03, op, U, odd_only)
        assert np.array_equal(a, b)


def test_odd_extent_is_rejected(orc):
    dims = (3, 2, 2, 2)
    U = make_gauge(dims, 0.3, 6)
    with pytest.raises(ValueError):
        orc.eo_apply(dims, -1, 0.16, 0.03, 0, U, random_spinor(dims, 1))
    with pytest.raises(ValueError):
        orc.cgnr_eo(dims, -1, 0.16, 0.03, U, orc.noise_z4(dims, 1, 0), 1e-6)


def test_gamma5_hermiticity(orc):
    dims, kappa, mu = (2, 2, 2, 4), 0.16, 0.05
    U = make_gauge(dims, 0.3, 9)
    S_p = oracle_schur_matrix(orc, dims, U, kappa, mu, 0)
    S_m = oracle_schur_matrix(orc, dims, U, kappa, -mu, 0)
    n = S_p.shape[0] // 12
    g5 = np.kron(np.eye(n), np.kron(np.diag([1, 1, -1, -1]), np.eye(3)))
    assert np.max(np.abs(g5 @ S_p @ g5 - S_m.conj().T)) < 1e-13


@pytest.mark.parametrize("dims,eps,kappa,mu", LATS)
def test_solve_and_reconstruction(orc, dims, eps, kappa, mu):
    U = make_gauge(dims, eps, 7)
    M = dense_op(dims, -1, kappa, mu, U, orc.OP_M)
    eta = orc.noise_z4(dims, 11, 2)
    exact = np.linalg.solve(M, eta.reshape(-1)).reshape(eta.shape)
    x, st = orc.cgnr_eo(dims, -1, kappa, mu, U, eta, 1e-13)
    assert st["converged"]
    assert np.linalg.norm(x - exact) / np.linalg.norm(exact) < 1e-10
    assert st["resid_true"] < 1e-11
    # a truncated solve: the whole-system residual is the Schur residual,
    # and the reconstruction leaves nothing on the even sites
    par = parities(dims)
    for k in (1, 3):
        xk, sk = orc.cgnr_eo(dims, -1, kappa, mu, U, eta, 0.0, k)
        res = eta - orc.apply_op(dims, -1, kappa, mu, orc.OP_M, U, xk)
        assert np.max(np.abs(res[par == 0])) < 1e-13
        eh = orc.eo_source(dims, -1, kappa, mu, U, eta)
        xo = xk * (par == 1)[:, None, None]
        sres = eh - orc.eo_apply(dims, -1, kappa, mu, 0, U, xo)
        assert np.max(np.abs(sres[par == 1] - res[par == 1])) < 1e-13
        assert abs(sk["resid_true"] - np.linalg.norm(res) / np.linalg.norm(eta)) < 1e-13
        # the tracked true residual stops at the same point as the direct one
        xt, stt = orc.cgnr_eo(dims, -1, kappa, mu, U, eta, sk["resid_true"] * (1 + 1e-9), -1, orc.STOP_TRUE)
        assert stt["iters"] == k


@pytest.mark.parametrize("dims", [(2, 2, 2, 2), (2, 2, 2, 4)])
def test_cg_iterates_are_krylov_optimal(orc, dims):
    """The k-th iterate minimises |x - x*| in the Mhat^dag Mhat norm over
    K_k(Mhat^dag Mhat, Mhat^dag etahat) (before the reconstruction)."""
    kappa, mu = 0.16, 0.03125
    U = make_gauge(dims, 0.3, 13)
    S, od = dense_schur(orc, dims, U, kappa, mu, 0)
    A = S.conj().T @ S
    eta = orc.noise_z4(dims, 17, 1)
    eh = orc.eo_source(dims, -1, kappa, mu, U, eta).reshape(-1)[od]
    b = S.conj().T @ eh
    for k in range(1, 7):
        cols = [b]
        for _ in range(k - 1):
            cols.append(A @ cols[-1])
        Q, _ = np.linalg.qr(np.stack(cols, axis=1))
        ref = Q @ np.linalg.solve(Q.conj().T @ A @ Q, Q.conj().T @ b)
        x, st = orc.cgnr_eo(dims, -1, kappa, mu, U, eta, 0.0, k)
        got = x.reshape(-1)[od]
        assert st["iters"] == k
        assert np.linalg.norm(got - ref) / np.linalg.norm(ref) < 1e-9, k


def test_schur_source_matches_dense_blocks(orc):
    dims, kappa, mu = (2, 2, 4, 2), 0.16, 0.03
    U = make_gauge(dims, 0.3, 15)
    M = dense_op(dims, -1, kappa, mu, U, orc.OP_M)
    par = parities(dims)
    ev, od = comp_index(np.where(par == 0)[0]), comp_index(np.where(par == 1)[0])
    eta = orc.noise_z4(dims, 3, 4).reshape(-1)
    ref = eta[od] - M[np.ix_(od, ev)] @ np.linalg.solve(M[np.ix_(ev, ev)], eta[ev])
    got = orc.eo_source(dims, -1, kappa, mu, U, eta.reshape(-1, 4, 3)).reshape(-1)
    assert np.max(np.abs(got[od] - ref)) < 1e-13
    assert np.max(np.abs(got[ev])) == 0.0


def test_tsm_with_exact_eo_solves_equals_unreduced(orc):
    """HP solves to 1e-12 by either inverter give the same loops (the
    solution M^{-1} eta is unique), and an even-odd LP map gives an estimate
    whose total agrees with the unreduced one within its error."""
    dims = (4, 4, 4, 4)
    U = make_gauge(dims, 0.3, 1000)
    mom = momenta_27()[:4]
    a = orc.tsm(dims, -1, 0.16, 0.03125, U, 2000, 3, 0, 1e-2, -1, 1e-12, -1, mom)
    b = orc.tsm(dims, -1, 0.16, 0.03125, U, 2000, 3, 0, 1e-2, -1, 1e-12, -1, mom, lp_eo=True, hp_eo=True)
    # C = mean(HP - LP): the HP parts agree; compare T - B... with n_lp = 0, T = C
    ha = orc.tsm(dims, -1, 0.16, 0.03125, U, 2000, 3, 0, 1e-14, -1, 1e-12, -1, mom, per_source=True)
    hb = orc.tsm(dims, -1, 0.16, 0.03125, U, 2000, 3, 0, 1e-14, -1, 1e-12, -1, mom, per_source=True,
                 lp_eo=True, hp_eo=True)
    hp_a, hp_b = ha["per_source"][:, 1], hb["per_source"][:, 1]
    assert np.max(np.abs(hp_a - hp_b)) < 1e-9 * np.max(np.abs(hp_a))
    # the estimate with the even-odd LP map against the unreduced one
    ta = orc.tsm(dims, -1, 0.16, 0.03125, U, 2000, 4, 32, 1e-2, -1, 1e-12, -1, mom)
    tb = orc.tsm(dims, -1, 0.16, 0.03125, U, 2000, 4, 32, 1e-2, -1, 1e-12, -1, mom, lp_eo=True)
    d = np.abs(ta["loops"][2] - tb["loops"][2])
    sig = np.abs(ta["err"][2]) + np.abs(tb["err"][2])
    assert np.all(d.real <= 3 * (np.abs(ta["err"][2].real) + np.abs(tb["err"][2].real)) + 1e-12)
    assert np.all(d.imag <= 3 * (np.abs(ta["err"][2].imag) + np.abs(tb["err"][2].imag)) + 1e-12)
    assert np.all(np.isfinite(sig))
