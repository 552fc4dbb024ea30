"""Oracle pins for the learned preconditioner: the gauge-covariant
parallel-transport network, its adjoint, the loss gradient and flexible CG.

 - a single 1 -> 1 layer with the Wilson weights is exactly M (ties the
   layer's transports, path order and spin action to the pinned operator);
 - gauge covariance N[U^g](g phi) = g N[U](phi);
 - adjointness <phi, N psi> = <N^dag phi, psi> for a layer and the net;
 - the analytic gradient against central finite differences;
 - flexible CG with the identity network reproduces plain CG, converges to
   the dense solution with a trained-like network, and falls back to plain
   CG when the network is zero.
"""

import numpy as np
import pytest

from lattice_inputs import make_gauge, random_spinor, random_su3
from dense import dense_op

DIMS = (2, 4, 4, 6)
WIDTHS = [1, 2, 2, 1]
KAPPA, MU = 0.1632, 0.004


def wilson_layer_weights(orc, kappa, mu):
    W = np.zeros((9, 1, 1, 4, 4), dtype=np.complex128)
    g5 = orc.gamma_mu(4)
    W[0, 0, 0] = np.eye(4) + 2j * kappa * mu * g5
    for m in range(4):
        g = orc.gamma_mu(m)
        W[1 + 2 * m, 0, 0] = -kappa * (np.eye(4) - g)
        W[2 + 2 * m, 0, 0] = -kappa * (np.eye(4) + g)
    return W.reshape(-1)


def random_net(orc, seed, scale=0.3):
    rng = np.random.default_rng(seed)
    n = orc.net_weight_count(WIDTHS)
    return (rng.standard_normal(n) + 1j * rng.standard_normal(n)) * scale


@pytest.fixture(scope="module")
def U():
    return make_gauge(DIMS, 0.3, 41)


def vdot(a, b):
    return np.vdot(a.reshape(-1), b.reshape(-1))


def test_wilson_weights_reproduce_m(orc, U):
    W = wilson_layer_weights(orc, KAPPA, MU)
    psi = random_spinor(DIMS, 3)
    for tbc in (-1, 1):
        out = orc.pt_layer(DIMS, tbc, U, 1, 1, W, psi[None])[0]
        ref = orc.apply_op(DIMS, tbc, KAPPA, MU, orc.OP_M, U, psi)
        assert np.max(np.abs(out - ref)) < 1e-14
        # and its adjoint layer is M^dag
        outd = orc.pt_layer(DIMS, tbc, U, 1, 1, W, psi[None], adjoint=True)[0]
        refd = orc.apply_op(DIMS, tbc, KAPPA, MU, orc.OP_MDAG, U, psi)
        assert np.max(np.abs(outd - refd)) < 1e-14


def test_net_gauge_covariance(orc, U):
    v = int(np.prod(DIMS))
    g = random_su3(v, 5)
    s = np.arange(v)
    xs = [s % DIMS[0], (s // DIMS[0]) % DIMS[1], (s // (DIMS[0] * DIMS[1])) % DIMS[2],
          s // (DIMS[0] * DIMS[1] * DIMS[2])]
    strides = [1, DIMS[0], DIMS[0] * DIMS[1], DIMS[0] * DIMS[1] * DIMS[2]]
    Ug = np.empty_like(U)
    for mu in range(4):
        c = list(xs)
        c[mu] = (c[mu] + 1) % DIMS[mu]
        fwd = sum(c[k] * strides[k] for k in range(4))
        Ug[:, mu] = g @ U[:, mu] @ np.conj(np.transpose(g[fwd], (0, 2, 1)))
    W = random_net(orc, 1)
    phi = random_spinor(DIMS, 2)
    gphi = np.einsum("xij,xaj->xai", g, phi)
    lhs = orc.pt_net(DIMS, -1, Ug, WIDTHS, W, gphi[None])[0]
    rhs = np.einsum("xij,xaj->xai", g, orc.pt_net(DIMS, -1, U, WIDTHS, W, phi[None])[0])
    assert np.max(np.abs(lhs - rhs)) < 1e-12 * np.max(np.abs(rhs))


def test_adjoint_identity(orc, U):
    W = random_net(orc, 2)
    # one layer 2 -> 2
    Wl = W[orc.layer_weight_count(1, 2):orc.layer_weight_count(1, 2) + orc.layer_weight_count(2, 2)]
    a = random_spinor(DIMS, 4, 2)
    b = random_spinor(DIMS, 5, 2)
    lhs = vdot(a, orc.pt_layer(DIMS, -1, U, 2, 2, Wl, b))
    rhs = vdot(orc.pt_layer(DIMS, -1, U, 2, 2, Wl, a, adjoint=True), b)
    assert abs(lhs - rhs) < 1e-12 * abs(lhs)
    # the whole net 1 -> 2 -> 2 -> 1
    phi = random_spinor(DIMS, 6)[None]
    psi = random_spinor(DIMS, 7)[None]
    lhs = vdot(phi, orc.pt_net(DIMS, -1, U, WIDTHS, W, psi))
    rhs = vdot(orc.pt_net(DIMS, -1, U, WIDTHS, W, phi, adjoint=True), psi)
    assert abs(lhs - rhs) < 1e-12 * abs(lhs)


def test_gradient_finite_differences(orc, U):
    dims = (2, 2, 2, 4)
    U2 = make_gauge(dims, 0.3, 8)
    W = random_net(orc, 3)
    r = random_spinor(dims, 10, 2)
    e = random_spinor(dims, 11, 2)
    loss, grad = orc.pt_loss_grad(dims, -1, U2, WIDTHS, W, r, e)
    rng = np.random.default_rng(0)
    idx = rng.choice(W.size, 24, replace=False)
    h = 1e-6
    for k in idx:
        for unit, part in ((1.0, np.real), (1j, np.imag)):
            Wp, Wm = W.copy(), W.copy()
            Wp[k] += h * unit
            Wm[k] -= h * unit
            fd = (orc.pt_loss_grad(dims, -1, U2, WIDTHS, Wp, r, e)[0] -
                  orc.pt_loss_grad(dims, -1, U2, WIDTHS, Wm, r, e)[0]) / (2 * h)
            an = 2 * part(grad[k])
            # central differences carry ~eps*loss/h of rounding
            assert abs(fd - an) <= 1e-6 * abs(an) + 1e-8 * np.max(np.abs(grad)), (k, fd, an)


def identity_net(orc):
    W = np.zeros(orc.net_weight_count(WIDTHS), dtype=np.complex128)
    off = 0
    for l in range(len(WIDTHS) - 1):
        cin, cout = WIDTHS[l], WIDTHS[l + 1]
        blk = W[off:off + orc.layer_weight_count(cin, cout)].reshape(9, cout, cin, 4, 4)
        blk[0, 0, 0] = np.eye(4)
        off += orc.layer_weight_count(cin, cout)
    return W


def test_fcg_identity_net_is_cg(orc):
    dims = (4, 4, 4, 4)
    U = make_gauge(dims, 0.3, 1000)
    W = identity_net(orc)
    eta = orc.noise_z4(dims, 2000, 0)
    for k in (1, 4, 9):
        x1, s1 = orc.fcg(dims, -1, 0.16, 0.03125, U, WIDTHS, W, eta, 0.0, k)
        x2, s2 = orc.cgnr(dims, -1, 0.16, 0.03125, U, eta, 0.0, k)
        assert np.linalg.norm(x1 - x2) / np.linalg.norm(x2) < 1e-12 and not s1["fell_back"]


def test_fcg_converges_to_dense_solution(orc):
    dims = (2, 2, 2, 4)
    U = make_gauge(dims, 0.3, 2)
    kappa, mu = 0.16, 0.03125
    M = dense_op(dims, -1, kappa, mu, U, orc.OP_M)
    eta = orc.noise_z4(dims, 9, 0)
    exact = np.linalg.solve(M, eta.reshape(-1)).reshape(eta.shape)
    # a generic (non-trivial) network near the identity
    W = identity_net(orc) + random_net(orc, 4, scale=0.02)
    x, st = orc.fcg(dims, -1, kappa, mu, U, WIDTHS, W, eta, 1e-12)
    assert st["converged"]
    assert np.linalg.norm(x - exact) / np.linalg.norm(exact) < 1e-9


def test_fcg_zero_net_falls_back(orc):
    dims = (4, 4, 4, 4)
    U = make_gauge(dims, 0.3, 1000)
    W = np.zeros(orc.net_weight_count(WIDTHS), dtype=np.complex128)
    eta = orc.noise_z4(dims, 2000, 1)
    x, st = orc.fcg(dims, -1, 0.16, 0.03125, U, WIDTHS, W, eta, 1e-8)
    x2, st2 = orc.cgnr(dims, -1, 0.16, 0.03125, U, eta, 1e-8)
    assert st["fell_back"] and st["converged"]
    assert st["iters"] == st2["iters"]
    assert np.linalg.norm(x - x2) / np.linalg.norm(x2) < 1e-12


def _dense_precond(orc, dims, U, W, adjoint_first=True):
    """P = N N^dag (adjoint_first) or N^dag N as a dense matrix, column by
    column from the oracle's network."""
    v = int(np.prod(dims))
    n = 12 * v
    P = np.zeros((n, n), dtype=np.complex128)
    e = np.zeros((1, v, 4, 3), dtype=np.complex128)
    flat = e.reshape(-1)
    for i in range(n):
        flat[:] = 0
        flat[i] = 1.0
        a = orc.pt_net(dims, -1, U, WIDTHS, W, e, adjoint=adjoint_first)
        P[:, i] = orc.pt_net(dims, -1, U, WIDTHS, W, a, adjoint=not adjoint_first).reshape(-1)
    return P


def _pcg_optimal_iterate(A, P, b, k):
    """The A-norm-optimal approximation to A^{-1} b over the Krylov space
    K_k(PA, Pb) (what preconditioned CG from x = 0 reaches after k steps),
    from an orthonormal basis of that space and a dense solve."""
    cols = [P @ b]
    for _ in range(k - 1):
        cols.append(P @ (A @ cols[-1]))
    Q, _ = np.linalg.qr(np.stack(cols, axis=1))
    y = np.linalg.solve(Q.conj().T @ A @ Q, Q.conj().T @ b)
    return Q @ y


@pytest.mark.parametrize("dims", [(2, 2, 2, 2), (2, 2, 2, 4)])
def test_fcg_iterates_are_pcg_krylov_optimal(orc, dims):
    """For a fixed network N, flexible CG's preconditioner z = N N^dag r is a
    fixed Hermitian positive definite P, and its k-th iterate is the
    A-norm-optimal point of K_k(PA, Pb) with A = M^dag M, b = M^dag eta
    (the defining property of preconditioned CG).  The reference comes from
    dense matrices of M and of N N^dag and an orthonormal Krylov basis, so a
    wrong step length (<r, r> for <z, r>), a wrong ordering (N^dag N) or a
    dropped preconditioner fails it."""
    U = make_gauge(dims, 0.3, 61)
    kappa, mu = 0.16, 0.03125
    W = identity_net(orc) + random_net(orc, 12, scale=0.08)
    M = dense_op(dims, -1, kappa, mu, U, orc.OP_M)
    A = M.conj().T @ M
    eta = orc.noise_z4(dims, 31, 0)
    b = M.conj().T @ eta.reshape(-1)
    P = _dense_precond(orc, dims, U, W, adjoint_first=True)
    assert np.max(np.abs(P - P.conj().T)) < 1e-12 * np.max(np.abs(P))
    assert np.min(np.linalg.eigvalsh(P)) > 0
    # the alternatives a mistake would produce are far from the right answer
    # for this network, so the pin can tell them apart
    P_wrong = _dense_precond(orc, dims, U, W, adjoint_first=False)
    x1 = _pcg_optimal_iterate(A, P, b, 1)
    assert np.linalg.norm(_pcg_optimal_iterate(A, P_wrong, b, 1) - x1) > 1e-3 * np.linalg.norm(x1)
    z0 = P @ b
    assert abs(np.vdot(z0, b) - np.vdot(b, b)) > 1e-3 * abs(np.vdot(b, b))
    for k in range(1, 7):
        x, st = orc.fcg(dims, -1, kappa, mu, U, WIDTHS, W, eta, 0.0, k)
        assert st["iters"] == k and not st["fell_back"]
        ref = _pcg_optimal_iterate(A, P, b, k)
        dev = np.linalg.norm(x.reshape(-1) - ref) / np.linalg.norm(ref)
        assert dev < 1e-9, (k, dev)
