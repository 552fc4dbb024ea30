"""Oracle pins for flexible GMRES on M with the network as right
preconditioner.

With a fixed linear network N, FGMRES is GMRES on M N: after k iterations of
a cycle started from x0 the iterate is x0 + N y with y minimising
|r0 - M N y| over the Krylov space K_k(M N, r0).  The pins build that space
from the dense matrices (M from the pinned operator, N column by column from
the pinned network) and solve the least-squares problem with LAPACK:
 - the identity network (plain GMRES) and a random network, k = 1..6;
 - restarts: the second cycle of FGMRES(3) starts from the first cycle's
   residual;
 - the rotated residual equals the true residual of the iterate;
 - convergence to a tolerance, the iteration cap and a zero source.
"""

import numpy as np
import pytest

from lattice_inputs import make_gauge, random_spinor
from dense import dense_op

DIMS = (2, 2, 2, 4)
KAPPA, MU = 0.1632, 0.004


def identity_net():
    W = np.zeros((9, 1, 1, 4, 4), dtype=np.complex128)
    W[0, 0, 0] = np.eye(4)
    return [1, 1], W.reshape(-1)


def random_net(orc, seed):
    widths = [1, 2, 1]
    rng = np.random.default_rng(seed)
    n = orc.net_weight_count(widths)
    W = (rng.standard_normal(n) + 1j * rng.standard_normal(n)) * 0.05
    # identity-path weights dominate, so N is close to the identity and M N
    # stays well conditioned (restarted GMRES converges)
    W = W.reshape(-1)
    n1 = orc.layer_weight_count(1, 2)
    W[:n1].reshape(9, 2, 1, 4, 4)[0, :, 0] += np.eye(4)
    W[n1:].reshape(9, 1, 2, 4, 4)[0, 0, :] += 0.5 * np.eye(4)
    return widths, W


def dense_net(orc, U, widths, W):
    v = int(np.prod(DIMS))
    n = 12 * v
    N = np.zeros((n, n), dtype=np.complex128)
    e = np.zeros((1, v, 4, 3), dtype=np.complex128)
    flat = e.reshape(-1)
    for i in range(n):
        flat[:] = 0
        flat[i] = 1
        N[:, i] = orc.pt_net(DIMS, -1, U, widths, W, e)[0].reshape(-1)
    return N


def gmres_dense(A, r0, k):
    K = np.stack([np.linalg.matrix_power(A, i) @ r0 for i in range(k)], axis=1)
    Q, _ = np.linalg.qr(K)
    y, *_ = np.linalg.lstsq(A @ Q, r0, rcond=None)
    return Q @ y


@pytest.fixture(scope="module")
def setup(orc):
    U = make_gauge(DIMS, 0.3, 61)
    M = dense_op(DIMS, -1, KAPPA, MU, U, orc.OP_M)
    eta = orc.noise_z4(DIMS, 77, 0)
    return U, M, eta


@pytest.mark.parametrize("net", ["identity", "random"])
def test_iterates_minimise_residual_over_krylov_space(orc, setup, net):
    U, M, eta = setup
    widths, W = identity_net() if net == "identity" else random_net(orc, 5)
    N = dense_net(orc, U, widths, W)
    b = eta.reshape(-1)
    for k in range(1, 7):
        x, st = orc.fgmres(DIMS, -1, KAPPA, MU, U, widths, W, eta, 0.0, m=16, maxit=k)
        assert st["iters"] == k and st["truncated"]
        ref = N @ gmres_dense(M @ N, b, k)
        assert np.linalg.norm(x.reshape(-1) - ref) <= 1e-9 * np.linalg.norm(ref), k
        # the rotated residual is the true residual of the iterate
        assert abs(st["resid"] - st["resid_true"]) <= 1e-10


def test_restart_starts_from_the_cycle_residual(orc, setup):
    U, M, eta = setup
    widths, W = random_net(orc, 9)
    N = dense_net(orc, U, widths, W)
    A = M @ N
    b = eta.reshape(-1)
    x1 = N @ gmres_dense(A, b, 3)
    x2 = x1 + N @ gmres_dense(A, b - M @ x1, 3)
    x, st = orc.fgmres(DIMS, -1, KAPPA, MU, U, widths, W, eta, 0.0, m=3, maxit=6)
    assert st["iters"] == 6
    assert np.linalg.norm(x.reshape(-1) - x2) <= 1e-9 * np.linalg.norm(x2)
    # and it differs from unrestarted GMRES(6)
    x6 = N @ gmres_dense(A, b, 6)
    assert np.linalg.norm(x2 - x6) > 1e-6 * np.linalg.norm(x6)


def test_converges_caps_and_zero_source(orc, setup):
    """Convergence on a lighter operator (kappa = 0.10: the spectrum of M
    stays away from the origin, where restarted GMRES converges steadily; at
    kappa = 0.1632 on this rough 2x2x2x4 field restarted GMRES(8) stalls, as
    restarted GMRES may for an indefinite spectrum)."""
    U, _, eta = setup
    kappa = 0.10
    M = dense_op(DIMS, -1, kappa, MU, U, orc.OP_M)
    widths, W = random_net(orc, 3)
    x, st = orc.fgmres(DIMS, -1, kappa, MU, U, widths, W, eta, 1e-10, m=8, maxit=400)
    assert st["converged"] and st["resid"] <= 1e-10 and st["resid_true"] <= 2e-10
    ex = np.linalg.solve(M, eta.reshape(-1))
    assert np.linalg.norm(x.reshape(-1) - ex) <= 1e-8 * np.linalg.norm(ex)
    x, st = orc.fgmres(DIMS, -1, kappa, MU, U, widths, W, eta, 0.0, m=8, maxit=0)
    assert st["iters"] == 0 and st["truncated"] and np.all(x == 0)
    x, st = orc.fgmres(DIMS, -1, kappa, MU, U, widths, W, 0 * eta, 1e-3, m=8, maxit=400)
    assert st["iters"] == 0 and st["converged"] and np.all(x == 0)
    # a random right-hand side, not only Z4 noise
    rhs = random_spinor(DIMS, 4)
    x, st = orc.fgmres(DIMS, -1, kappa, MU, U, widths, W, rhs, 1e-9, m=5, maxit=400)
    assert st["converged"] and st["resid_true"] <= 2e-9
