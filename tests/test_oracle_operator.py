"""Oracle pins for the twisted-mass Wilson-Dirac operator.

Identities checked (section 2.2 and 2.3 of the paper and plain algebra):
 - adjointness <phi, M psi> = <M^dag phi, psi> (M^dag is coded separately);
 - gamma_5-hermiticity gamma_5 M(mu) gamma_5 = M(-mu)^dag;
 - the flavour identities M_u - M_d = 2i(2 kappa mu) gamma_5 and
   M_u + M_d = 2 (1 - kappa H) (hopping normalisation);
 - M^dag M = (1 - kappa H)^dag (1 - kappa H) + (2 kappa mu)^2, hence the
   twisted-mass lower bound lambda_min(M^dag M) >= (2 kappa mu)^2;
 - plane waves at unit links map to the momentum-space closed form;
 - gauge covariance H[U^g](g psi) = g H[U] psi.
"""

import numpy as np
import pytest

from lattice_inputs import make_gauge, random_spinor, random_su3, unit_gauge
from dense import dense_op

ANISO = (2, 4, 6, 8)
KAPPA, MU = 0.1632, 0.004


@pytest.fixture(scope="module")
def U():
    return make_gauge(ANISO, 0.3, 123)


def vdot(a, b):
    return np.vdot(a.reshape(-1), b.reshape(-1))


def g5(psi):
    out = psi.copy()
    out[..., 2:, :] *= -1
    return out


def test_adjoint(orc, U):
    phi = random_spinor(ANISO, 1)
    psi = random_spinor(ANISO, 2)
    for tbc in (-1, 1):
        Mpsi = orc.apply_op(ANISO, tbc, KAPPA, MU, orc.OP_M, U, psi)
        Mdphi = orc.apply_op(ANISO, tbc, KAPPA, MU, orc.OP_MDAG, U, phi)
        a, b = vdot(phi, Mpsi), vdot(Mdphi, psi)
        assert abs(a - b) <= 1e-13 * abs(a)


def test_gamma5_hermiticity(orc, U):
    psi = random_spinor(ANISO, 3)
    lhs = g5(orc.apply_op(ANISO, -1, KAPPA, MU, orc.OP_M, U, g5(psi)))
    rhs = orc.apply_op(ANISO, -1, KAPPA, -MU, orc.OP_MDAG, U, psi)
    assert np.max(np.abs(lhs - rhs)) < 1e-14


def test_flavour_identities(orc, U):
    psi = random_spinor(ANISO, 4)
    mu_ = orc.apply_op(ANISO, -1, KAPPA, MU, orc.OP_M, U, psi)
    md_ = orc.apply_op(ANISO, -1, KAPPA, -MU, orc.OP_M, U, psi)
    hop = orc.apply_op(ANISO, -1, KAPPA, MU, orc.OP_HOP, U, psi)
    # M_u - M_d = 2i (2 kappa mu) gamma_5
    assert np.max(np.abs((mu_ - md_) - 2j * (2 * KAPPA * MU) * g5(psi))) < 1e-15
    # M_u + M_d = 2 D_W with D_W = 1 - kappa H in hopping normalisation
    assert np.max(np.abs((mu_ + md_) - 2 * (psi - KAPPA * hop))) < 1e-14


def test_normal_operator(orc, U):
    psi = random_spinor(ANISO, 5)
    mdm = orc.apply_op(ANISO, -1, KAPPA, MU, orc.OP_MDAGM, U, psi)
    comp = orc.apply_op(ANISO, -1, KAPPA, MU, orc.OP_MDAG, U, orc.apply_op(ANISO, -1, KAPPA, MU, orc.OP_M, U, psi))
    assert np.max(np.abs(mdm - comp)) < 1e-14
    a = psi - KAPPA * orc.apply_op(ANISO, -1, KAPPA, MU, orc.OP_HOP, U, psi)
    # A^dag A psi + (2 kappa mu)^2 psi using A^dag = 1 - kappa H^dag = M(mu=0)^dag
    ada = orc.apply_op(ANISO, -1, KAPPA, 0.0, orc.OP_MDAG, U, a)
    assert np.max(np.abs(mdm - (ada + (2 * KAPPA * MU) ** 2 * psi))) < 1e-14


def test_spectral_lower_bound(orc):
    dims = (2, 2, 2, 2)
    U = make_gauge(dims, 0.3, 9)
    kappa, mu = 0.16, 0.03125
    A = dense_op(dims, -1, kappa, mu, U, orc.OP_MDAGM)
    assert np.allclose(A, A.conj().T, atol=1e-14)
    lam = np.linalg.eigvalsh(A)
    assert lam.min() >= (2 * kappa * mu) ** 2 * (1 - 1e-12)
    # and the bound is approached at zero twist only through A^dag A >= 0
    M = dense_op(dims, -1, kappa, mu, U, orc.OP_M)
    assert np.allclose(M.conj().T @ M, A, atol=1e-13)


@pytest.mark.parametrize("tbc", [-1, 1])
def test_free_field_plane_wave(orc, tbc):
    dims = ANISO
    U = unit_gauge(dims)
    v = int(np.prod(dims))
    s = np.arange(v)
    xs = [s % dims[0], (s // dims[0]) % dims[1], (s // (dims[0] * dims[1])) % dims[2],
          s // (dims[0] * dims[1] * dims[2])]
    rng = np.random.default_rng(0)
    chi = rng.standard_normal((4, 3)) + 1j * rng.standard_normal((4, 3))
    from dense import gammas_numpy
    g = gammas_numpy()
    g5m = np.diag([1, 1, -1, -1]).astype(complex)
    kappa, mu = 0.16, 0.03125
    for n in [(0, 0, 0, 0), (1, 2, 3, 5), (1, 0, 2, 7)]:
        p = [2 * np.pi * n[k] / dims[k] for k in range(3)]
        p.append((2 * np.pi * n[3] + (np.pi if tbc == -1 else 0.0)) / dims[3])
        phase = np.exp(1j * sum(p[k] * xs[k] for k in range(4)))
        psi = phase[:, None, None] * chi[None]
        out = orc.apply_op(dims, tbc, kappa, mu, orc.OP_M, U, psi)
        Mp = (1 - 2 * kappa * sum(np.cos(pk) for pk in p)) * np.eye(4) \
            + 2j * kappa * sum(g[k] * np.sin(p[k]) for k in range(4)) + 2j * kappa * mu * g5m
        expect = phase[:, None, None] * (Mp @ chi)[None]
        assert np.max(np.abs(out - expect)) < 1e-13


def test_gauge_covariance(orc, U):
    dims = ANISO
    v = int(np.prod(dims))
    g = random_su3(v, 77)
    s = np.arange(v)
    xs = [s % dims[0], (s // dims[0]) % dims[1], (s // (dims[0] * dims[1])) % dims[2],
          s // (dims[0] * dims[1] * dims[2])]
    Ug = np.empty_like(U)
    strides = [1, dims[0], dims[0] * dims[1], dims[0] * dims[1] * dims[2]]
    for mu in range(4):
        c = list(xs)
        c[mu] = (c[mu] + 1) % dims[mu]
        fwd = sum(c[k] * strides[k] for k in range(4))
        Ug[:, mu] = g @ U[:, mu] @ np.conj(np.transpose(g[fwd], (0, 2, 1)))
    psi = random_spinor(dims, 6)
    gpsi = np.einsum("xij,xaj->xai", g, psi)
    lhs = orc.apply_op(dims, -1, KAPPA, MU, orc.OP_HOP, Ug, gpsi)
    rhs = np.einsum("xij,xaj->xai", g, orc.apply_op(dims, -1, KAPPA, MU, orc.OP_HOP, U, psi))
    assert np.max(np.abs(lhs - rhs)) < 1e-13


def test_smallest_lattice_l2(orc):
    # L = 2: x + mu and x - mu coincide; adjointness and gamma_5-hermiticity still hold
    dims = (2, 2, 2, 2)
    U = make_gauge(dims, 0.3, 5)
    phi, psi = random_spinor(dims, 7), random_spinor(dims, 8)
    a = vdot(phi, orc.apply_op(dims, -1, KAPPA, MU, orc.OP_M, U, psi))
    b = vdot(orc.apply_op(dims, -1, KAPPA, MU, orc.OP_MDAG, U, phi), psi)
    assert abs(a - b) < 1e-13 * abs(a)
