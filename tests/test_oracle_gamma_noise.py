"""Oracle pins: gamma algebra and Z4 noise (Eq. 1)."""

import os

import numpy as np
import pytest

from dense import gammas_numpy

pytestmark = pytest.mark.filterwarnings("ignore")

HERE = os.path.dirname(os.path.abspath(__file__))


def test_clifford_algebra(orc):
    g = [orc.gamma_mu(mu) for mu in range(4)]
    for mu in range(4):
        assert np.allclose(g[mu], g[mu].conj().T, atol=0)  # hermitian
        for nu in range(4):
            ac = g[mu] @ g[nu] + g[nu] @ g[mu]
            assert np.allclose(ac, 2 * np.eye(4) * (mu == nu), atol=0)


def test_gamma5_diagonal_and_basis(orc):
    g5 = orc.gamma_mu(4)
    assert np.array_equal(g5, np.diag([1, 1, -1, -1]).astype(complex))
    assert np.array_equal(orc.gamma(15), g5)
    assert np.array_equal(orc.gamma(0), np.eye(4, dtype=complex))
    # the 16 Gamma_n form an orthogonal basis: Tr(G_m^dag G_n) = 4 delta_mn
    G = [orc.gamma(n) for n in range(16)]
    for m in range(16):
        for n in range(16):
            assert abs(np.trace(G[m].conj().T @ G[n]) - 4 * (m == n)) < 1e-14
    # each Gamma_n is a phase-signed permutation: one unit-modulus entry per row
    for n in range(16):
        nz = np.abs(G[n]) > 0
        assert (nz.sum(axis=1) == 1).all() and (nz.sum(axis=0) == 1).all()
        assert np.allclose(np.abs(G[n][nz]), 1)


def test_gammas_match_block_form(orc):
    # the chiral basis written from the 2x2 block definition
    for mu, gm in enumerate(gammas_numpy()):
        assert np.allclose(orc.gamma_mu(mu), gm, atol=0)


def _kat():
    rows = []
    with open(os.path.join(HERE, "golden", "splitmix64_kat.txt")) as f:
        for line in f:
            if line.startswith("#") or not line.strip():
                continue
            seed, idx, val = line.split()
            rows.append((int(seed), int(idx), int(val)))
    return rows


def test_splitmix64_known_answers(orc):
    rows = _kat()
    seed = rows[0][0]
    seq = orc.splitmix64_sequence(seed, len(rows))
    for s, i, v in rows:
        assert s == seed
        assert seq[i] == v


def test_noise_hash_is_stream_output(orc):
    # the per-site hash is output number 1 + j*V + site of the splitmix64
    # stream started at state mix64(seed) (= first output of a stream seeded
    # with seed - increment)
    seed = 2000
    gamma = 0x9E3779B97F4A7C15
    start = orc.splitmix64_sequence((seed - gamma) % 2**64, 1)[0]
    vol = 7
    seq = orc.splitmix64_sequence(start, 3 * vol)
    for j in range(3):
        for s in range(vol):
            assert orc.noise_hash(seed, j, vol, s) == seq[j * vol + s]


def test_z4_values_and_codes(orc):
    dims = (2, 4, 6, 8)
    codes = orc.noise_codes(dims, 77, 3)
    eta = orc.noise_z4(dims, 77, 3)
    z4 = np.array([1, 1j, -1, -1j])
    assert codes.max() <= 3
    assert np.array_equal(eta.reshape(-1, 12), z4[codes])
    # |eta|^2 = 1 exactly for every component
    assert np.array_equal(np.abs(eta) ** 2, np.ones(eta.shape))


def test_z4_eq1_statistics(orc):
    """Eq. 1: (1/N) sum eta = O(1/sqrt N) and (1/N) sum eta eta^dag = 1 + O(1/sqrt N)."""
    dims = (2, 2, 2, 2)
    n_comp = 12 * 16
    N = 400
    E = np.stack([orc.noise_z4(dims, 11, j).reshape(-1) for j in range(N)])  # [N][n]
    mean = E.mean(axis=0)
    # each component mean has variance 1/N: RMS over components ~ 1/sqrt(N)
    rms_mean = np.sqrt(np.mean(np.abs(mean) ** 2))
    assert 0.8 / np.sqrt(N) < rms_mean < 1.2 / np.sqrt(N)
    P = E.T @ E.conj() / N
    assert np.allclose(np.diag(P), 1.0, atol=1e-15)  # exactly one on the diagonal
    off = P[~np.eye(n_comp, dtype=bool)]
    rms_off = np.sqrt(np.mean(np.abs(off) ** 2))
    assert 0.9 / np.sqrt(N) < rms_off < 1.1 / np.sqrt(N)
    # E[eta^2] = 0 for Z4 (not for Z2)
    assert abs(np.mean(E ** 2)) < 4 / np.sqrt(N * n_comp)


def test_z4_codes_uniform(orc):
    codes = np.concatenate([orc.noise_codes((4, 4, 4, 4), 5, j).reshape(-1) for j in range(8)])
    counts = np.bincount(codes, minlength=4)
    exp = codes.size / 4
    chi2 = ((counts - exp) ** 2 / exp).sum()
    assert chi2 < 16.27  # p = 0.001 for 3 degrees of freedom


def test_noise_depends_on_seed_source_site(orc):
    dims = (4, 4, 4, 4)
    a = orc.noise_codes(dims, 1, 0)
    assert not np.array_equal(a, orc.noise_codes(dims, 2, 0))
    assert not np.array_equal(a, orc.noise_codes(dims, 1, 1))
    assert not np.array_equal(a[0], a[1])
