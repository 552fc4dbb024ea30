"""Dense tiny-lattice helpers for the oracle pins (tests only).

The dense matrix of an operator is built column by column by applying the
oracle to unit vectors, so every dense check exercises the oracle itself;
the exact inverse and traces then come from LAPACK through numpy.
"""

from __future__ import annotations

import numpy as np

import oracle


def dense_op(dims, t_bc, kappa, mu, U, op=oracle.OP_M) -> np.ndarray:
    v = int(np.prod(dims))
    n = 12 * v
    m = np.zeros((n, n), dtype=np.complex128)
    e = np.zeros((v, 4, 3), dtype=np.complex128)
    flat = e.reshape(-1)
    for i in range(n):
        flat[:] = 0
        flat[i] = 1.0
        m[:, i] = oracle.apply_op(dims, t_bc, kappa, mu, op, U, e).reshape(-1)
    return m


def coords(dims):
    v = int(np.prod(dims))
    s = np.arange(v)
    x = s % dims[0]
    y = (s // dims[0]) % dims[1]
    z = (s // (dims[0] * dims[1])) % dims[2]
    t = s // (dims[0] * dims[1] * dims[2])
    return x, y, z, t


def gammas_numpy():
    """gamma_1..gamma_4 of the Euclidean chiral basis, written independently of
    the oracle from the 2x2 block form [[0, -i s_k], [i s_k, 0]], [[0,1],[1,0]]."""
    s = [np.array([[0, 1], [1, 0]], complex), np.array([[0, -1j], [1j, 0]]), np.array([[1, 0], [0, -1]], complex)]
    z = np.zeros((2, 2), complex)
    g = [np.block([[z, -1j * sk], [1j * sk, z]]) for sk in s]
    g.append(np.block([[z, np.eye(2)], [np.eye(2), z]]))
    return g


def big_gamma_numpy(n: int) -> np.ndarray:
    g = gammas_numpy()
    r = np.eye(4, dtype=complex)
    for mu in range(4):
        if (n >> mu) & 1:
            r = r @ g[mu]
    return r


def exact_loops(dims, minv: np.ndarray, mom) -> np.ndarray:
    """Tr over each timeslice of exp(-i p.x) Gamma_n M^{-1}(x, x): the exact
    value the loop estimator targets; complex128 [16][n_mom][Lt]."""
    v = int(np.prod(dims))
    x, y, z, t = coords(dims)
    blocks = minv.reshape(v, 4, 3, v, 4, 3)
    diag = blocks[np.arange(v), :, :, np.arange(v), :, :]  # [v][4][3][4][3]
    spin = np.einsum("xbcac->xba", diag)  # sum over colour: [x][beta][alpha]
    mom = np.asarray(mom).reshape(-1, 3)
    out = np.zeros((16, mom.shape[0], dims[3]), dtype=np.complex128)
    for n in range(16):
        G = big_gamma_numpy(n)
        tr = np.einsum("ab,xba->x", G, spin)
        for m, (nx, ny, nz) in enumerate(mom):
            ph = np.exp(-2j * np.pi * (nx * x / dims[0] + ny * y / dims[1] + nz * z / dims[2]))
            np.add.at(out[n, m], t, ph * tr)
    return out
