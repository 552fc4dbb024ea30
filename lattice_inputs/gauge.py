"""Synthetic gauge fields and spinors.

Canonical gauge layout: complex128 array of shape [V][4][3][3], where
site = x + Lx*(y + Ly*(z + Lz*t)), the second index is the direction
mu = 0..3 (x, y, z, t) and the last two are the colour row and column of the
link U_mu(x), which transports from x+mu to x.  No boundary sign is stored in
the links; the antiperiodic time boundary is a property of the operator.

Canonical spinor layout: complex128 [V][4][3] (spin, colour); component
index 3*spin + colour.

The link recipe is the one the workloads specify: W = 1 + eps*X with X a
complex Gaussian matrix (real and imaginary parts each N(0, 1/2)), rows
orthonormalised by Gram-Schmidt in the order 0, 1, 2, then the determinant
phase removed by multiplying with exp(-i arg(det)/3) (principal branch).
"""

from __future__ import annotations

import numpy as np

_CHUNK = 1 << 19  # links generated per chunk (bounds host memory at 32^3x64)


def lattice_volume(dims) -> int:
    v = 1
    for d in dims:
        v *= int(d)
    return v


def _gram_schmidt_su3(w: np.ndarray) -> np.ndarray:
    """Row Gram-Schmidt of a stack of 3x3 complex matrices, det phase removed."""
    u0 = w[:, 0, :]
    u0 = u0 / np.linalg.norm(u0, axis=1, keepdims=True)
    w1 = w[:, 1, :]
    u1 = w1 - np.sum(np.conj(u0) * w1, axis=1, keepdims=True) * u0
    u1 = u1 / np.linalg.norm(u1, axis=1, keepdims=True)
    w2 = w[:, 2, :]
    u2 = (w2 - np.sum(np.conj(u0) * w2, axis=1, keepdims=True) * u0
          - np.sum(np.conj(u1) * w2, axis=1, keepdims=True) * u1)
    u2 = u2 / np.linalg.norm(u2, axis=1, keepdims=True)
    u = np.stack([u0, u1, u2], axis=1)
    det = np.linalg.det(u)
    u *= np.exp(-1j * np.angle(det) / 3.0)[:, None, None]
    return u


def make_gauge(dims, eps: float, seed: int) -> np.ndarray:
    """Links (1 + eps*X) reunitarised; returns complex128 [V][4][3][3]."""
    v = lattice_volume(dims)
    n = 4 * v
    rng = np.random.default_rng(seed)
    out = np.empty((n, 3, 3), dtype=np.complex128)
    eye = np.eye(3, dtype=np.complex128)
    scale = np.sqrt(0.5)
    for a in range(0, n, _CHUNK):
        m = min(_CHUNK, n - a)
        re = rng.standard_normal((m, 3, 3))
        im = rng.standard_normal((m, 3, 3))
        x = (re + 1j * im) * scale
        out[a:a + m] = _gram_schmidt_su3(eye + eps * x)
    return out.reshape(v, 4, 3, 3)


def unit_gauge(dims) -> np.ndarray:
    v = lattice_volume(dims)
    u = np.zeros((v, 4, 3, 3), dtype=np.complex128)
    u[:, :, 0, 0] = u[:, :, 1, 1] = u[:, :, 2, 2] = 1.0
    return u


def random_su3(n: int, seed: int) -> np.ndarray:
    """n random SU(3) matrices (Gaussian matrix, Gram-Schmidt, det phase removed)."""
    rng = np.random.default_rng(seed)
    x = (rng.standard_normal((n, 3, 3)) + 1j * rng.standard_normal((n, 3, 3))) * np.sqrt(0.5)
    return _gram_schmidt_su3(x)


def random_spinor(dims, seed: int, nrhs: int | None = None) -> np.ndarray:
    """Gaussian complex spinor(s), complex128 [V][4][3] or [nrhs][V][4][3]."""
    v = lattice_volume(dims)
    rng = np.random.default_rng(seed)
    shape = (v, 4, 3) if nrhs is None else (nrhs, v, 4, 3)
    return (rng.standard_normal(shape) + 1j * rng.standard_normal(shape)) * np.sqrt(0.5)
