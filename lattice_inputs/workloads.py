"""Workload recipes: lattice shape, operator parameters, source counts, seeds.

The operator parameters are kappa and a*mu; the twisted-mass term in the
hopping normalisation is 2*kappa*mu (so a quoted 2*kappa*mu = 0.01 at
kappa = 0.160 means a*mu = 0.03125).  Time is antiperiodic, space periodic.

Momenta are the 27 vectors n in {-1,0,1}^3 (all |n|^2 <= 3), p = 2*pi*n/L,
ordered by index (nx+1) + 3*(ny+1) + 9*(nz+1); p = 0 is index 13.
"""

from __future__ import annotations

from dataclasses import dataclass, field

import numpy as np


def momenta_27() -> np.ndarray:
    out = np.zeros((27, 3), dtype=np.int32)
    for i in range(27):
        out[i] = (i % 3 - 1, (i // 3) % 3 - 1, i // 9 - 1)
    return out


def momenta_zero() -> np.ndarray:
    return np.zeros((1, 3), dtype=np.int32)


@dataclass(frozen=True)
class Workload:
    name: str
    dims: tuple            # (Lx, Ly, Lz, Lt)
    kappa: float
    mu: float              # a*mu
    eps: float             # link spread
    gauge_seed: int
    noise_seed: int
    n_hp: int
    n_lp: int
    hp_tol: float
    lp_tol: float
    lp_maxit: int          # -1 = no iteration cap
    n_mom: int             # 1 (p = 0) or 27
    t_bc: int = -1
    rhs_blocks: tuple = field(default=(1,))

    @property
    def volume(self) -> int:
        v = 1
        for d in self.dims:
            v *= d
        return v

    def momenta(self) -> np.ndarray:
        return momenta_zero() if self.n_mom == 1 else momenta_27()


WORKLOADS = {
    # 4^4, kappa 0.160, 2 kappa mu = 0.01, eps 0.3, 4 HP at 1e-12, 32 LP at 1e-2, p = 0, FP64
    "c0_4x4x4x4": Workload("c0_4x4x4x4", (4, 4, 4, 4), 0.160, 0.03125, 0.3, 1000, 2000,
                           4, 32, 1e-12, 1e-2, -1, 1),
    # 16^3x32, a mu 0.004, 8 HP at 1e-10, 256 LP at 1e-2 (or 50 iterations), 27 momenta
    "c1_16x16x16x32": Workload("c1_16x16x16x32", (16, 16, 16, 32), 0.1632, 0.004, 0.25, 1001, 2001,
                               8, 256, 1e-10, 1e-2, 50, 27),
    # 24^3x48, reduced-precision LP storage, FP32 HP with FP64 reliable updates
    "c2_24x24x24x48": Workload("c2_24x24x24x48", (24, 24, 24, 48), 0.1632, 0.004, 0.25, 1002, 2002,
                               16, 1024, 1e-10, 1e-2, -1, 27),
    # 32^3x64, a mu 0.003, 2048 LP in multi-RHS blocks, 32 HP
    "c3_32x32x32x64": Workload("c3_32x32x32x64", (32, 32, 32, 64), 0.1632, 0.003, 0.25, 1003, 2003,
                               32, 2048, 1e-10, 1e-2, -1, 27, rhs_blocks=(4, 8, 16, 32)),
    # 24^3x48 with the learned preconditioner
    "c4_24x24x24x48": Workload("c4_24x24x24x48", (24, 24, 24, 48), 0.1632, 0.004, 0.25, 1004, 2004,
                               16, 1024, 1e-10, 1e-2, -1, 27),
}


def get_workload(name: str) -> Workload:
    if name in WORKLOADS:
        return WORKLOADS[name]
    for k, w in WORKLOADS.items():
        if k.startswith(name):
            return w
    raise KeyError(name)
