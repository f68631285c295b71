"""Seeded synthetic inputs shared by the HIP path and its test oracle.

This module holds only workload descriptions (grid sizes, ECS layer, energies,
channel counts, tolerances, seeds) and the seeded initial-guess generator.  It
contains none of the solver's arithmetic: no operator, no potential, no
right-hand side.  Both the product path and the oracle read their inputs from
here so that they see identical data.

Field layout used everywhere: an ``(n+1) x (n+1)`` complex array indexed
``[k, j]`` where row ``k`` runs along x2 and column ``j`` along x1 (x1 is
contiguous).  Rows/columns 0 and n are the homogeneous Dirichlet ring.

The Temkin-Poet model (potentials -Z1/x1, -Z2/x2, lambda/max(x1,x2)) and the
exterior-complex-scaled grid follow Sec. 2.2 (eq. partialwave2d), Sec. 5.2 and
Sec. 6.2 of Cools & Vanroose, arXiv:1412.1953.
"""
from __future__ import annotations

import dataclasses
import math

import numpy as np


@dataclasses.dataclass(frozen=True)
class Workload:
    """One MG-CCCS problem instance (grid + potential + energy + solver knobs)."""

    name: str
    n: int                 # intervals per dimension on the finest grid (power of two)
    L: float               # domain [0, L]^2
    R0: float              # exterior complex scaling starts at x = R0
    theta: float           # ECS angle
    E: float               # total energy
    levels: int            # multigrid levels including the coarsest
    M: int                 # channels (bound states) per coordinate
    tol: float             # relative residual target
    seed: int              # seed of the complex-normal initial guess
    Z1: float = 1.0
    Z2: float = 1.0
    lam: float = 1.0
    omega: float = 2.0 / 3.0
    nu1: int = 1
    nu2: int = 1
    # preconditioning hierarchy: levels >= pc_first_level put the real
    # interior on the rotated contour z = x exp(i pc_gamma) (Sec. 3.1), the
    # levels below it on z = x exp(i pc_gamma0); the autotuner replaces these
    # defaults per grid size, channel count and energy
    pc_gamma: float = math.radians(15.0)
    pc_first_level: int = 1
    pc_gamma0: float = math.radians(10.0)

    @property
    def unknowns(self) -> int:
        return (self.n - 1) ** 2


def tp_workload(name, n, L, E, levels, M, tol, seed, **kw) -> Workload:
    """Temkin-Poet instance with ECS beyond 0.75 L at angle pi/6."""
    return Workload(name=name, n=n, L=L, R0=0.75 * L, theta=math.pi / 6, E=E,
                    levels=levels, M=M, tol=tol, seed=seed, **kw)


# Plain FP64, 129^2 nodes on [0,40]^2, ECS beyond 30, E = 0.1, 5 levels, 4 channels.
SMALL_129 = tp_workload("tp129_E0.1_fp64", 128, 40.0, 0.1, 5, 4, 1e-8, 0)

# Plain FP64, 1025^2 nodes on [0,80]^2, ECS beyond 60, 7 levels, 8 channels.
TP1025 = {E: tp_workload(f"tp1025_E{E}_fp64", 1024, 80.0, E, 7, 8, 1e-10, 1)
          for E in (0.05, 0.5, 2.0)}

# Mixed precision, 2049^2 nodes on [0,160]^2, ECS beyond 120, 8 levels, 8 channels.
TP2049 = tp_workload("tp2049_E0.1_mixed", 2048, 160.0, 0.1, 8, 8, 1e-10, 2)

# Out-of-cache bandwidth probe: 4097^2 nodes (one FP64 field = 270 MB, more
# than the 256 MB on-die cache) at the 1025^2 spacing, [0,320]^2, ECS beyond
# 240, 9 levels (coarsest 16 intervals), 8 channels, E = 0.5.
TP4097 = tp_workload("tp4097_E0.5_probe", 4096, 320.0, 0.5, 9, 8, 1e-10, 5)

# Differentiation: 1025^2 on [0,80]^2 at E = 0.5.
TP1025_GRAD = tp_workload("tp1025_E0.5_grad", 1024, 80.0, 0.5, 7, 8, 1e-13, 4)


def batch_workloads() -> list[Workload]:
    """64 independent solves: energies uniform in [0.02, 3.0], grid sizes
    257^2 / 513^2 / 1025^2 (16 / 24 / 24 solves) with domains 20 / 40 / 80
    (constant spacing), ECS beyond 0.75 L, channel counts 4..16."""
    perm = np.random.default_rng(3).permutation(64)
    size_of = {}
    for pos, i in enumerate(perm):
        size_of[int(i)] = 256 if pos < 16 else (512 if pos < 40 else 1024)
    out = []
    for i in range(64):
        n = size_of[i]
        L = {256: 20.0, 512: 40.0, 1024: 80.0}[n]
        levels = {256: 5, 512: 6, 1024: 7}[n]
        E = 0.02 + 2.98 * i / 63
        M = 4 + (i % 13)
        out.append(tp_workload(f"batch{i}_n{n}", n, L, E, levels, M, 1e-10, 3000 + i))
    return out


def initial_guess(n: int, seed: int) -> np.ndarray:
    """Complex-normal initial guess on the interior, zero Dirichlet ring.

    Returns an ``(n+1, n+1)`` complex128 array indexed ``[k, j]``.
    """
    g = np.random.default_rng(seed).standard_normal((2, n - 1, n - 1))
    u = np.zeros((n + 1, n + 1), dtype=np.complex128)
    u[1:n, 1:n] = (g[0] + 1j * g[1]) / math.sqrt(2.0)
    return u


def random_field(n: int, seed: int) -> np.ndarray:
    """Another seeded complex-normal interior field (used as a generic
    right-hand side or test vector)."""
    return initial_guess(n, seed)
