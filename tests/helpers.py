"""Shared helpers of the GPU parity tests: build the HIP handle and the
oracle for the same problem, and compare fields."""
from __future__ import annotations

import dataclasses
import math
import warnings

import numpy as np

from oracle.grid import ExpModel
from oracle.solvers import MGCCCS
from paper_1412_1953_amd.workloads import initial_guess, random_field

warnings.simplefilter("ignore")


@dataclasses.dataclass
class Case:
    n: int
    L: float
    E: float
    levels: int
    M: int
    theta: float = math.pi / 6
    R0frac: float = 0.75
    Z1: float = 1.0
    Z2: float = 1.0
    lam: float = 1.0
    pc_gamma: float = 0.0
    pc_gamma0: float = 0.0
    gamma: float = 0.0
    smoother: int = 0
    gs_from: int = 0
    pc_order: int = 0
    pc_first_level: int = 0
    seed: int = 11
    Lch: int | None = None
    # exponential model (a1, b1, a2, b2, c12, d12) instead of Temkin-Poet
    exp: tuple | None = None

    @property
    def R0(self):
        return self.R0frac * self.L

    def oracle(self, **kw) -> MGCCCS:
        return MGCCCS(self.n, self.L, self.R0, self.theta, self.Z1, self.Z2, self.lam, self.E,
                      self.levels, self.M, pc_gamma=self.pc_gamma, pc_gamma0=self.pc_gamma0, gamma=self.gamma,
                      smoother=("gmres3" if self.smoother else "jacobi"), gs_from=self.gs_from,
                      pc_order=("deflation" if self.pc_order else "mg-cccs"),
                      pc_first_level=self.pc_first_level, Lch=self.Lch,
                      model=ExpModel(*self.exp) if self.exp else None, **kw)

    def grid(self, max_restart=10, fp32=True):
        from paper_1412_1953_amd import mgcccs
        g = mgcccs.Grid(self.n, self.L, self.R0, self.theta, self.levels, self.M, Lch=self.Lch,
                        pc_gamma=self.pc_gamma, pc_first_level=self.pc_first_level, pc_gamma0=self.pc_gamma0,
                        gamma=self.gamma, smoother=self.smoother, gs_from=self.gs_from, pc_order=self.pc_order,
                        max_restart=max_restart, fp32=fp32, pot_tables=1 if self.exp else 0)
        if self.exp:
            g.set_potential_exp(*self.exp)
        else:
            g.set_potential(self.Z1, self.Z2, self.lam)
        g.set_energy(self.E)
        return g

    def u0(self):
        return initial_guess(self.n, self.seed)

    def rand(self, k=1):
        return random_field(self.n, self.seed + 1000 * k)


def to_np(t):
    return t.detach().cpu().numpy().astype(np.complex128)


def rel_err(a, b):
    """max |a - b| / max |b| over the whole field."""
    return float(np.abs(a - b).max() / np.abs(b).max())


def rel2(a, b):
    return float(np.linalg.norm(a - b) / np.linalg.norm(b))
