"""Geometric multigrid V-cycle (TEST INFRASTRUCTURE ONLY; see ``oracle/__init__``).

Components named in Sec. 1 and Sec. 3.2 (proof of concept): a V(1,1)-cycle
with an omega-Jacobi smoother (or the GMRES(3) smoothing substitute of
Sec. 6.1), full-weighting restriction and bilinear interpolation.  Readings where the paper is silent: coarse operators are
rediscretised at 2h; the coarsest level is solved exactly by a dense LU
factorisation (partial pivoting, FP64); the transfer stencils use the
standard index-space weights, also inside the complex-scaled layer.
"""
from __future__ import annotations

import numpy as np
import scipy.linalg as sla

from .grid import Grid1D, Operator, TPModel, model_operator


def jacobi(op: Operator, u: np.ndarray, f: np.ndarray, omega: float) -> np.ndarray:
    """One omega-Jacobi sweep u <- u + omega D^{-1} (f - A u) (new array)."""
    n = op.n
    r = op.residual(u, f)
    out = u.copy()
    out[1:n, 1:n] += omega * r[1:n, 1:n] / op.diag[1:n, 1:n]
    return out


def gmres_smooth(op: Operator, u: np.ndarray, f: np.ndarray, m: int = 3) -> np.ndarray:
    """One GMRES(m) cycle used as a smoother (Sec. 6.1: the GMRES(3) pre- and
    post-smoothing substitute of the V(1,1)-cycle): u + V y with y minimising
    ||f - A (u + V y)||_2 over the Krylov space K_m(A, r0), r0 = f - A u.
    Arnoldi with classical Gram-Schmidt (one pass), the small least-squares
    problem min ||beta e1 - H y|| by LAPACK's least squares; an exact
    breakdown ends the space early (new array)."""
    r = op.residual(u, f)
    beta = np.linalg.norm(r)
    if beta == 0:
        return u.copy()
    V = [r / beta]
    H = np.zeros((m + 1, m), np.complex128)
    k = m
    for i in range(m):
        w = op.apply(V[i])
        w[0, :] = w[-1, :] = w[:, 0] = w[:, -1] = 0
        h = np.array([np.vdot(v, w) for v in V])
        for q, v in enumerate(V):
            w = w - h[q] * v
        H[:i + 1, i] = h
        H[i + 1, i] = np.linalg.norm(w)
        if H[i + 1, i] == 0:
            k = i + 1
            break
        V.append(w / H[i + 1, i])
    e1 = np.zeros(k + 1, np.complex128)
    e1[0] = beta
    y = np.linalg.lstsq(H[:k + 1, :k], e1, rcond=None)[0]
    out = u.copy()
    for q in range(k):
        out = out + y[q] * V[q]
    return out


def restrict_fw(r: np.ndarray) -> np.ndarray:
    """Full weighting (1/16)[1 2 1; 2 4 2; 1 2 1] onto the coarse interior."""
    n = r.shape[0] - 1
    nc = n // 2
    out = np.zeros((nc + 1, nc + 1), r.dtype)
    K = slice(2, n - 1, 2)                   # fine index 2K for K = 1..nc-1
    Km, Kp = slice(1, n - 2, 2), slice(3, n, 2)
    out[1:nc, 1:nc] = (4.0 * r[K, K]
                       + 2.0 * (r[Km, K] + r[Kp, K] + r[K, Km] + r[K, Kp])
                       + r[Km, Km] + r[Km, Kp] + r[Kp, Km] + r[Kp, Kp]) / 16.0
    return out


def prolong_bilinear(ec: np.ndarray) -> np.ndarray:
    """Bilinear interpolation of a coarse field (zero ring) to the fine grid."""
    nc = ec.shape[0] - 1
    n = 2 * nc
    e = np.zeros((n + 1, n + 1), ec.dtype)
    e[0::2, 0::2] = ec
    e[0::2, 1::2] = 0.5 * (ec[:, :-1] + ec[:, 1:])
    e[1::2, 0::2] = 0.5 * (ec[:-1, :] + ec[1:, :])
    e[1::2, 1::2] = 0.25 * (ec[:-1, :-1] + ec[:-1, 1:] + ec[1:, :-1] + ec[1:, 1:])
    return e


class CoarsestSolver:
    """Dense LU (partial pivoting) of the coarsest operator."""

    def __init__(self, op: Operator):
        self.op = op
        A = op.sparse().toarray()
        self.lu = sla.lu_factor(A)

    def solve(self, f: np.ndarray) -> np.ndarray:
        n = self.op.n
        u = np.zeros_like(f)
        u[1:n, 1:n] = sla.lu_solve(self.lu, f[1:n, 1:n].ravel()).reshape(n - 1, n - 1)
        return u


class Hierarchy:
    """Operators on every level: level 0 finest, level ``levels-1`` coarsest.

    ``gammas[l]`` is the interior contour rotation of level l (all zero: every
    level is the exterior-complex-scaled operator).  ``model`` (TPModel or
    ExpModel) replaces the Temkin-Poet strengths Z1, Z2, lam when given.
    With smoother = "gmres3", levels below ``gs_from`` keep omega-Jacobi and
    the levels from it on take the GMRES(3) substitute (Jacobi where kh is
    small, a Krylov smoother on the coarse levels where Jacobi amplifies the
    near-resonant modes: the split of Elman, Ernst and O'Leary's Krylov-enhanced
    Helmholtz multigrid, 2001)."""

    def __init__(self, g: Grid1D, Z1: float, Z2: float, lam: float, E: float,
                 levels: int, omega: float = 2.0 / 3.0, nu1: int = 1, nu2: int = 1,
                 gammas=None, smoother: str = "jacobi", model=None, gs_from: int = 0):
        if levels < 1:
            raise ValueError("levels >= 1")
        gammas = [g.gamma] * levels if gammas is None else list(gammas)
        grids = [Grid1D(g.n, g.L, g.R0, g.theta, gammas[0])]
        for l in range(1, levels):
            grids.append(grids[-1].coarsen(gammas[l]))
        model = TPModel(Z1, Z2, lam) if model is None else model
        self.ops = [model_operator(gl, model, E) for gl in grids]
        self.coarsest = CoarsestSolver(self.ops[-1])
        self.omega, self.nu1, self.nu2 = omega, nu1, nu2
        if smoother not in ("jacobi", "gmres3"):
            raise ValueError("smoother: 'jacobi' or 'gmres3'")
        self.smoother = smoother
        self.gs_from = gs_from

    def smooth(self, op: Operator, u: np.ndarray, f: np.ndarray, level: int = 0) -> np.ndarray:
        """One smoothing step on ``level``: omega-Jacobi, or one GMRES(3) cycle."""
        if self.smoother == "gmres3" and level >= self.gs_from:
            return gmres_smooth(op, u, f, 3)
        return jacobi(op, u, f, self.omega)

    @property
    def levels(self) -> int:
        return len(self.ops)

    def vcycle(self, u: np.ndarray, f: np.ndarray, level: int = 0) -> np.ndarray:
        """One V(nu1, nu2)-cycle on ``level`` starting from ``u`` (new array)."""
        op = self.ops[level]
        if level == self.levels - 1:
            return self.coarsest.solve(f)
        for _ in range(self.nu1):
            u = self.smooth(op, u, f, level)
        fc = restrict_fw(op.residual(u, f))
        ec = self.vcycle(np.zeros_like(fc), fc, level + 1)
        u = u + prolong_bilinear(ec)
        for _ in range(self.nu2):
            u = self.smooth(op, u, f, level)
        return u
