"""Outer iterations around one MG-CCCS cycle (TEST INFRASTRUCTURE ONLY).

* Stationary MG-CCCS: repeat {V-cycle; CCCS} (Sec. 6.1).
* BiCGSTAB right-preconditioned by one MG-CCCS cycle from zero (Sec. 6.1,
  Fig. convrate2D).
* FGMRES(m) right-preconditioned by one MG-CCCS cycle from a zero guess per
  preconditioner application (Sec. 6; Table 1), classical Gram-Schmidt with
  one re-orthogonalisation, Givens rotations, true residual at every restart.
* Iterative refinement: r = f - A u, s = sqrt(N)/||r||_2 (RMS scaling),
  e = k cycles on A e = s r from zero, u += e/s.  (Reading; the paper has no
  mixed-precision loop.)  Every cycle is affine with a fixed linear part, so
  one refinement step with k inner cycles equals k stationary cycles from u,
  whatever s is; the pins check that and the fixed point against a dense
  direct solve.

Preconditioning hierarchy.  The cycle may act on the complex-contour operator
of Sec. 3.1 (interior rotated by ``pc_gamma``) on levels >= ``pc_first_level``
and by ``pc_gamma0`` below it, while the outer iteration solves the
exterior-complex-scaled system; with both angles 0 the cycle uses the exact
operator on every level.

All stop tests use ||f - A u||_2 / ||f||_2 over the interior (Table 1 caption).
"""
from __future__ import annotations

import dataclasses

import numpy as np

from .cccs import CCCS
from .grid import Grid1D, TPModel, model_operator, rel_residual, tp_rhs
from .mg import Hierarchy


@dataclasses.dataclass
class SolveResult:
    u: np.ndarray
    relres: float
    iters: int
    vcycles: int
    history: list


class MGCCCS:
    """Multigrid hierarchy plus channel correction for one (grid, potential, E)."""

    def __init__(self, n, L, R0, theta, Z1, Z2, lam, E, levels, M,
                 omega=2.0 / 3.0, nu1=1, nu2=1, Lch=None, refine_steps=2,
                 pc_gamma=0.0, pc_first_level=0, pc_gamma0=0.0, gamma=0.0, smoother="jacobi",
                 pc_order="mg-cccs", model=None, gs_from=0):
        # gamma: contour angle of the system itself (Sec. 3.1; 0 = the
        # exterior-complex-scaled grid with a real interior); model: the
        # potentials (default: Temkin-Poet with Z1, Z2, lam)
        self.g = Grid1D(n, L, R0, theta, gamma)
        self.Z1, self.Z2, self.lam, self.E = Z1, Z2, lam, E
        self.model = TPModel(Z1, Z2, lam) if model is None else model
        gammas = [pc_gamma if l >= pc_first_level else pc_gamma0 for l in range(levels)]
        self.mg = Hierarchy(self.g, Z1, Z2, lam, E, levels, omega, nu1, nu2, gammas, smoother, self.model,
                            gs_from)
        self.op = model_operator(self.g, self.model, E)     # exact operator
        self.pc_op = self.mg.ops[0]                         # level 0 of the hierarchy
        self.M = M
        self.cc = CCCS(self.pc_op, M, Lch, refine_steps) if M > 0 else None
        if pc_order not in ("mg-cccs", "deflation"):
            raise ValueError("pc_order: 'mg-cccs' or 'deflation'")
        self.pc_order = pc_order

    @classmethod
    def from_workload(cls, w, **kw):
        kw.setdefault("pc_gamma", w.pc_gamma)
        kw.setdefault("pc_first_level", w.pc_first_level)
        kw.setdefault("pc_gamma0", w.pc_gamma0)
        return cls(w.n, w.L, w.R0, w.theta, w.Z1, w.Z2, w.lam, w.E, w.levels, w.M,
                   w.omega, w.nu1, w.nu2, **kw)

    def rhs(self) -> np.ndarray:
        """The Temkin-Poet impact right-hand side (Temkin-Poet model only)."""
        if not isinstance(self.model, TPModel):
            raise ValueError("the impact right-hand side is defined for the Temkin-Poet model")
        return tp_rhs(self.g, self.Z1, self.Z2, self.lam, self.E)

    def cycle(self, u: np.ndarray, f: np.ndarray) -> np.ndarray:
        """One MG-CCCS cycle: V-cycle, then the channel correction."""
        u = self.mg.vcycle(u, f)
        if self.cc is not None:
            u = self.cc.step(u, f)
        return u

    def precondition(self, v: np.ndarray) -> np.ndarray:
        """z = one MG-CCCS cycle on A z = v from z = 0 (a fixed linear map).

        pc_order = 'deflation' embeds the channel correction as a deflation
        step instead (Sec. 7, the alternative the paper names; the additive
        coarse-space form of deflated Krylov preconditioners): the channel
        correction of v first, z1 = e*(v), then the V-cycle on the deflated
        residual, z = z1 + V(v - A z1).  On residuals that lie in the channel
        space and without two-body coupling the correction is exact and the
        V-cycle then sees a zero residual."""
        if self.pc_order == "deflation" and self.cc is not None:
            z1 = self.cc.correction(v)
            r1 = self.pc_op.residual(z1, v)
            return z1 + self.mg.vcycle(np.zeros_like(v), r1)
        return self.cycle(np.zeros_like(v), v)

    # ------------------------------------------------------------------ #
    def solve_stationary(self, u, f, tol, max_it=200) -> SolveResult:
        """Repeat the cycle on the exact system (needs an exact level 0)."""
        if self.pc_op.g.gamma != self.g.gamma:
            raise ValueError("stationary iteration needs the exact level-0 operator")
        hist = [rel_residual(self.op, u, f)]
        it = 0
        while hist[-1] > tol and it < max_it:
            u = self.cycle(u, f)
            it += 1
            hist.append(rel_residual(self.op, u, f))
            if not np.isfinite(hist[-1]):
                break
        return SolveResult(u, hist[-1], it, it, hist)

    def solve_fgmres(self, u, f, tol, restart=20, max_it=500) -> SolveResult:
        op = self.op
        n = op.n
        fn = np.linalg.norm(f)
        r = op.residual(u, f)
        hist = [np.linalg.norm(r) / fn]
        it = 0
        while hist[-1] > tol and it < max_it:
            beta = np.linalg.norm(r)
            V = [r / beta]
            Z = []
            H = np.zeros((restart + 1, restart), np.complex128)
            cs = np.zeros(restart, np.complex128)
            sn = np.zeros(restart, np.complex128)
            gvec = np.zeros(restart + 1, np.complex128)
            gvec[0] = beta
            j = 0
            while j < restart and it < max_it:
                z = self.precondition(V[j])
                Z.append(z)
                w = op.apply(z)
                w[0, :] = w[-1, :] = w[:, 0] = w[:, -1] = 0
                for _ in range(2):                      # CGS2
                    coef = np.array([np.vdot(v, w) for v in V])
                    H[:j + 1, j] += coef
                    for v, cf in zip(V, coef):
                        w = w - cf * v
                H[j + 1, j] = np.linalg.norm(w)
                hnext = H[j + 1, j]
                for i in range(j):                      # earlier Givens rotations
                    x1, x2 = H[i, j], H[i + 1, j]
                    H[i, j] = np.conj(cs[i]) * x1 + np.conj(sn[i]) * x2
                    H[i + 1, j] = -sn[i] * x1 + cs[i] * x2
                den = np.sqrt(abs(H[j, j]) ** 2 + abs(H[j + 1, j]) ** 2)
                cs[j] = H[j, j] / den
                sn[j] = H[j + 1, j] / den
                H[j, j] = den
                H[j + 1, j] = 0
                gvec[j + 1] = -sn[j] * gvec[j]
                gvec[j] = np.conj(cs[j]) * gvec[j]
                it += 1
                j += 1
                if abs(gvec[j]) / fn <= tol or hnext == 0:
                    break
                V.append(w / hnext)
            y = np.linalg.solve(np.triu(H[:j, :j]), gvec[:j])
            for zz, yy in zip(Z, y):
                u = u + yy * zz
            r = op.residual(u, f)
            hist.append(np.linalg.norm(r) / fn)
            if not np.isfinite(hist[-1]):
                break
        return SolveResult(u, hist[-1], it, it, hist)

    def solve_bicgstab(self, u, f, tol, max_it=500) -> SolveResult:
        """BiCGSTAB (van der Vorst's stabilised bi-conjugate gradients) on the
        system, right-preconditioned by one MG-CCCS cycle from zero per
        application (Sec. 6.1, Fig. convrate2D), with the shadow vector equal
        to the initial residual and conjugated inner products.  One iteration
        applies the operator and the preconditioner twice:
            rho = (r~, r);  beta = (rho / rho_old)(alpha / omega)
            p = r + beta (p - omega v);  p^ = B p;  v = A p^
            alpha = rho / (r~, v);  s = r - alpha v
            s^ = B s;  t = A s^;  omega = (t, s) / (t, t)
            u += alpha p^ + omega s^;  r = s - omega t
        history: ||r||/||f|| of the recurred residual at the start and after
        every iteration; the final relres is recomputed from u."""
        op = self.op
        fn = np.linalg.norm(f)
        r = op.residual(u, f)
        rt = r.copy()
        hist = [np.linalg.norm(r) / fn]
        p = np.zeros_like(r)
        v = np.zeros_like(r)
        rho_old = alpha = omega = 1.0
        it = 0

        def apply(x):
            y = op.apply(x)
            y[0, :] = y[-1, :] = y[:, 0] = y[:, -1] = 0
            return y

        while hist[-1] > tol and it < max_it:
            rho = np.vdot(rt, r)
            beta = (rho / rho_old) * (alpha / omega)
            p = r + beta * (p - omega * v)
            ph = self.precondition(p)
            v = apply(ph)
            alpha = rho / np.vdot(rt, v)
            s = r - alpha * v
            it += 1
            if np.linalg.norm(s) / fn <= tol:
                u = u + alpha * ph
                hist.append(np.linalg.norm(s) / fn)
                break
            sh = self.precondition(s)
            t = apply(sh)
            omega = np.vdot(t, s) / np.vdot(t, t)
            u = u + alpha * ph + omega * sh
            r = s - omega * t
            rho_old = rho
            hist.append(np.linalg.norm(r) / fn)
            if not np.isfinite(hist[-1]):
                break
        return SolveResult(u, rel_residual(op, u, f), it, 2 * it, hist)

    def solve_ir(self, u, f, tol, inner_cycles=2, max_it=200) -> SolveResult:
        op = self.op
        hist = [rel_residual(op, u, f)]
        it = 0
        while hist[-1] > tol and it < max_it:
            r = op.residual(u, f)
            s = np.sqrt((op.n - 1) ** 2) / np.linalg.norm(r)
            e = np.zeros_like(r)
            for _ in range(inner_cycles):
                e = self.cycle(e, s * r)
            u = u + e / s
            it += 1
            hist.append(rel_residual(op, u, f))
            if not np.isfinite(hist[-1]):
                break
        return SolveResult(u, hist[-1], it, it * inner_cycles, hist)
