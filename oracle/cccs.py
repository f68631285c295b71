"""Coupled Channel Correction Step (TEST INFRASTRUCTURE ONLY; see ``oracle/__init__``).

Follows Sec. 4 of the paper:
  * 1D bound states H1 phi_n = lambda_n phi_n, H2 varphi_n = mu_n varphi_n
    (Sec. 2.4 eq. 1d_eigenstate), normalised with the bilinear form
    int phi^2 dz = 1 without conjugation (Sec. 3.1 Remark 3, Sec. 4.2 footnote),
    refined by two shift-and-invert steps (Sec. 5.1);
  * the channel expansion u ~ sum_m A_m(y) phi_m(x) + sum_l B_l(x) varphi_l(y)
    (Sec. 4.1 eq. coupled_channel_expansion) made unique by the convention
    a_ji = 0 for j > i, b_ij = 0 for i >= j (Remark 4, eqs. convention_a/b),
    with the coefficients from eq. coefficients;
  * the coupled channel equations (Sec. 4.2 eqs. channel1/channel2) with the
    channel potentials V^A_im(y) = int V12 phi_i phi_m dx and
    V^B_jl(x) = int V12 varphi_j varphi_l dy;
  * the correction u* = u + sum e^A_m phi_m + sum e^B_l varphi_l (Sec. 4.3 eq. cccs).

Discrete integrals use the dual weights w_j of the complex grid.  Readings
(garbled indices in the B equations are read as functions of x after the
integration over y).  The channel systems are solved with LAPACK's banded LU
(partial pivoting) in the interleaved ordering (node, channel).
"""
from __future__ import annotations

import numpy as np
import scipy.linalg as sla

from .grid import Grid1D, Operator


def select_lowest(evals: np.ndarray, M: int) -> np.ndarray:
    """Indices of the M eigenvalues with the smallest real part; near-ties
    (|delta Re| < 1e-12) go to the smaller |Im|."""
    order = sorted(range(len(evals)), key=lambda i: evals[i].real)
    # resolve near-ties explicitly, keeping the real-part order otherwise
    out = []
    i = 0
    while i < len(order) and len(out) < M:
        grp = [order[i]]
        while i + len(grp) < len(order) and \
                abs(evals[order[i + len(grp)]].real - evals[grp[0]].real) < 1e-12:
            grp.append(order[i + len(grp)])
        grp.sort(key=lambda t: abs(evals[t].imag))
        out.extend(grp)
        i += len(grp)
    return np.array(out[:M], dtype=int)


def bound_states(g: Grid1D, V: np.ndarray, M: int, refine_steps: int = 2):
    """Lowest M eigenpairs of H = -1/2 d^2/dz^2 + V on the complex grid.

    The discrete eigenproblem H phi = lambda phi (eq. 1d_eigenstate; H = W^-1 S
    with the complex-symmetric S = W H) solved densely in this standard form;
    bilinear normalisation phi^T W phi = 1; sign fixed so that the
    entry of largest modulus has a positive real part; then ``refine_steps``
    shift-and-invert steps (S - lambda W) psi = W phi (Sec. 5.1) and a
    Rayleigh-quotient update of lambda.

    Returns (lam[M], phi[M, n+1]) with phi zero on the ring.
    """
    n = g.n
    if not (1 <= M <= n - 1):
        raise ValueError("need 1 <= M <= n-1")
    S = g.weighted_hamiltonian_dense(V)
    W = np.diag(g.w[1:n])
    evals, evecs = sla.eig(S / g.w[1:n, None])
    sel = select_lowest(evals, M)
    lam = np.empty(M, np.complex128)
    phi = np.zeros((M, n + 1), np.complex128)
    wv = g.w[1:n]
    for t, idx in enumerate(sel):
        lt = evals[idx]
        v = evecs[:, idx]
        for _ in range(refine_steps):
            v = sla.solve(S - lt * W, wv * v)
            v = v / np.sqrt(np.sum(wv * v * v))
        v = v / np.sqrt(np.sum(wv * v * v))
        if v[np.argmax(np.abs(v))].real < 0:
            v = -v
        lt = (v @ S @ v) / np.sum(wv * v * v)
        lam[t] = lt
        phi[t, 1:n] = v
    return lam, phi


def channel_potential(g: Grid1D, V12: np.ndarray, phi: np.ndarray, axis: str) -> np.ndarray:
    """Channel potentials.

    axis='A':  VA[k, i, m] = sum_j w_j V12[k, j] phi_i(z_j) phi_m(z_j)   (channels in x)
    axis='B':  VB[j, l, p] = sum_k w_k V12[k, j] varphi_l(z_k) varphi_p(z_k)  (channels in y)
    Returned with the first index over all n+1 nodes (ring rows zero).
    """
    n = g.n
    G = g.w[:, None, None] * phi.T[:, :, None] * phi.T[:, None, :]   # [node, i, m]
    M = phi.shape[0]
    if axis == "A":
        V = V12 @ G.reshape(n + 1, M * M)       # sum over j (columns)
    else:
        V = V12.T @ G.reshape(n + 1, M * M)     # sum over k (rows)
    V = V.reshape(n + 1, M, M)
    V[0] = 0
    V[n] = 0
    return V


class ChannelSystem:
    """Block-tridiagonal coupled channel operator on one axis.

    Unknown e[t, i] (node t = 1..n-1, channel i); equation at (t, i):
        a_t e[t-1,i] + c_t e[t+1,i] + (b_t + Vone_t + lam_i - E) e[t,i]
        + sum_m Vch[t,i,m] e[t,m] = rhs[t,i]
    (eqs. channel1/channel2 in error form, Sec. 4.3).  The sum includes m = i,
    i.e. the diagonal channel potential V_ii sits on the block diagonal.
    """

    def __init__(self, g: Grid1D, Vone: np.ndarray, lam: np.ndarray,
                 Vch: np.ndarray, E: float):
        n, M = g.n, len(lam)
        self.n, self.M = n, M
        N = (n - 1) * M
        ab = np.zeros((2 * M + 1, N), np.complex128)     # LAPACK band storage, kl=ku=M

        def put(row, col, val):
            ab[M + row - col, col] = val

        for t in range(1, n):
            for i in range(M):
                r = (t - 1) * M + i
                for m in range(M):
                    v = Vch[t, i, m]
                    if m == i:
                        v = v + g.b[t] + Vone[t] + lam[i] - E
                    put(r, (t - 1) * M + m, v)
                if t > 1:
                    put(r, (t - 2) * M + i, g.a[t])
                if t < n - 1:
                    put(r, t * M + i, g.c[t])
        self.ab = ab

    def solve(self, rhs: np.ndarray) -> np.ndarray:
        """rhs[t, i] for t = 0..n (rows 0 and n ignored) -> e (same shape)."""
        n, M = self.n, self.M
        x = sla.solve_banded((M, M), self.ab, rhs[1:n].reshape(-1))
        out = np.zeros_like(rhs)
        out[1:n] = x.reshape(n - 1, M)
        return out


class CCCS:
    """One Coupled Channel Correction Step on the finest level."""

    def __init__(self, op: Operator, M: int, L: int | None = None, refine_steps: int = 2):
        g = op.g
        L = M if L is None else L
        self.op = op
        self.lamA, self.phi = bound_states(g, op.V1, M, refine_steps)     # channels in x1
        self.lamB, self.vphi = bound_states(g, op.V2, L, refine_steps)    # channels in x2
        self.VA = channel_potential(g, op.V12, self.phi, "A")
        self.VB = channel_potential(g, op.V12, self.vphi, "B")
        self.sysA = ChannelSystem(g, op.V2, self.lamA, self.VA, op.E)
        self.sysB = ChannelSystem(g, op.V1, self.lamB, self.VB, op.E)

    def project(self, r: np.ndarray):
        """rho^A[k, i] = sum_j w_j phi_i(j) r[k, j];
        rho^B[j, l] = sum_k w_k varphi_l(k) r[k, j];
        c[i, l] = sum_{k,j} w_j w_k phi_i(j) varphi_l(k) r[k, j]  (eq. coefficients)."""
        w = self.op.g.w
        rhoA = r @ (w[:, None] * self.phi.T)            # [k, i]
        rhoB = r.T @ (w[:, None] * self.vphi.T)         # [j, l]
        c = (w[:, None] * self.vphi.T).T @ rhoA         # [l, i]
        return rhoA, rhoB, c.T                          # c as [i, l]

    def channel_rhs(self, r: np.ndarray):
        """Unique expansion of the residual (Remark 4): with c[i,l] from
        eq. coefficients, a_{l i} = c[i,l] for l <= i (else 0) and
        b_{i l} = c[i,l] for l > i (else 0);
        r^A_i = rho^A_i - sum_l b_il varphi_l,  r^B_l = rho^B_l - sum_m a_lm phi_m."""
        rhoA, rhoB, c = self.project(r)
        M, L = c.shape
        i_idx = np.arange(M)[:, None]
        l_idx = np.arange(L)[None, :]
        b = np.where(l_idx > i_idx, c, 0)           # b[i, l]
        a = np.where(l_idx <= i_idx, c, 0).T        # a[l, i]
        rA = rhoA - self.vphi.T @ b.T               # [k, i]: sum_l b[i,l] varphi_l(k)
        rB = rhoB - self.phi.T @ a.T                # [j, l]: sum_m a[l,m] phi_m(j)
        return rA, rB

    def correction(self, r: np.ndarray) -> np.ndarray:
        """e* = sum_m e^A_m(y) phi_m(x) + sum_l e^B_l(x) varphi_l(y) for residual r."""
        rA, rB = self.channel_rhs(r)
        eA = self.sysA.solve(rA)                    # [k, i]
        eB = self.sysB.solve(rB)                    # [j, l]
        return eA @ self.phi + (eB @ self.vphi).T   # [k, j]

    def expand(self, rA: np.ndarray, rB: np.ndarray) -> np.ndarray:
        """r* = sum_m r^A_m(y) phi_m(x) + sum_l r^B_l(x) varphi_l(y)."""
        return rA @ self.phi + (rB @ self.vphi).T

    def step(self, u: np.ndarray, f: np.ndarray) -> np.ndarray:
        """u* = u + e*(f - A u)  (eq. cccs), new array."""
        return u + self.correction(self.op.residual(u, f))
