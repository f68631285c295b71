"""Grid, operator and right-hand side of the discretised 2D driven Schroedinger
equation (TEST INFRASTRUCTURE ONLY; see ``oracle/__init__``).

Problem (Sec. 2.2, eq. partialwave2d):
    (-1/2 Laplace + V1(x) + V2(y) + V12(x,y) - E) u = f,   u = 0 on x = 0 or y = 0,
discretised with the 3-point finite-difference Laplacian (Sec. 2.5,
eq. discrete_schrodinger) on a uniform real grid whose coordinates are
rotated into the complex plane beyond R0 (exterior complex scaling, Sec. 2.5
and Sec. 3.3).  Temkin-Poet potentials V1 = -Z1/x, V2 = -Z2/y,
V12 = lambda/max(x,y) (Sec. 5.2 and Sec. 6.2), or the exponential model
V1 = -a1 exp(-b1 x^2), V2 = -a2 exp(-b2 y^2), V12 = c12 exp(-d12 (x+y)^2)
(Sec. 6.1; Sec. 3.3 Fig. 4).

Arrays are full ``(n+1, n+1)`` complex arrays indexed ``[k, j]`` with ``k``
along x2 (= y) and ``j`` along x1 (= x); row/column 0 and n are the Dirichlet
ring and stay zero.
"""
from __future__ import annotations

import math

import numpy as np


class Grid1D:
    """One coordinate axis: nodes x_j = j h on [0, L], complex nodes z_j.

    ECS map (Sec. 2.5, Sec. 3.3; reading: node-based, R0 on a grid node),
    optionally preceded by the complex-contour rotation of Sec. 3.1
    (z = x e^{i gamma}, the rotated domain Z_1) on the interior:
        z_j = x_j exp(i gamma)                            for x_j <= R0
        z_j = R0 exp(i gamma) + (x_j - R0) exp(i theta)   for x_j >  R0
    gamma = 0 is the exterior-complex-scaled grid with a real interior.
    Spacings h_j = z_{j+1} - z_j, dual weights w_j = (h_{j-1} + h_j)/2 and the
    3-point coefficients of -1/2 d^2/dz^2 on the non-uniform complex grid:
        (-1/2 u'')_j ~ a_j u_{j-1} + b_j u_j + c_j u_{j+1}
        a_j = -1/(2 w_j h_{j-1}),  c_j = -1/(2 w_j h_j),
        b_j = (1/h_{j-1} + 1/h_j)/(2 w_j).
    Index 0 and n of w, a, b, c are zero (the ring carries no unknown).
    """

    def __init__(self, n: int, L: float, R0: float, theta: float, gamma: float = 0.0):
        if n < 2:
            raise ValueError("need at least 2 intervals")
        self.n, self.L, self.R0, self.theta = n, float(L), float(R0), float(theta)
        self.gamma = float(gamma)
        self.h = self.L / n
        j0 = int(round(self.R0 / self.h))
        if abs(j0 * self.h - self.R0) > 1e-9 * self.L or not (0 < j0 <= n):
            raise ValueError("R0 must lie on a grid node")
        self.j0 = j0
        self.x = self.h * np.arange(n + 1, dtype=np.float64)
        z = self.x * np.exp(1j * self.gamma)
        z[j0 + 1:] = (self.R0 * np.exp(1j * self.gamma)
                      + (self.x[j0 + 1:] - self.R0) * np.exp(1j * self.theta))
        self.z = z
        hs = z[1:] - z[:-1]                      # h_j for j = 0 .. n-1
        self.hs = hs
        w = np.zeros(n + 1, np.complex128)
        a = np.zeros(n + 1, np.complex128)
        b = np.zeros(n + 1, np.complex128)
        c = np.zeros(n + 1, np.complex128)
        hm, hp = hs[:-1], hs[1:]                 # h_{j-1}, h_j for j = 1 .. n-1
        w[1:n] = 0.5 * (hm + hp)
        a[1:n] = -1.0 / (2.0 * w[1:n] * hm)
        c[1:n] = -1.0 / (2.0 * w[1:n] * hp)
        b[1:n] = (1.0 / hm + 1.0 / hp) / (2.0 * w[1:n])
        self.w, self.a, self.b, self.c = w, a, b, c

    def coarsen(self, gamma: float | None = None) -> "Grid1D":
        """Same domain, ECS start and angle at twice the spacing (rotation
        ``gamma``, default: this grid's)."""
        if self.n % 2:
            raise ValueError("odd interval count cannot be coarsened")
        return Grid1D(self.n // 2, self.L, self.R0, self.theta,
                      self.gamma if gamma is None else gamma)

    # ---- 1D Hamiltonians -------------------------------------------------
    def hamiltonian_dense(self, V: np.ndarray) -> np.ndarray:
        """Dense (n-1)x(n-1) matrix of H = -1/2 d^2/dz^2 + V on the interior
        nodes (row j-1 <-> node j), in the unweighted (row-scaled) form."""
        n = self.n
        H = np.zeros((n - 1, n - 1), np.complex128)
        i = np.arange(n - 1)
        H[i, i] = self.b[1:n] + V[1:n]
        H[i[1:], i[1:] - 1] = self.a[2:n]
        H[i[:-1], i[:-1] + 1] = self.c[1:n - 1]
        return H

    def weighted_hamiltonian_dense(self, V: np.ndarray) -> np.ndarray:
        """S = W H with W = diag(w): the complex-symmetric form (Sec. 2.5)."""
        return self.w[1:self.n, None] * self.hamiltonian_dense(V)


def tp_one_body(g: Grid1D, Z: float) -> np.ndarray:
    """-Z/z_j on the interior nodes, zero on the ring."""
    V = np.zeros(g.n + 1, np.complex128)
    V[1:g.n] = -Z / g.z[1:g.n]
    return V


def tp_two_body(g: Grid1D, lam: float) -> np.ndarray:
    """V12[k, j] = lambda / z_{max(j,k)} on interior nodes (reading: the max is
    taken on the real grid parameter, then mapped; the ECS map is monotone)."""
    n = g.n
    V = np.zeros((n + 1, n + 1), np.complex128)
    idx = np.arange(1, n)
    m = np.maximum(idx[:, None], idx[None, :])
    V[1:n, 1:n] = lam / g.z[m]
    return V


def exp_one_body(g: Grid1D, a: float, b: float) -> np.ndarray:
    """-a exp(-b z_j^2) on the interior nodes, zero on the ring (the
    exponential model of Sec. 6.1 and Sec. 3.3 Fig. 4)."""
    V = np.zeros(g.n + 1, np.complex128)
    z = g.z[1:g.n]
    V[1:g.n] = -a * np.exp(-b * z * z)
    return V


def exp_two_body(g: Grid1D, c: float, d: float) -> np.ndarray:
    """V12[k, j] = c exp(-d (z_j + z_k)^2) on interior nodes (Sec. 6.1:
    c = 2, d = 0.1; Sec. 3.3 Fig. 4: c = 2, d = 1)."""
    n = g.n
    V = np.zeros((n + 1, n + 1), np.complex128)
    s = g.z[1:n, None] + g.z[None, 1:n]
    V[1:n, 1:n] = c * np.exp(-d * s * s)
    return V


class TPModel:
    """Temkin-Poet potentials -Z1/x1, -Z2/x2, lambda/max(x1, x2)."""

    def __init__(self, Z1: float, Z2: float, lam: float):
        self.Z1, self.Z2, self.lam = Z1, Z2, lam

    def potentials(self, g: Grid1D):
        return tp_one_body(g, self.Z1), tp_one_body(g, self.Z2), tp_two_body(g, self.lam)


class ExpModel:
    """Exponential potentials V1 = -a1 exp(-b1 x1^2), V2 = -a2 exp(-b2 x2^2),
    V12 = c12 exp(-d12 (x1 + x2)^2), continued analytically onto the complex
    nodes (Sec. 6.1; the defaults are its values)."""

    def __init__(self, a1=4.5, b1=1.0, a2=4.5, b2=1.0, c12=2.0, d12=0.1):
        self.a1, self.b1, self.a2, self.b2, self.c12, self.d12 = a1, b1, a2, b2, c12, d12

    def potentials(self, g: Grid1D):
        return (exp_one_body(g, self.a1, self.b1), exp_one_body(g, self.a2, self.b2),
                exp_two_body(g, self.c12, self.d12))


class Operator:
    """A = H1 (x) I + I (x) H2 + V12 - E  (Sec. 3.4, eq. hamiltonian2d),
    applied as the 5-point stencil

        (A u)_{k,j} = a_j u_{k,j-1} + c_j u_{k,j+1} + a_k u_{k-1,j} + c_k u_{k+1,j}
                      + (b_j + b_k + V1_j + V2_k + V12_{k,j} - E) u_{k,j}.
    """

    def __init__(self, g: Grid1D, V1: np.ndarray, V2: np.ndarray,
                 V12: np.ndarray, E: float):
        self.g, self.V1, self.V2, self.V12, self.E = g, V1, V2, V12, float(E)
        n = g.n
        d = np.zeros((n + 1, n + 1), np.complex128)
        d[1:n, 1:n] = (g.b[None, 1:n] + g.b[1:n, None] + V1[None, 1:n]
                       + V2[1:n, None] + V12[1:n, 1:n] - self.E)
        self.diag = d

    @property
    def n(self) -> int:
        return self.g.n

    def apply(self, u: np.ndarray) -> np.ndarray:
        g, n = self.g, self.g.n
        out = np.zeros_like(u)
        out[1:n, 1:n] = (g.a[None, 1:n] * u[1:n, 0:n - 1]
                         + g.c[None, 1:n] * u[1:n, 2:n + 1]
                         + g.a[1:n, None] * u[0:n - 1, 1:n]
                         + g.c[1:n, None] * u[2:n + 1, 1:n]
                         + self.diag[1:n, 1:n] * u[1:n, 1:n])
        return out

    def residual(self, u: np.ndarray, f: np.ndarray) -> np.ndarray:
        r = f - self.apply(u)
        r[0, :] = r[-1, :] = r[:, 0] = r[:, -1] = 0
        return r

    def sparse(self):
        """Assembled sparse matrix on the interior unknowns, flattened
        row-major in [k, j] (Kronecker form of eq. hamiltonian2d)."""
        import scipy.sparse as sp
        n, g = self.n, self.g
        H1 = self.g.hamiltonian_dense(self.V1)
        H2 = self.g.hamiltonian_dense(self.V2)
        I = sp.identity(n - 1, dtype=np.complex128, format="csr")
        A = (sp.kron(I, sp.csr_matrix(H1)) + sp.kron(sp.csr_matrix(H2), I)
             + sp.diags((self.V12[1:n, 1:n] - self.E).ravel()))
        return A.tocsc()


def tp_operator(g: Grid1D, Z1: float, Z2: float, lam: float, E: float) -> Operator:
    return Operator(g, tp_one_body(g, Z1), tp_one_body(g, Z2), tp_two_body(g, lam), E)


def model_operator(g: Grid1D, model, E: float) -> Operator:
    """The operator of a potential model (TPModel or ExpModel) on grid g."""
    return Operator(g, *model.potentials(g), E)


def tp_rhs(g: Grid1D, Z1: float, Z2: float, lam: float, E: float) -> np.ndarray:
    """Impact-ionisation right-hand side of the Temkin-Poet model.

    Incoming wave u_in = phi_1s(x1) sin(k0 x2) (Sec. 3.1 Remark 3 and
    Sec. 5.1), source (V2 + V12) u_in with V2 = -Z2/x2, V12 = lambda/max:
        chi0[k, j] = (lambda/z_max(j,k) - Z2/z_k) phi_1s(z_j) sin(k0 z_k),
        phi_1s(z) = 2 Z1^{3/2} z exp(-Z1 z),  k0 = sqrt(2 (E + Z1^2/2)).
    Reading: chi0 is confined to the real region j, k <= j0 (the sine grows
    on the complex part, Sec. 5.1), then symmetrised chi = (chi0 + chi0^T)/sqrt 2.
    """
    n, j0 = g.n, g.j0
    k0 = math.sqrt(2.0 * (E + 0.5 * Z1 * Z1))
    z = g.z
    chi0 = np.zeros((n + 1, n + 1), np.complex128)
    jj = np.arange(1, min(j0, n - 1) + 1)
    zj = z[jj]
    phi = 2.0 * Z1 ** 1.5 * zj * np.exp(-Z1 * zj)
    m = np.maximum(jj[:, None], jj[None, :])               # [k, j]
    chi0[np.ix_(jj, jj)] = ((lam / z[m] - Z2 / zj[:, None])
                            * phi[None, :] * np.sin(k0 * zj[:, None]))
    return (chi0 + chi0.T) / math.sqrt(2.0)


def rel_residual(op: Operator, u: np.ndarray, f: np.ndarray) -> float:
    """||f - A u||_2 / ||f||_2 over the interior nodes (unweighted 2-norm)."""
    r = op.residual(u, f)
    return float(np.linalg.norm(r) / np.linalg.norm(f))
