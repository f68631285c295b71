"""Ionisation amplitude and cross section (TEST INFRASTRUCTURE ONLY).

Sec. 3.3: the double-ionisation amplitude (eq. double-ionization)
    zeta(k1,k2) = int phi_{k1}(x) phi_{k2}(y) (f - V12 u) dx dy
with phi_k the regular solution of (-1/2 d^2/dx^2 + V1 - k^2/2) phi_k = 0
(eq. testfunction), normalised as in eq. testfunction (Sec. 3.3) to
asymptotic amplitude 1/sqrt(k), and
    sigma(k1,k2) = 8 pi^2 / k0^2 * |zeta|^2 / (k1 k2).

Under the exponential model (Sec. 3.3 Fig. 4) the same definitions take that
model's potentials (the *_model functions at the end).

Readings (the paper leaves them open for an ECS grid): the integral runs over
the real region x, y <= R0 with trapezoid weights (h, and h/2 at R0);
phi_k comes from the 3-point recurrence of eq. testfunction on the real nodes
and is scaled so that its local amplitude at R0,
    a^2 = phi(R0)^2 + (phi'(R0)/p)^2,   p = sqrt(k^2 - 2 V1(R0)),
equals 1/sqrt(p).  Physical cross-section values are parity unpinned (the
paper prints none for this model); the pins are the Z1 = 0 closed form, the
Z1 > 0 shape against the regular Coulomb function F_0(-Z1/k, kx) (second
order in h, amplitude 1/sqrt(k)), linearity in u, the factorisation for a
separable source and the exchange symmetry of the two coordinates.
"""
from __future__ import annotations

import math

import numpy as np

from .grid import Grid1D


def test_function(g: Grid1D, Z1: float, k: float) -> np.ndarray:
    """phi_k on the real nodes 0 .. min(j0+1, n) (array of that length + 1)."""
    h, j0, n = g.h, g.j0, g.n
    top = min(j0 + 1, n)
    ph = np.zeros(top + 1)
    ph[1] = h
    for j in range(1, top):
        V1 = -Z1 / (j * h)
        # -1/2 (phi_{j+1} - 2 phi_j + phi_{j-1}) / h^2 + (V1 - k^2/2) phi_j = 0
        ph[j + 1] = 2.0 * ph[j] - ph[j - 1] + 2.0 * h * h * (V1 - 0.5 * k * k) * ph[j]
    jr = min(j0, top - 1)
    p = math.sqrt(k * k - 2.0 * (-Z1 / (jr * h)))
    dphi = (ph[jr + 1] - ph[jr - 1]) / (2.0 * h)
    amp = math.sqrt(ph[jr] ** 2 + (dphi / p) ** 2)
    return ph / (amp * math.sqrt(p))


def trapezoid_weights(g: Grid1D) -> np.ndarray:
    """t_j on nodes 0..n: h on 1..j0-1, h/2 at j0, zero elsewhere."""
    t = np.zeros(g.n + 1)
    top = min(g.j0, g.n - 1)
    t[1:top + 1] = g.h
    if g.j0 <= g.n - 1:
        t[g.j0] = 0.5 * g.h
    return t


def zeta(g: Grid1D, Z1: float, lam: float, u: np.ndarray, chi: np.ndarray,
         k1: float, k2: float) -> complex:
    """Double-ionisation amplitude over the real region (eq. double-ionization)."""
    n = g.n
    t = trapezoid_weights(g)
    f1 = np.zeros(n + 1)
    f2 = np.zeros(n + 1)
    p1 = test_function(g, Z1, k1)
    p2 = test_function(g, Z1, k2)
    top = min(g.j0, n - 1)
    f1[1:top + 1] = t[1:top + 1] * p1[1:top + 1]
    f2[1:top + 1] = t[1:top + 1] * p2[1:top + 1]
    idx = np.arange(n + 1)
    m = np.maximum(idx[:, None], idx[None, :])
    zr = g.z.copy()
    zr[0] = 1.0                                # never used (weights vanish on the ring)
    V12 = lam / zr[m]
    src = chi - V12 * u
    return complex(f2 @ src @ f1)              # sum_k f2[k] sum_j src[k, j] f1[j]


def zeta_sweep(g: Grid1D, Z1: float, lam: float, u: np.ndarray, chi: np.ndarray, k1s, k2s) -> list:
    """zeta for each momentum pair (k1s[a], k2s[a]), pair by pair.  An energy
    sharing sweep (Sec. 3.3) takes k1 = K cos a, k2 = K sin a, K^2/2 the excess
    energy, for a in [0, pi/2]."""
    return [zeta(g, Z1, lam, u, chi, k1, k2) for k1, k2 in zip(k1s, k2s)]


def sigma(z: complex, E: float, Z1: float, k1: float, k2: float) -> float:
    """sigma = 8 pi^2 / k0^2 |zeta|^2 / (k1 k2), k0^2 = 2 (E + Z1^2/2)."""
    k0sq = 2.0 * (E + 0.5 * Z1 * Z1)
    return 8.0 * math.pi ** 2 / k0sq * abs(z) ** 2 / (k1 * k2)


# ---------------------------------------------------------------------------
# Objective J(p) = sigma(k1, k2) of u = A(p)^{-1} chi(p), p = (Z1, Z2, lambda),
# and its gradient (test infrastructure for the adjoint of the HIP library).
def objective(g: Grid1D, p, E: float, k1: float, k2: float):
    """J and the pieces it is built from, with an exact sparse direct solve."""
    import scipy.sparse.linalg as spla
    from .grid import tp_operator, tp_rhs
    Z1, Z2, lam = p
    n = g.n
    op = tp_operator(g, Z1, Z2, lam, E)
    chi = tp_rhs(g, Z1, Z2, lam, E)
    lu = spla.splu(op.sparse())
    u = np.zeros_like(chi)
    u[1:n, 1:n] = lu.solve(chi[1:n, 1:n].ravel()).reshape(n - 1, n - 1)
    z = zeta(g, Z1, lam, u, chi, k1, k2)
    return sigma(z, E, Z1, k1, k2), dict(op=op, chi=chi, u=u, zeta=z, lu=lu)


def grad_central(g: Grid1D, p, E, k1, k2, step=1e-5):
    """Central differences of J with exact solves."""
    out = np.zeros(3)
    for q in range(3):
        pp, pm = list(p), list(p)
        pp[q] += step
        pm[q] -= step
        out[q] = (objective(g, pp, E, k1, k2)[0] - objective(g, pm, E, k1, k2)[0]) / (2 * step)
    return out


def grad_adjoint(g: Grid1D, p, E, k1, k2, fd_step=1e-6):
    """dJ/dp through the holomorphic adjoint A^T v = d zeta/du.  The explicit
    partial derivatives of chi, V12 and the test functions are taken by central
    differences of their (closed-form) builders, which are cheap and exact to
    O(fd_step^2)."""
    import scipy.sparse.linalg as spla
    from .grid import tp_rhs, tp_two_body
    Z1, Z2, lam = p
    n = g.n
    J, s = objective(g, p, E, k1, k2)
    u, chi, zt = s["u"], s["chi"], s["zeta"]
    t = trapezoid_weights(g)
    top = min(g.j0, n - 1)

    def weights(Z):
        f1, f2 = np.zeros(n + 1), np.zeros(n + 1)
        f1[1:top + 1] = t[1:top + 1] * test_function(g, Z, k1)[1:top + 1]
        f2[1:top + 1] = t[1:top + 1] * test_function(g, Z, k2)[1:top + 1]
        return np.outer(f2, f1)                          # F[k, j]

    F = weights(Z1)
    V12 = tp_two_body(g, lam)
    gu = -F * V12                                        # d zeta / du (holomorphic)
    AT = s["op"].sparse().T.tocsc()
    v = np.zeros_like(u)
    v[1:n, 1:n] = spla.spsolve(AT, gu[1:n, 1:n].ravel()).reshape(n - 1, n - 1)
    zz = g.z.copy()
    zz[0] = 1.0
    inv = 1.0 / zz
    dA = [np.zeros_like(u) for _ in range(3)]
    dA[0][1:n, 1:n] = -np.broadcast_to(inv[None, 1:n], (n - 1, n - 1))
    dA[1][1:n, 1:n] = -np.broadcast_to(inv[1:n, None], (n - 1, n - 1))
    idx = np.arange(n + 1)
    dA[2] = np.where((idx[:, None] > 0) & (idx[None, :] > 0) & (idx[:, None] < n) & (idx[None, :] < n),
                     inv[np.maximum(idx[:, None], idx[None, :])], 0)
    dJ = np.zeros(3)
    k0sq = 2 * E + Z1 ** 2
    C = 8 * np.pi ** 2 / (k0sq * k1 * k2)
    for q in range(3):
        pp, pm = list(p), list(p)
        pp[q] += fd_step
        pm[q] -= fd_step
        dchi = (tp_rhs(g, *pp, E) - tp_rhs(g, *pm, E)) / (2 * fd_step)
        dF = (weights(pp[0]) - weights(pm[0])) / (2 * fd_step) if q == 0 else 0.0
        dV12 = dA[2] if q == 2 else 0.0
        explicit = np.sum(dF * (chi - V12 * u)) + np.sum(F * (dchi - dV12 * u))
        adjoint = np.sum(v * (dchi - dA[q] * u))
        dz = explicit + adjoint
        dJ[q] = 2 * C * np.real(np.conj(zt) * dz)
    dJ[0] += -J * 2 * Z1 / k0sq
    return dJ, dict(J=J, v=v, zeta=zt)


# ---------------------------------------------------------------------------
# Single ionisation and the total double-ionisation cross section (Sec. 3.3).
def source_term(g: Grid1D, lam: float, u: np.ndarray, chi: np.ndarray) -> np.ndarray:
    """f - V12 u on every node (V12 = lambda / z_max(j,k); the ring is never
    weighted)."""
    n = g.n
    idx = np.arange(n + 1)
    m = np.maximum(idx[:, None], idx[None, :])
    zr = g.z.copy()
    zr[0] = 1.0
    return chi - (lam / zr[m]) * u


def single_ionization(g: Grid1D, Z1: float, Z2: float, lam: float, E: float,
                      u: np.ndarray, chi: np.ndarray, nstates: int):
    """Single-ionisation amplitudes s_n(E), n = 1 .. nstates (eq. single-ionization):
        s_n = sum_{j,k <= j0} t_j t_k phi_{k_n}(x1_j) phi_n(x2_k) (f - V12 u)_{kj},
    phi_n the n-th lowest bound state of the x2 one-body Hamiltonian
    -1/2 d^2/dz^2 - Z2/z on the exterior-complex-scaled grid (eq. 1d_eigenstate,
    bilinear normalisation), k_n = sqrt(2 (E - lambda_n)) and phi_{k_n} the
    test function of eq. testfunction in x1.  Readings: the real region with
    trapezoid weights as for zeta; k_n from the real part of the discrete
    eigenvalue (its imaginary part is round-off for a true bound state).
    Returns (lambda_n, k_n, s_n) as arrays."""
    from .cccs import bound_states
    from .grid import tp_one_body
    n, top = g.n, min(g.j0, g.n - 1)
    lamB, vphi = bound_states(g, tp_one_body(g, Z2), nstates)
    t = trapezoid_weights(g)
    src = source_term(g, lam, u, chi)
    ks, out = [], []
    for q in range(nstates):
        kq = math.sqrt(2.0 * (E - lamB[q].real))
        p1 = test_function(g, Z1, kq)
        f1 = np.zeros(n + 1)
        f1[1:top + 1] = t[1:top + 1] * p1[1:top + 1]
        f2 = np.zeros(n + 1, np.complex128)
        f2[1:top + 1] = t[1:top + 1] * vphi[q, 1:top + 1]
        ks.append(kq)
        out.append(complex(f2 @ src @ f1))
    return lamB, np.array(ks), np.array(out)


def sigma_total(g: Grid1D, Z1: float, lam: float, E: float, u: np.ndarray, chi: np.ndarray,
                nodes: int = 32) -> float:
    """Total double-ionisation cross section (eq. total-double-ionization),
        sigma_tot(E) = int_0^E sigma(sqrt(2 eps), sqrt(2 (E - eps))) d eps,
    with eps = E sin^2 a (k1 = sqrt(2E) sin a, k2 = sqrt(2E) cos a, the
    sharing angle of the sweeps): the Jacobian 2 E sin a cos a cancels the
    1/(k1 k2) of sigma, so
        sigma_tot = 8 pi^2 / k0^2 int_0^{pi/2} |zeta(k1(a), k2(a))|^2 da,
    a smooth integrand, taken by Gauss-Legendre quadrature with `nodes` points."""
    x, w = np.polynomial.legendre.leggauss(nodes)
    a = (x + 1.0) * math.pi / 4.0
    wa = w * math.pi / 4.0
    K = math.sqrt(2.0 * E)
    zs = zeta_sweep(g, Z1, lam, u, chi, K * np.sin(a), K * np.cos(a))
    k0sq = 2.0 * (E + 0.5 * Z1 * Z1)
    return float(8.0 * math.pi ** 2 / k0sq * np.sum(wa * np.abs(np.array(zs)) ** 2))


# ---------------------------------------------------------------------------
# The same amplitudes under a general potential model (TPModel or ExpModel of
# oracle.grid): the test functions take the model's x1 potential at the real
# nodes, the source the model's V12, and the prefactor's k0^2 is twice the
# energy of the incoming electron over the target's ground state,
# 2 (E - lambda_1) with lambda_1 the lowest x1 bound state (Temkin-Poet:
# lambda_1 = -Z1^2 / 2 in closed form, as above).
def model_v1_real(g: Grid1D, model) -> np.ndarray:
    """V1 at the real nodes x_j = j h, j = 1 .. n (entry 0 unused)."""
    from .grid import ExpModel
    V = np.zeros(g.n + 1)
    x = g.h * np.arange(1, g.n + 1)
    if isinstance(model, ExpModel):
        V[1:] = -model.a1 * np.exp(-model.b1 * x * x)
    else:
        V[1:] = -model.Z1 / x
    return V


def test_function_v(g: Grid1D, V1: np.ndarray, k: float) -> np.ndarray:
    """phi_k of eq. testfunction with the potential table V1 (real nodes):
    the 3-point recurrence and the local-amplitude scaling of test_function."""
    h, j0, n = g.h, g.j0, g.n
    top = min(j0 + 1, n)
    ph = np.zeros(top + 1)
    ph[1] = h
    for j in range(1, top):
        ph[j + 1] = 2.0 * ph[j] - ph[j - 1] + 2.0 * h * h * (V1[j] - 0.5 * k * k) * ph[j]
    jr = min(j0, top - 1)
    p = math.sqrt(k * k - 2.0 * V1[jr])
    dphi = (ph[jr + 1] - ph[jr - 1]) / (2.0 * h)
    amp = math.sqrt(ph[jr] ** 2 + (dphi / p) ** 2)
    return ph / (amp * math.sqrt(p))


def model_k0sq(g: Grid1D, model, E: float) -> float:
    from .cccs import bound_states
    from .grid import ExpModel, exp_one_body
    if not isinstance(model, ExpModel):
        return 2.0 * (E + 0.5 * model.Z1 * model.Z1)
    lam, _ = bound_states(g, exp_one_body(g, model.a1, model.b1), 1)
    return 2.0 * (E - lam[0].real)


def model_source(g: Grid1D, model, u: np.ndarray, chi: np.ndarray) -> np.ndarray:
    """chi - V12 u with the model's two-body potential (zero on the ring)."""
    return chi - model.potentials(g)[2] * u


def _weights(g: Grid1D, vals: np.ndarray) -> np.ndarray:
    n, top = g.n, min(g.j0, g.n - 1)
    t = trapezoid_weights(g)
    f = np.zeros(n + 1, vals.dtype)
    f[1:top + 1] = t[1:top + 1] * vals[1:top + 1]
    return f


def zeta_model(g: Grid1D, model, u: np.ndarray, chi: np.ndarray, k1: float, k2: float) -> complex:
    V1 = model_v1_real(g, model)
    f1 = _weights(g, test_function_v(g, V1, k1))
    f2 = _weights(g, test_function_v(g, V1, k2))
    return complex(f2 @ model_source(g, model, u, chi) @ f1)


def single_ionization_model(g: Grid1D, model, E: float, u: np.ndarray, chi: np.ndarray, nstates: int):
    """(lambda_n, k_n, s_n) of eq. single-ionization under the model: phi_n the
    bound states of the x2 one-body Hamiltonian, phi_{k_n} in x1."""
    from .cccs import bound_states
    V2 = model.potentials(g)[1]
    lamB, vphi = bound_states(g, V2, nstates)
    V1 = model_v1_real(g, model)
    src = model_source(g, model, u, chi)
    ks, out = [], []
    for q in range(nstates):
        kq = math.sqrt(2.0 * (E - lamB[q].real))
        f1 = _weights(g, test_function_v(g, V1, kq))
        f2 = _weights(g, vphi[q])
        ks.append(kq)
        out.append(complex(f2 @ src @ f1))
    return lamB, np.array(ks), np.array(out)


def sigma_total_model(g: Grid1D, model, E: float, u: np.ndarray, chi: np.ndarray, nodes: int = 32) -> float:
    """sigma_tot of eq. total-double-ionization under the model (the
    Gauss-Legendre form of sigma_total)."""
    x, w = np.polynomial.legendre.leggauss(nodes)
    a = (x + 1.0) * math.pi / 4.0
    wa = w * math.pi / 4.0
    K = math.sqrt(2.0 * E)
    zs = np.array([zeta_model(g, model, u, chi, K * math.sin(t), K * math.cos(t)) for t in a])
    return float(8.0 * math.pi ** 2 / model_k0sq(g, model, E) * np.sum(wa * np.abs(zs) ** 2))
