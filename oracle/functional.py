"""Ionisation amplitude and cross section (TEST INFRASTRUCTURE ONLY).

Sec. 3.3: the double-ionisation amplitude (eq. double-ionization)
    zeta(k1,k2) = int phi_{k1}(x) phi_{k2}(y) (f - V12 u) dx dy
with phi_k the regular solution of (-1/2 d^2/dx^2 + V1 - k^2/2) phi_k = 0
(eq. testfunction) "normalised by 1/sqrt(k)", and
    sigma(k1,k2) = 8 pi^2 / k0^2 * |zeta|^2 / (k1 k2).

Readings (the paper leaves them open for an ECS grid): the integral runs over
the real region x, y <= R0 with trapezoid weights (h, and h/2 at R0);
phi_k comes from the 3-point recurrence of eq. testfunction on the real nodes
and is scaled so that its local amplitude at R0,
    a^2 = phi(R0)^2 + (phi'(R0)/p)^2,   p = sqrt(k^2 - 2 V1(R0)),
equals 1/sqrt(p).  Physical cross-section values are parity unpinned (the
paper prints none for this model); the pins are the Z1 = 0 closed form and
linearity in u.
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


def sigma(z: complex, E: float, Z1: float, k1: float, k2: float) -> float:
    """sigma = 8 pi^2 / k0^2 |zeta|^2 / (k1 k2), k0^2 = 2 (E + Z1^2/2)."""
    k0sq = 2.0 * (E + 0.5 * Z1 * Z1)
    return 8.0 * math.pi ** 2 / k0sq * abs(z) ** 2 / (k1 * k2)
