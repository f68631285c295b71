"""GPU parity of the adjoint gradient d sigma / d(Z1, Z2, lambda) (differentiation
pattern) against the oracle's adjoint and central differences."""
import math

import numpy as np
import pytest

from helpers import Case, to_np
from oracle import functional as fn
from oracle.grid import Grid1D

pytestmark = pytest.mark.gpu
GAM = math.radians(5.0)


@pytest.mark.parametrize("p", [(1.0, 1.0, 1.0), (1.1, 0.9, 1.3)])
def test_gradient_matches_oracle_adjoint(p):
    from paper_1412_1953_amd import mgcccs
    c = Case(64, 20.0, 0.5, 4, 4, pc_gamma=GAM, Z1=p[0], Z2=p[1], lam=p[2])
    g = c.grid()
    chi = g.build_rhs_tp(g.field())
    u = g.field()
    res = g.solve(u, chi, outer=mgcccs.FGMRES, restart=10, max_it=3000, tol=1e-13)
    assert res.status == mgcccs.MGC_OK
    k = math.sqrt(c.E)
    v = g.field()
    ds, zeta, sig, ares = g.cross_section_grad(u, chi, k, k, v, tol=1e-13)
    assert ares.status == mgcccs.MGC_OK
    go = Grid1D(c.n, c.L, c.R0, c.theta)
    ref, info = fn.grad_adjoint(go, p, c.E, k, k)
    assert abs(sig - info["J"]) < 1e-9 * info["J"]
    assert abs(zeta - info["zeta"]) < 1e-9 * abs(info["zeta"])
    assert np.all(np.abs(np.array(ds) - ref) <= 1e-6 * np.abs(ref)), (ds, ref)
    # the adjoint field itself
    vo = info["v"]
    assert np.linalg.norm(to_np(v) - vo) / np.linalg.norm(vo) < 1e-9


def test_gradient_513_matches_oracle_adjoint():
    """The differentiation workload's spacing (h = 0.078125, ECS beyond
    0.75 L at pi/6, 8 channels, E = 0.5, Z1 = Z2 = lambda = 1) on [0,40]^2:
    the library's adjoint gradient against the oracle's adjoint with sparse
    direct solves, to 1e-6 relative per component."""
    from paper_1412_1953_amd import mgcccs
    c = Case(512, 40.0, 0.5, 6, 8, pc_gamma=GAM)
    g = c.grid()
    chi = g.build_rhs_tp(g.field())
    u = g.from_numpy(c.u0())
    res = g.solve(u, chi, outer=mgcccs.FGMRES, restart=10, max_it=20000, tol=1e-12)
    assert res.status == mgcccs.MGC_OK, (res.iters, res.relres)
    k = math.sqrt(c.E)
    v = g.field()
    ds, zeta, sig, ares = g.cross_section_grad(u, chi, k, k, v, tol=1e-12, max_it=20000)
    assert ares.status == mgcccs.MGC_OK, (ares.iters, ares.relres)
    go = Grid1D(c.n, c.L, c.R0, c.theta)
    ref, info = fn.grad_adjoint(go, (c.Z1, c.Z2, c.lam), c.E, k, k)
    print(f"513^2: forward {res.iters} it, adjoint {ares.iters} it; sigma {sig:.9e} vs {info['J']:.9e}; "
          f"gradient {np.array(ds)} vs {ref}")
    assert abs(sig - info["J"]) < 1e-8 * info["J"]
    assert np.all(np.abs(np.array(ds) - ref) <= 1e-6 * np.abs(ref)), (ds, ref)


def test_autograd_function_matches_central_differences():
    import torch
    from paper_1412_1953_amd import autograd
    c = Case(64, 20.0, 0.5, 4, 4, pc_gamma=GAM)
    g = c.grid()
    k = math.sqrt(c.E)
    u0 = g.field()
    params = torch.tensor([1.0, 1.0, 1.0], dtype=torch.float64, requires_grad=True)
    J = autograd.IonizationCrossSection.apply(params, g, c.E, k, k, u0)
    J.backward()
    grad = params.grad.numpy()
    h = 1e-5
    fd = np.zeros(3)
    for q in range(3):
        pp = params.detach().clone()
        pm = params.detach().clone()
        pp[q] += h
        pm[q] -= h
        Jp = autograd.IonizationCrossSection.apply(pp, g, c.E, k, k, u0).item()
        Jm = autograd.IonizationCrossSection.apply(pm, g, c.E, k, k, u0).item()
        fd[q] = (Jp - Jm) / (2 * h)
    assert np.all(np.abs(grad - fd) <= 1e-6 * np.abs(fd)), (grad, fd)


def test_transpose_solve_solves_the_transposed_system():
    import scipy.sparse as sp
    from paper_1412_1953_amd import mgcccs
    c = Case(32, 10.0, 0.3, 3, 2, pc_gamma=GAM)
    g = c.grid()
    o = c.oracle()
    n = c.n
    rhs = c.rand(5)
    vt, gt = g.field(), g.from_numpy(rhs)
    res = g.solve_transpose(vt, gt, outer=mgcccs.FGMRES, restart=10, max_it=2000, tol=1e-13)
    assert res.status == mgcccs.MGC_OK
    AT = o.op.sparse().T
    v = to_np(vt)[1:n, 1:n].ravel()
    r = AT @ v - rhs[1:n, 1:n].ravel()
    assert np.linalg.norm(r) / np.linalg.norm(rhs) < 1e-11
