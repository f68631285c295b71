"""torch.autograd.Function for the ionisation cross section of the Temkin-Poet
problem: J(Z1, Z2, lambda) = sigma(k1, k2) of u = A^{-1} chi (Sec. 3.3,
eqs. double-ionization and total-double-ionization).

forward  : set_potential, set_energy, build_rhs_tp, MG-CCCS solve, cross_section
backward : mgc_cross_section_grad (adjoint MG-CCCS solve on the transposed,
           complex-symmetric operator, Sec. 2.5)
All arithmetic runs in the HIP library; this module only marshals arguments.
"""
from __future__ import annotations

import torch

from . import mgcccs


class IonizationCrossSection(torch.autograd.Function):
    @staticmethod
    def forward(ctx, params, grid, E, k1, k2, u0, tol=1e-13, restart=10, max_it=20000):
        Z1, Z2, lam = (float(x) for x in params.detach().cpu().tolist())
        grid.set_potential(Z1, Z2, lam)
        grid.set_energy(E)
        chi = grid.build_rhs_tp(grid.field())
        u = grid.field()
        u.copy_(u0)
        res = grid.solve(u, chi, outer=mgcccs.FGMRES, restart=restart, max_it=max_it, tol=tol)
        if res.status != mgcccs.MGC_OK:
            raise mgcccs.MGCError(res.status, f"forward solve stopped at relres {res.relres:.3e}")
        _, sig = grid.cross_section(u, chi, k1, k2)
        ctx.grid, ctx.state = grid, (Z1, Z2, lam, E, k1, k2, tol, restart, max_it)
        ctx.u, ctx.chi = u, chi
        return params.new_tensor(sig)

    @staticmethod
    def backward(ctx, gout):
        grid = ctx.grid
        Z1, Z2, lam, E, k1, k2, tol, restart, max_it = ctx.state
        grid.set_potential(Z1, Z2, lam)      # the handle may have moved on since forward
        grid.set_energy(E)
        v = grid.field()
        ds, _, _, res = grid.cross_section_grad(ctx.u, ctx.chi, k1, k2, v, restart=restart,
                                                max_it=max_it, tol=tol)
        if res.status != mgcccs.MGC_OK:
            raise mgcccs.MGCError(res.status, f"adjoint solve stopped at relres {res.relres:.3e}")
        g = gout * gout.new_tensor(ds)
        return g, None, None, None, None, None, None, None, None


def cross_section(params, grid, E, k1, k2, u0, **kw):
    """sigma(k1, k2) as a differentiable function of params = (Z1, Z2, lambda)."""
    return IonizationCrossSection.apply(params, grid, E, k1, k2, u0, *kw.values())
