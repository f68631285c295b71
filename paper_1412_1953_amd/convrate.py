"""Convergence rate against the energy (the diagnostic of Sec. 6.1 / 6.2,
Fig. convrate2D): for each energy, the mean residual reduction per iteration
of four solvers built on the library,

  mg        stationary V(1,1) cycles, no channel correction (M = L = 0);
  mg-cccs   stationary MG-CCCS cycles (V-cycle + CCCS with M = L channels);
  bicgstab  BiCGSTAB right-preconditioned by one MG-CCCS cycle;
  fgmres    FGMRES(5) right-preconditioned by one MG-CCCS cycle,

on the Temkin-Poet system (Sec. 6.2) or the exponential-potential model
(Sec. 6.1: V1 = V2 = -4.5 exp(-x^2), V12 = 2 exp(-0.1 (x1 + x2)^2))
discretised on the full complex contour z = x e^{i gamma} (Sec. 3.1; R0 = L,
the multigrid hierarchy on the same contour) with the source
f = exp(-3 (z1 + z2)^2) of both sections, from a zero initial guess to a
relative residual of 1e-6 (Table 1) or an iteration cap.
rate = (||r_k|| / ||r_0||)^(1 / k) over the k iterations performed (one
iteration = one cycle for the stationary solvers, one Krylov step otherwise).

    python -m paper_1412_1953_amd.convrate OUT.json [n L gamma_deg M E0 E1 dE [smoother [model [levels]]]]

(smoother: 0 = omega-Jacobi, 1 = the GMRES(3) smoothing substitute; model: tp
or exp; Sec. 6.1's exponential case is 256 20 10 2 -2 3 0.25 1 exp).
"""
from __future__ import annotations

import json
import math
import sys


def contour_source(g, n, L, gamma, s=3.0):
    """exp(-s (z1 + z2)^2) at the contour nodes z_j = j (L/n) e^{i gamma}."""
    import torch
    h = L / n
    z = torch.arange(n + 1, dtype=torch.float64) * h * complex(math.cos(gamma), math.sin(gamma))
    f = torch.exp(-s * (z[:, None] + z[None, :]) ** 2).to(torch.complex128)
    f[0, :] = f[-1, :] = f[:, 0] = f[:, -1] = 0
    return g.from_numpy(f.numpy())


def rates(n=1024, L=100.0, gamma_deg=10.0, M=2, energies=None, levels=None, tol=1e-6, cap=200, smoother=0,
          model="tp", log=print):
    from . import mgcccs
    gamma = math.radians(gamma_deg)
    levels = levels or int(math.log2(n)) - 3           # coarsest 16 intervals
    energies = energies if energies is not None else [-2.0 + 0.25 * i for i in range(21)]
    out = []
    for E in energies:
        row = {"E": E, "smoother": "gmres3" if smoother else "jacobi", "model": model}
        for name, m, outer, restart in (("mg", 0, mgcccs.STATIONARY, 1), ("mg-cccs", M, mgcccs.STATIONARY, 1),
                                        ("bicgstab", M, mgcccs.BICGSTAB, 1), ("fgmres", M, mgcccs.FGMRES, 5)):
            g = mgcccs.Grid(n, L, L, math.pi / 6, levels, m, pc_gamma=gamma, pc_gamma0=gamma, pc_first_level=0,
                            gamma=gamma, max_restart=10, fp32=False, smoother=smoother,
                            pot_tables=1 if model == "exp" else 0)
            if model == "exp":
                g.set_potential_exp(4.5, 1.0, 4.5, 1.0, 2.0, 0.1)
            else:
                g.set_potential(1.0, 1.0, 1.0)
            g.set_energy(E)
            f = contour_source(g, n, L, gamma)
            u = g.field()
            r = g.solve(u, f, outer=outer, restart=restart, max_it=cap if outer != mgcccs.STATIONARY else 60,
                        tol=tol)
            h = r.history
            k = max(r.iters, 1)
            rate = (r.relres / h[0]) ** (1.0 / k) if math.isfinite(r.relres) and r.relres > 0 else float("inf")
            row[name] = {"rate": rate, "iters": r.iters, "relres": r.relres, "status": r.status}
            del g
        log(json.dumps(row))
        out.append(row)
    return out


if __name__ == "__main__":
    if len(sys.argv) < 2:
        raise SystemExit(__doc__)
    args = sys.argv[2:]
    kw = {}
    if args:
        n, L, gd, M, e0, e1, de = args[:7]
        if len(args) > 7:
            kw["smoother"] = int(args[7])
        if len(args) > 8:
            kw["model"] = args[8]
        if len(args) > 9:
            kw["levels"] = int(args[9])
        ne = int(round((float(e1) - float(e0)) / float(de))) + 1
        kw.update(n=int(n), L=float(L), gamma_deg=float(gd), M=int(M),
                  energies=[float(e0) + float(de) * i for i in range(ne)])
    res = rates(log=lambda m: print(m, flush=True), **kw)
    with open(sys.argv[1], "w") as fh:
        json.dump(res, fh, indent=1)
