"""Ionisation curves of the exponential model against the energy (the setup
of Sec. 3.3, Fig. 4): V1 = V2 = -4.5 exp(-x^2), V12 = 2 exp(-(x1 + x2)^2),
source exp(-3 (x1 + x2)^2), exterior complex scaling at pi/7 on the figure's
spacing h = 0.05 (here 512 intervals on [0, 25.6], real up to 12.8, so that
the multigrid hierarchy has its coarse levels).  For each energy E the system
is solved with MG-CCCS-preconditioned FGMRES, then

  |s_n(E)|^2 for the open single-ionisation channels (E > lambda_n; the
             channel's curve starts at its threshold lambda_n),
  sigma_tot(E) of double ionisation for E > 0 (no pair of real momenta
             shares a negative energy, so the curve is zero below 0).

    python -m paper_1412_1953_amd.xsec_curves OUT.json [E0 E1 dE [nstates]]
"""
from __future__ import annotations

import json
import math
import sys

FIG4 = (4.5, 1.0, 4.5, 1.0, 2.0, 1.0)


def curves(energies, nstates=2, n=512, L=25.6, R0=12.8, levels=6, M=2, tol=1e-10, log=print):
    import numpy as np
    from . import mgcccs
    g = mgcccs.Grid(n, L, R0, math.pi / 7, levels, M, pc_gamma=math.radians(10.0), pc_first_level=1,
                    max_restart=10, fp32=False, pot_tables=1)
    g.set_potential_exp(*FIG4)
    lam, _ = g.channel_energies()
    h = L / n
    j0 = int(round(R0 / h))
    x = h * np.arange(n + 1)
    th = math.pi / 7
    z = np.where(np.arange(n + 1) <= j0, x, R0 + (x - R0) * complex(math.cos(th), math.sin(th)))
    f = np.zeros((n + 1, n + 1), complex)
    f[1:n, 1:n] = np.exp(-3.0 * (z[1:n, None] + z[None, 1:n]) ** 2)
    ft = g.from_numpy(f)
    out = []
    for E in energies:
        g.set_energy(E)
        u = g.field()
        r = g.solve(u, ft, outer=mgcccs.FGMRES, restart=10, max_it=4000, tol=tol)
        row = {"E": E, "iters": r.iters, "relres": r.relres, "lambda": [l.real for l in lam]}
        opened = [q for q in range(nstates) if q < len(lam) and E > lam[q].real]
        if opened:
            s, kn = g.single_ionization(u, ft, len(opened))
            row["s2"] = [abs(v) ** 2 for v in s]
            row["k_n"] = kn
        row["sigma_tot"] = g.total_double_ionization(u, ft, nodes=32)[0] if E > 0 else 0.0
        log(json.dumps(row))
        out.append(row)
    return out


if __name__ == "__main__":
    if len(sys.argv) < 2:
        raise SystemExit(__doc__)
    a = sys.argv[2:]
    e0, e1, de = (float(a[0]), float(a[1]), float(a[2])) if len(a) >= 3 else (-1.0, 2.0, 0.1)
    ns = int(a[3]) if len(a) > 3 else 2
    m = int(round((e1 - e0) / de)) + 1
    res = curves([e0 + de * i for i in range(m)], nstates=ns, log=lambda s: print(s, flush=True))
    with open(sys.argv[1], "w") as fh:
        json.dump(res, fh, indent=1)
