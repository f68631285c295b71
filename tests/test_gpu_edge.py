"""Edge cases of the path on the GPU: no channels at all (M = L = 0, plain
multigrid: the channel correction is the identity) and a grid near the
largest the library takes (8193^2 nodes, every field 1.07 GB)."""
import math

import numpy as np
import pytest
import scipy.sparse.linalg as spla

from helpers import Case, rel2, rel_err, to_np
from oracle.grid import Grid1D, tp_operator, tp_rhs

pytestmark = pytest.mark.gpu
GAM = math.radians(10.0)


@pytest.mark.parametrize("fp32", [False, True], ids=["fp64", "fp32"])
def test_zero_channels(fp32):
    from paper_1412_1953_amd import mgcccs
    c = Case(128, 40.0, 0.4, 5, 0, pc_gamma=GAM, pc_first_level=1)
    g = c.grid()
    o = c.oracle()
    chi = tp_rhs(o.g, c.Z1, c.Z2, c.lam, c.E)
    u = c.u0()
    # the channel correction leaves u as it is
    ut, ft = g.from_numpy(u, fp32), g.from_numpy(chi, fp32)
    before = to_np(ut).copy()
    g.cccs(ut, ft)
    assert np.array_equal(to_np(ut), before)
    # the cycle is the V-cycle alone
    g.vcycle(ut, ft)
    assert rel_err(to_np(ut), o.mg.vcycle(u, chi)) < (5e-5 if fp32 else 1e-12)
    inner = mgcccs.FP32 if fp32 else mgcccs.FP64
    ut, ft = g.from_numpy(u), g.from_numpy(chi)
    g.solve(ut, ft, outer=mgcccs.FGMRES, inner=inner, restart=10, max_it=10, tol=1e-300)
    ref = o.solve_fgmres(u, chi, 1e-300, restart=10, max_it=10)
    assert rel2(to_np(ut), ref.u) < (1e-4 if fp32 else 1e-10)
    ut = g.from_numpy(u)
    res = g.solve(ut, ft, outer=mgcccs.FGMRES, inner=inner, restart=10, max_it=3000, tol=1e-11)
    assert res.status == mgcccs.MGC_OK
    n = c.n
    x = spla.spsolve(o.op.sparse(), chi[1:n, 1:n].ravel()).reshape(n - 1, n - 1)
    assert rel2(to_np(ut)[1:n, 1:n], x) < 1e-9


def test_near_largest_grid():
    """n = 8192 (the library takes n <= 16384): the residual against the
    oracle's operator over the whole field, then FGMRES(6) steps with the
    complex-FP32 cycle that reduce the true residual in every restart cycle."""
    from paper_1412_1953_amd import mgcccs
    n, L, E = 8192, 640.0, 0.5
    R0, theta = 0.75 * L, math.pi / 6
    print(f"[maxsize] n={n} grid", flush=True)
    g = mgcccs.Grid(n, L, R0, theta, 10, 4, pc_gamma=GAM, pc_first_level=1, max_restart=6, fp32=True)
    g.set_potential(1.0, 1.0, 1.0)
    g.set_energy(E)
    rng = np.random.default_rng(17)
    u = np.zeros((n + 1, n + 1), complex)
    f = np.zeros((n + 1, n + 1), complex)
    u[1:n, 1:n] = rng.standard_normal((n - 1, n - 1)) + 1j * rng.standard_normal((n - 1, n - 1))
    f[1:n, 1:n] = rng.standard_normal((n - 1, n - 1)) + 1j * rng.standard_normal((n - 1, n - 1))
    print("[maxsize] residual", flush=True)
    ut, ft, rt = g.from_numpy(u), g.from_numpy(f), g.field()
    g.residual(ut, ft, rt)
    r = to_np(rt)
    del ut, rt
    ref = tp_operator(Grid1D(n, L, R0, theta), 1.0, 1.0, 1.0, E).residual(u, f)
    assert rel_err(r, ref) < 1e-13
    del r, ref, u, f, ft
    print("[maxsize] solve", flush=True)
    chi = g.build_rhs_tp(g.field())
    ut = g.field()
    res = g.solve(ut, chi, outer=mgcccs.FGMRES, inner=mgcccs.FP32, restart=6, max_it=24, tol=1e-300)
    h = res.history
    assert len(h) == 5 and all(b < a for a, b in zip(h, h[1:])), h
    assert h[-1] < 0.5 * h[0], h
