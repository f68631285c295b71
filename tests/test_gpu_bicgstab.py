"""GPU parity of the MG-CCCS-preconditioned BiCGSTAB outer loop (Sec. 6.1,
Fig. convrate2D) and of the system on the full complex contour (Sec. 3.1),
against the oracle on the same seeded inputs."""
import math

import numpy as np
import pytest
import scipy.sparse.linalg as spla

from helpers import Case, rel2, to_np
from oracle.grid import rel_residual, tp_rhs

pytestmark = pytest.mark.gpu
GAM = math.radians(10.0)

CASES = [Case(64, 20.0, 0.3, 4, 4, pc_gamma=GAM), Case(128, 40.0, 0.9, 5, 6, pc_gamma=GAM, pc_first_level=1,
                                                       pc_gamma0=math.radians(5.0))]


@pytest.mark.parametrize("c", CASES, ids=["n64", "n128"])
@pytest.mark.parametrize("fp32", [False, True], ids=["fp64", "fp32"])
def test_bicgstab_trajectory(c, fp32):
    """Six BiCGSTAB iterations from the same seed: the oracle's iterate (FP64
    1e-10; the FP32 cycle's rounding stated against the FP64 oracle, 1e-4)
    and its recurred residual history."""
    from paper_1412_1953_amd import mgcccs
    g = c.grid()
    o = c.oracle()
    chi = tp_rhs(o.g, c.Z1, c.Z2, c.lam, c.E)
    u = c.u0()
    ut, ft = g.from_numpy(u), g.from_numpy(chi)
    res = g.solve(ut, ft, outer=mgcccs.BICGSTAB, inner=mgcccs.FP32 if fp32 else mgcccs.FP64, max_it=6, tol=1e-300)
    assert res.status == mgcccs.MGC_ENOCONV and res.iters == 6 and res.vcycles == 12
    ref = o.solve_bicgstab(u, chi, 1e-300, max_it=6)
    err = rel2(to_np(ut), ref.u)
    assert err < (1e-4 if fp32 else 1e-10), err
    h, hr = np.array(res.history), np.array(ref.history)
    assert np.all(np.abs(h - hr) <= (1e-3 if fp32 else 1e-8) * hr)


@pytest.mark.parametrize("c", CASES, ids=["n64", "n128"])
@pytest.mark.parametrize("fp32", [False, True], ids=["fp64", "fp32"])
def test_bicgstab_solution_matches_direct_solve(c, fp32):
    from paper_1412_1953_amd import mgcccs
    g = c.grid()
    o = c.oracle()
    n = c.n
    chi = tp_rhs(o.g, c.Z1, c.Z2, c.lam, c.E)
    ut, ft = g.from_numpy(c.u0()), g.from_numpy(chi)
    res = g.solve(ut, ft, outer=mgcccs.BICGSTAB, inner=mgcccs.FP32 if fp32 else mgcccs.FP64, max_it=2000, tol=1e-11)
    assert res.status == mgcccs.MGC_OK and res.relres <= 1e-11, res
    x = spla.spsolve(o.op.sparse(), chi[1:n, 1:n].ravel()).reshape(n - 1, n - 1)
    assert rel2(to_np(ut)[1:n, 1:n], x) < 1e-9
    assert rel_residual(o.op, to_np(ut), chi) < 2e-11


def test_bicgstab_needs_its_basis():
    from paper_1412_1953_amd import mgcccs
    c = CASES[0]
    g = c.grid(max_restart=4)
    u, f = g.field(), g.build_rhs_tp(g.field())
    with pytest.raises(mgcccs.MGCError) as e:
        g.solve(u, f, outer=mgcccs.BICGSTAB, max_it=5, tol=1e-8)
    assert e.value.status == mgcccs.MGC_EINVAL


def _contour_rhs(o, s=3.0):
    """f = exp(-s (z1 + z2)^2) on the contour nodes (the source of Table 1)."""
    z = o.g.z
    n = o.g.n
    f = np.zeros((n + 1, n + 1), complex)
    f[1:n, 1:n] = np.exp(-s * (z[1:n, None] + z[None, 1:n]) ** 2)
    return f


@pytest.mark.parametrize("fp32", [False, True], ids=["fp64", "fp32"])
def test_full_contour_system(fp32):
    """The system itself on the full complex contour (R0 = L, gamma = 10 deg,
    the hierarchy on the same contour): one V-cycle + CCCS against the oracle,
    and an FGMRES solve against a sparse direct solve of the rotated system."""
    from paper_1412_1953_amd import mgcccs
    c = Case(128, 20.0, 0.7, 5, 2, R0frac=1.0, gamma=GAM, pc_gamma=GAM, pc_gamma0=GAM, pc_first_level=0)
    g = c.grid()
    o = c.oracle()
    n = c.n
    f = _contour_rhs(o)
    u = c.u0()
    ut, ft = g.from_numpy(u, fp32), g.from_numpy(f, fp32)
    g.vcycle(ut, ft)
    ref = o.mg.vcycle(u, f)
    assert np.abs(to_np(ut) - ref).max() < (5e-5 if fp32 else 1e-12) * np.abs(ref).max()
    ut, ft = g.from_numpy(u), g.from_numpy(f)
    r = g.solve(ut, ft, outer=mgcccs.FGMRES, inner=mgcccs.FP32 if fp32 else mgcccs.FP64, restart=10, max_it=500,
                tol=1e-11)
    assert r.status == mgcccs.MGC_OK
    x = spla.spsolve(o.op.sparse(), f[1:n, 1:n].ravel()).reshape(n - 1, n - 1)
    assert rel2(to_np(ut)[1:n, 1:n], x) < 1e-9
    with pytest.raises(mgcccs.MGCError) as e:                  # amplitudes need a real interior
        g.cross_section(ut, ft, 0.5, 0.5)
    assert e.value.status == mgcccs.MGC_EINVAL


GS = [Case(64, 20.0, 0.6, 4, 3, pc_gamma=GAM, smoother=1), Case(128, 20.0, 1.2, 5, 2, R0frac=1.0, gamma=GAM,
                                                              pc_gamma=GAM, pc_gamma0=GAM, smoother=1)]


@pytest.mark.parametrize("c", GS, ids=["n64_ecs", "n128_contour"])
@pytest.mark.parametrize("fp32", [False, True], ids=["fp64", "fp32"])
def test_gmres3_smoothed_vcycle(c, fp32):
    """The V-cycle with the GMRES(3) smoothing substitute (Sec. 6.1) against
    the oracle's hierarchy with the same smoother: from a random guess (one
    smoothing step per level and pass, the Krylov space of each residual)."""
    g = c.grid()
    o = c.oracle()
    f = c.rand(2)
    u = c.u0()
    ut, ft = g.from_numpy(u, fp32), g.from_numpy(f, fp32)
    g.vcycle(ut, ft)
    ref = o.mg.vcycle(u, f)
    err = np.abs(to_np(ut) - ref).max() / np.abs(ref).max()
    assert err < (2e-4 if fp32 else 1e-11), err


@pytest.mark.parametrize("c", GS, ids=["n64_ecs", "n128_contour"])
@pytest.mark.parametrize("fp32", [False, True], ids=["fp64", "fp32"])
def test_gmres3_smoothed_fgmres_matches_direct_solve(c, fp32):
    from paper_1412_1953_amd import mgcccs
    g = c.grid()
    o = c.oracle()
    n = c.n
    f = c.rand(2)
    ut, ft = g.from_numpy(c.u0()), g.from_numpy(f)
    r = g.solve(ut, ft, outer=mgcccs.FGMRES, inner=mgcccs.FP32 if fp32 else mgcccs.FP64, restart=10, max_it=400,
                tol=1e-11)
    assert r.status == mgcccs.MGC_OK, r
    ref = o.solve_fgmres(c.u0(), f, 1e-11, restart=10, max_it=400)
    if not fp32:
        assert abs(r.iters - ref.iters) <= 1, (r.iters, ref.iters)
    x = spla.spsolve(o.op.sparse(), f[1:n, 1:n].ravel()).reshape(n - 1, n - 1)
    assert rel2(to_np(ut)[1:n, 1:n], x) < 1e-9
