"""GPU parity of the channel correction embedded as a deflation step of the
Krylov preconditioner (the alternative of Sec. 7): z = e*(v) + V(v - A e*(v)),
against the oracle on the same seeded inputs, for FGMRES and BiCGSTAB."""
import math

import numpy as np
import pytest
import scipy.sparse.linalg as spla

from helpers import Case, rel2, to_np
from oracle.grid import rel_residual, tp_rhs

pytestmark = pytest.mark.gpu
GAM = math.radians(10.0)

CASES = [Case(64, 20.0, 0.3, 4, 4, pc_gamma=GAM, pc_order=1),
         Case(128, 40.0, 0.9, 5, 6, pc_gamma=math.radians(15.0), pc_first_level=1, pc_gamma0=math.radians(5.0),
              pc_order=1)]
IDS = ["n64", "n128"]


@pytest.mark.parametrize("c", CASES, ids=IDS)
@pytest.mark.parametrize("fp32", [False, True], ids=["fp64", "fp32"])
def test_deflated_fgmres_trajectory(c, fp32):
    """The first FGMRES(10) restart cycle from the same seed with the
    deflation-ordered preconditioner: same iterate as the oracle."""
    from paper_1412_1953_amd import mgcccs
    g = c.grid()
    o = c.oracle()
    chi = tp_rhs(o.g, c.Z1, c.Z2, c.lam, c.E)
    u = c.u0()
    ut, ft = g.from_numpy(u), g.from_numpy(chi)
    res = g.solve(ut, ft, outer=mgcccs.FGMRES, inner=mgcccs.FP32 if fp32 else mgcccs.FP64,
                  restart=10, max_it=10, tol=1e-300)
    ref = o.solve_fgmres(u, chi, 1e-300, restart=10, max_it=10)
    assert res.iters == 10
    err = rel2(to_np(ut), ref.u)
    assert err < (1e-4 if fp32 else 1e-10), err
    assert abs(res.relres - ref.relres) < (1e-3 if fp32 else 1e-8) * ref.relres


@pytest.mark.parametrize("c", CASES, ids=IDS)
def test_deflated_bicgstab_trajectory(c):
    from paper_1412_1953_amd import mgcccs
    g = c.grid()
    o = c.oracle()
    chi = tp_rhs(o.g, c.Z1, c.Z2, c.lam, c.E)
    u = c.u0()
    ut, ft = g.from_numpy(u), g.from_numpy(chi)
    res = g.solve(ut, ft, outer=mgcccs.BICGSTAB, inner=mgcccs.FP64, max_it=6, tol=1e-300)
    assert res.iters == 6
    ref = o.solve_bicgstab(u, chi, 1e-300, max_it=6)
    err = rel2(to_np(ut), ref.u)
    assert err < 1e-10, err


@pytest.mark.parametrize("c", CASES, ids=IDS)
@pytest.mark.parametrize("fp32", [False, True], ids=["fp64", "fp32"])
def test_deflated_solve_matches_direct_solve(c, fp32):
    from paper_1412_1953_amd import mgcccs
    g = c.grid()
    o = c.oracle()
    n = c.n
    chi = tp_rhs(o.g, c.Z1, c.Z2, c.lam, c.E)
    ut, ft = g.from_numpy(c.u0()), g.from_numpy(chi)
    res = g.solve(ut, ft, outer=mgcccs.FGMRES, inner=mgcccs.FP32 if fp32 else mgcccs.FP64, restart=10,
                  max_it=2000, tol=1e-11)
    assert res.status == mgcccs.MGC_OK and res.relres <= 1e-11, res
    x = spla.spsolve(o.op.sparse(), chi[1:n, 1:n].ravel()).reshape(n - 1, n - 1)
    assert rel2(to_np(ut)[1:n, 1:n], x) < 1e-9
    assert rel_residual(o.op, to_np(ut), chi) < 2e-11


@pytest.mark.parametrize("fp32", [False, True], ids=["fp64", "fp32"])
def test_deflated_preconditioner_is_exact_on_the_channel_space(fp32):
    """Without two-body coupling (lambda = 0) and with the exact operator on
    level 0, a source in the channel space is solved exactly by the
    correction: FGMRES with the deflation-ordered preconditioner stops after
    one iteration (to the cycle precision's rounding), while the V-cycle-first
    cycle needs several."""
    from paper_1412_1953_amd import mgcccs
    n = 64
    base = dict(Z2=0.9, lam=0.0, pc_gamma=math.radians(15.0), pc_first_level=1)
    cd = Case(n, 20.0, 0.3, 4, 4, pc_order=1, **base)
    cm = Case(n, 20.0, 0.3, 4, 4, pc_order=0, **base)
    o = cd.oracle()
    rng = np.random.default_rng(17)
    rA = np.zeros((n + 1, 4), complex)
    rB = np.zeros((n + 1, 4), complex)
    rA[1:n] = rng.standard_normal((n - 1, 4)) + 1j * rng.standard_normal((n - 1, 4))
    rB[1:n] = rng.standard_normal((n - 1, 4)) + 1j * rng.standard_normal((n - 1, 4))
    v = o.cc.expand(rA, rB)
    tol = 1e-5 if fp32 else 1e-10
    iters = []
    for c in (cd, cm):
        g = c.grid()
        ut, ft = g.field(), g.from_numpy(v)
        res = g.solve(ut, ft, outer=mgcccs.FGMRES, inner=mgcccs.FP32 if fp32 else mgcccs.FP64, restart=10,
                      max_it=400, tol=tol)
        assert res.status == mgcccs.MGC_OK, res
        iters.append(res.iters)
    assert iters[0] == 1 and iters[1] > 2, iters


def test_pc_order_is_validated():
    from paper_1412_1953_amd import mgcccs
    with pytest.raises(mgcccs.MGCError) as e:
        Case(64, 20.0, 0.3, 4, 4, pc_order=2).grid()
    assert e.value.status == mgcccs.MGC_EINVAL
