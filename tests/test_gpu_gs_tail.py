"""The GMRES(3)-smoothed coarse tail (levels with n <= 64 and the coarsest
solve in one workgroup) against the per-level launches and the oracle."""
import math

import numpy as np
import pytest

from helpers import Case, rel2, rel_err, to_np
from oracle.grid import tp_rhs

pytestmark = pytest.mark.gpu
GAM = math.radians(10.0)

CASES = [Case(64, 20.0, 0.3, 4, 4, pc_gamma=GAM, smoother=1),                       # whole cycle in the tail
         Case(128, 40.0, 0.9, 5, 6, pc_gamma=GAM, pc_first_level=1, smoother=1, gs_from=1),   # 64, 32, 16 | 8
         Case(256, 80.0, 0.9, 6, 6, pc_gamma=GAM, pc_first_level=1, pc_gamma0=math.radians(5.0), smoother=1,
              gs_from=2),                                                             # 64, 32, 16 | 8
         Case(128, 40.0, 0.5, 4, 4, pc_gamma=GAM, smoother=1, gs_from=2)]              # 32 | 16
IDS = ["n64_all", "n128_gs1", "n256_gs2", "n128_gs2_c16"]


@pytest.mark.parametrize("c", CASES, ids=IDS)
@pytest.mark.parametrize("fp32", [False, True], ids=["fp64", "fp32"])
def test_gs_tail_cycle_matches_oracle_and_per_level_launches(c, fp32):
    """One preconditioner application through FGMRES (zero guess, scaled
    right-hand side) with the tail and with per-level launches: both match the
    oracle's FGMRES iterate; the two agree to rounding."""
    from paper_1412_1953_amd import mgcccs
    g = c.grid()
    o = c.oracle()
    chi = tp_rhs(o.g, c.Z1, c.Z2, c.lam, c.E)
    u = c.u0()
    inner = mgcccs.FP32 if fp32 else mgcccs.FP64
    ref = o.solve_fgmres(u, chi, 1e-300, restart=10, max_it=10)
    outs = []
    for tail in (1, 0):
        g.set_schedule(-1, 1, tail)
        ut, ft = g.from_numpy(u), g.from_numpy(chi)
        g.solve(ut, ft, outer=mgcccs.FGMRES, inner=inner, restart=10, max_it=10, tol=1e-300)
        outs.append(to_np(ut))
        assert rel2(outs[-1], ref.u) < (1e-4 if fp32 else 1e-10)
    assert rel2(outs[0], outs[1]) < (1e-5 if fp32 else 1e-12)


@pytest.mark.parametrize("fp32", [False, True], ids=["fp64", "fp32"])
def test_gs_tail_vcycle_from_a_nonzero_guess(fp32):
    """The V-cycle entry point (iterate given) through the tail."""
    c = Case(64, 20.0, 0.3, 4, 4, pc_gamma=GAM, smoother=1)
    g = c.grid()
    o = c.oracle()
    chi = tp_rhs(o.g, c.Z1, c.Z2, c.lam, c.E)
    u = c.u0()
    ut, ft = g.from_numpy(u, fp32), g.from_numpy(chi, fp32)
    g.vcycle(ut, ft)
    assert rel_err(to_np(ut), o.mg.vcycle(u, chi)) < (5e-5 if fp32 else 1e-12)


def test_gs_tail_solve_converges():
    from paper_1412_1953_amd import mgcccs
    import scipy.sparse.linalg as spla
    c = CASES[2]
    g = c.grid()
    o = c.oracle()
    chi = tp_rhs(o.g, c.Z1, c.Z2, c.lam, c.E)
    ut, ft = g.from_numpy(c.u0()), g.from_numpy(chi)
    res = g.solve(ut, ft, outer=mgcccs.FGMRES, inner=mgcccs.FP32, restart=10, max_it=1000, tol=1e-11)
    assert res.status == mgcccs.MGC_OK
    n = c.n
    x = spla.spsolve(o.op.sparse(), chi[1:n, 1:n].ravel()).reshape(n - 1, n - 1)
    assert rel2(to_np(ut)[1:n, 1:n], x) < 1e-9
