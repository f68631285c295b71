"""GPU parity of the split smoother: omega-Jacobi on the fine levels and the
GMRES(3) substitute of Sec. 6.1 from level gs_from on, against the oracle on
the same seeded inputs."""
import math

import numpy as np
import pytest
import scipy.sparse.linalg as spla

from helpers import Case, rel2, rel_err, to_np
from oracle.grid import tp_rhs

pytestmark = pytest.mark.gpu
GAM = math.radians(10.0)


def case(n, gs_from, **kw):
    base = dict(n=n, L=40.0 * n / 128, E=0.9, levels=int(math.log2(n)) - 2, M=6, pc_gamma=GAM,
                pc_first_level=1, pc_gamma0=math.radians(5.0), smoother=1, gs_from=gs_from)
    base.update(kw)
    return Case(**base)


CASES = [case(128, 1), case(128, 2), case(256, 2), case(256, 3)]
IDS = ["n128_gs1", "n128_gs2", "n256_gs2", "n256_gs3"]


@pytest.mark.parametrize("c", CASES, ids=IDS)
@pytest.mark.parametrize("fp32", [False, True], ids=["fp64", "fp32"])
def test_split_smoother_cycle(c, fp32):
    g = c.grid()
    o = c.oracle()
    chi = tp_rhs(o.g, c.Z1, c.Z2, c.lam, c.E)
    u = c.u0()
    ut, ft = g.from_numpy(u, fp32), g.from_numpy(chi, fp32)
    g.vcycle(ut, ft)
    assert rel_err(to_np(ut), o.mg.vcycle(u, chi)) < (5e-5 if fp32 else 1e-12)


@pytest.mark.parametrize("c", CASES, ids=IDS)
@pytest.mark.parametrize("fp32", [False, True], ids=["fp64", "fp32"])
def test_split_smoother_fgmres(c, fp32):
    """The first FGMRES(10) restart cycle against the oracle's iterate, then a
    converged solve against a sparse direct solve."""
    from paper_1412_1953_amd import mgcccs
    g = c.grid()
    o = c.oracle()
    chi = tp_rhs(o.g, c.Z1, c.Z2, c.lam, c.E)
    u = c.u0()
    inner = mgcccs.FP32 if fp32 else mgcccs.FP64
    ut, ft = g.from_numpy(u), g.from_numpy(chi)
    g.solve(ut, ft, outer=mgcccs.FGMRES, inner=inner, restart=10, max_it=10, tol=1e-300)
    ref = o.solve_fgmres(u, chi, 1e-300, restart=10, max_it=10)
    assert rel2(to_np(ut), ref.u) < (1e-4 if fp32 else 1e-10)
    ut = g.from_numpy(u)
    res = g.solve(ut, ft, outer=mgcccs.FGMRES, inner=inner, restart=10, max_it=2000, tol=1e-11)
    assert res.status == mgcccs.MGC_OK, res
    n = c.n
    x = spla.spsolve(o.op.sparse(), chi[1:n, 1:n].ravel()).reshape(n - 1, n - 1)
    assert rel2(to_np(ut)[1:n, 1:n], x) < 1e-9


@pytest.mark.parametrize("fp32", [False, True], ids=["fp64", "fp32"])
def test_split_smoother_schedules_agree_bitwise(fp32):
    """Level pairs and tile sizes never change the arithmetic: those
    schedules give the same iterate bit for bit, with the
    GMRES(3) levels in the single-workgroup tail and with per-level launches;
    the tail itself sums its reductions in another order, so tail and
    per-level launches agree to rounding."""
    from paper_1412_1953_amd import mgcccs
    c = case(256, 3)
    g = c.grid()
    chi = g.build_rhs_tp(g.field())
    out = {}
    for sch in ((-1, 1, 1), (0b11111, 0, 1), (0, 1, 1), (-1, 1, 0), (0, 0, 0), (0b11111, 1, 0)):
        g.set_schedule(*sch)
        u = g.from_numpy(c.u0())
        g.solve(u, chi, outer=mgcccs.FGMRES, inner=mgcccs.FP32 if fp32 else mgcccs.FP64, restart=10,
                max_it=12, tol=1e-300)
        out[sch] = to_np(u)
    tail = [v for k, v in out.items() if k[2] == 1]
    per_level = [v for k, v in out.items() if k[2] == 0]
    assert all(np.array_equal(tail[0], v) for v in tail[1:])
    assert all(np.array_equal(per_level[0], v) for v in per_level[1:])
    assert rel2(tail[0], per_level[0]) < (1e-5 if fp32 else 1e-12)


def test_gs_from_is_validated():
    from paper_1412_1953_amd import mgcccs
    with pytest.raises(mgcccs.MGCError) as e:
        case(128, 7).grid()
    assert e.value.status == mgcccs.MGC_EINVAL
