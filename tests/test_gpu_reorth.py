"""The second Gram-Schmidt pass of the FGMRES Arnoldi step, forced in every
step (MGC_REORTH_ETA > 1): the launch that sweeps and then, in its last
block to finish, forms the Hessenberg column.  Against the default (second
pass only when needed), the oracle's FGMRES iterate, a direct solve, and
itself on a repeated solve (its block counter starts from zero each time)."""
import math

import numpy as np
import pytest
import scipy.sparse.linalg as spla

from helpers import Case, rel2, to_np
from oracle.grid import tp_rhs

pytestmark = pytest.mark.gpu
GAM = math.radians(10.0)
CASES = [Case(128, 40.0, 0.5, 5, 4, pc_gamma=GAM), Case(512, 80.0, 0.9, 6, 8, pc_gamma=GAM, pc_first_level=1)]


@pytest.mark.parametrize("c", CASES, ids=["n128", "n512"])
@pytest.mark.parametrize("fp32", [False, True], ids=["fp64", "fp32"])
def test_forced_second_pass(c, fp32, monkeypatch):
    from paper_1412_1953_amd import mgcccs
    inner = mgcccs.FP32 if fp32 else mgcccs.FP64
    o = c.oracle()
    chi = tp_rhs(o.g, c.Z1, c.Z2, c.lam, c.E)
    u0 = c.u0()
    outs = {}
    for eta in (None, "4"):
        if eta is None:
            monkeypatch.delenv("MGC_REORTH_ETA", raising=False)
        else:
            monkeypatch.setenv("MGC_REORTH_ETA", eta)
        g = c.grid()                       # a new handle: its restart graphs are captured with this setting
        ft = g.from_numpy(chi)
        runs = []
        for _ in range(2):
            ut = g.from_numpy(u0)
            r = g.solve(ut, ft, outer=mgcccs.FGMRES, inner=inner, restart=10, max_it=14, tol=1e-300)
            runs.append((to_np(ut), r.history))
        assert np.array_equal(runs[0][0], runs[1][0]) and runs[0][1] == runs[1][1]
        outs[eta] = runs[0][0]
    # (an FP32 cycle turns the second pass's rounding-level change of its
    # input into FP32-rounding-level changes of its output)
    assert rel2(outs["4"], outs[None]) < (1e-4 if fp32 else 1e-12)
    if c.n <= 128:
        ref = o.solve_fgmres(u0, chi, 1e-300, restart=10, max_it=14)
        assert rel2(outs["4"], ref.u) < (1e-4 if fp32 else 1e-10)


def test_forced_second_pass_solve_converges(monkeypatch):
    from paper_1412_1953_amd import mgcccs
    monkeypatch.setenv("MGC_REORTH_ETA", "4")
    c = CASES[0]
    g = c.grid()
    o = c.oracle()
    chi = tp_rhs(o.g, c.Z1, c.Z2, c.lam, c.E)
    ut, ft = g.from_numpy(c.u0()), g.from_numpy(chi)
    res = g.solve(ut, ft, outer=mgcccs.FGMRES, inner=mgcccs.FP64, restart=6, max_it=2000, tol=1e-11)
    assert res.status == mgcccs.MGC_OK
    n = c.n
    x = spla.spsolve(o.op.sparse(), chi[1:n, 1:n].ravel()).reshape(n - 1, n - 1)
    assert rel2(to_np(ut)[1:n, 1:n], x) < 1e-9
