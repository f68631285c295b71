"""The CCCS entry point that allocates nothing (mgc_cccs_noalloc) against
mgc_cccs, whose scratch lives in the handle's workspace: two calls in a row
on one GPU, the second on a smaller grid (the static scratch keeps the first
call's contents), FP64 and FP32, results equal bit for bit; a grid whose
scratch exceeds the static array is refused."""
import numpy as np
import pytest

from helpers import Case, to_np
from oracle.grid import tp_rhs

pytestmark = pytest.mark.gpu


@pytest.mark.parametrize("fp32", [False, True], ids=["fp64", "fp32"])
def test_noalloc_cccs_matches_workspace_cccs_on_two_calls(fp32):
    for c in (Case(512, 40.0, 0.2, 6, 16, seed=31), Case(128, 40.0, 0.7, 5, 5, seed=32)):
        print(f"[noalloc] n={c.n} M={c.M} fp32={fp32}", flush=True)
        g = c.grid()
        o = c.oracle()
        chi = tp_rhs(o.g, c.Z1, c.Z2, c.lam, c.E)
        u0 = c.u0()
        f = g.from_numpy(chi, fp32)
        ua, ub = g.from_numpy(u0, fp32), g.from_numpy(u0, fp32)
        g.cccs(ua, f)
        g.cccs_noalloc(ub, f)
        a, b = to_np(ua), to_np(ub)
        assert np.array_equal(a, b), np.abs(a - b).max()
        assert np.abs(a - u0.astype(np.complex64 if fp32 else np.complex128)).max() > 0


def test_noalloc_cccs_refuses_a_scratch_beyond_the_static_array():
    from paper_1412_1953_amd import mgcccs
    c = Case(2048, 160.0, 0.1, 8, 16)
    g = c.grid(max_restart=0, fp32=False)
    u, f = g.field(), g.build_rhs_tp(g.field())
    with pytest.raises(mgcccs.MGCError) as e:
        g.cccs_noalloc(u, f)
    assert e.value.status == mgcccs.MGC_EINVAL
    g.cccs(u, f)                                  # the workspace variant still runs
