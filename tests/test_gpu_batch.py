"""Batched solves (mgc_batch_*): many energies, grid sizes and channel counts,
one captured graph per solve and restart round, launched over concurrent
streams with one synchronisation per round.

Each batched solve follows the arithmetic of a single mgc_solve on its
handle, so its iterate must equal the individual solve's bit for bit.  The
64-solve workload (257^2 / 513^2 / 1025^2, E in [0.02, 3.0], 4..16 channels,
complex-FP32 cycle inside FP64 FGMRES) must meet 1e-10 for every solve, in the
oracle's own norm for one solve of each size.
"""
import math
import time

import numpy as np
import pytest

from helpers import Case, to_np
from oracle.grid import Grid1D, rel_residual, tp_operator, tp_rhs
from paper_1412_1953_amd.workloads import batch_workloads

pytestmark = pytest.mark.gpu
GAM = math.radians(5.0)

MIXED = [Case(32, 10.0, 0.3, 3, 2, pc_gamma=GAM, seed=21),
         Case(64, 20.0, 0.1, 4, 4, pc_gamma=GAM, seed=22),
         Case(64, 24.0, 0.7, 4, 5, pc_gamma=GAM, seed=23),
         Case(128, 40.0, 0.05, 5, 8, pc_gamma=GAM, seed=24),
         Case(128, 40.0, 0.9, 5, 3, pc_gamma=GAM, seed=25),
         Case(64, 20.0, 1.5, 4, 8, pc_gamma=GAM, seed=26)]


SIXTEEN = [Case(64 if i % 2 else 128, 20.0 if i % 2 else 40.0, 0.05 + 0.11 * i, 4 if i % 2 else 5,
                2 + (i % 7), pc_gamma=GAM, seed=100 + i) for i in range(16)]


def test_batch_of_16_runs_groups_concurrently():
    """16 solves (one graph per solve and round over the batch's streams):
    every iterate equals its individual solve; batch time against one by
    one.  The host bookkeeping of this batch runs clean under AddressSanitizer
    (tests/test_host_asan.py)."""
    import torch
    from paper_1412_1953_amd import mgcccs
    grids = [c.grid() for c in SIXTEEN]
    chis = [g.build_rhs_tp(g.field()) for g in grids]
    us = [g.from_numpy(c.u0()) for g, c in zip(grids, SIXTEEN)]
    batch = mgcccs.Batch(grids)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    res = batch.solve(us, chis, inner=mgcccs.FP32, restart=10, max_it=5000, tol=1e-10)
    t_batch = time.perf_counter() - t0
    t0 = time.perf_counter()
    single = []
    for g, c, chi in zip(grids, SIXTEEN, chis):
        ui = g.from_numpy(c.u0())
        single.append((ui, g.solve(ui, chi, outer=mgcccs.FGMRES, inner=mgcccs.FP32, restart=10,
                                   max_it=5000, tol=1e-10)))
    torch.cuda.synchronize()
    t_single = time.perf_counter() - t0
    for r, u, (ui, ri) in zip(res, us, single):
        assert r.status == mgcccs.MGC_OK and r.iters == ri.iters
        assert np.array_equal(to_np(u), to_np(ui))
    print(f"16 solves, {sum(r.iters for r in res)} iterations: batch {t_batch:.3f} s, "
          f"one by one {t_single:.3f} s")


@pytest.mark.parametrize("inner", ["fp64", "fp32"])
def test_batch_equals_individual_solves(inner):
    from paper_1412_1953_amd import mgcccs
    prec = mgcccs.FP32 if inner == "fp32" else mgcccs.FP64
    grids = [c.grid() for c in MIXED]
    chis = [g.build_rhs_tp(g.field()) for g in grids]
    us = [g.from_numpy(c.u0()) for g, c in zip(grids, MIXED)]
    batch = mgcccs.Batch(grids)
    res = batch.solve(us, chis, inner=prec, restart=10, max_it=5000, tol=1e-10)
    for g, c, chi, u, r in zip(grids, MIXED, chis, us, res):
        assert r.status == mgcccs.MGC_OK and r.relres <= 1e-10
        ui = g.from_numpy(c.u0())
        ri = g.solve(ui, chi, outer=mgcccs.FGMRES, inner=prec, restart=10, max_it=5000, tol=1e-10)
        assert ri.iters == r.iters
        assert ri.history == r.history
        assert np.array_equal(to_np(ui), to_np(u))


def test_batch_reports_each_status():
    """An iteration limit between the solves' needs: the batch returns
    ENOCONV, the solves past the limit keep their last iterate, the others
    converge with their own iteration counts."""
    from paper_1412_1953_amd import mgcccs
    cases = MIXED
    grids = [c.grid() for c in cases]
    chis = [g.build_rhs_tp(g.field()) for g in grids]
    need = []
    for g, c, chi in zip(grids, cases, chis):
        ui = g.from_numpy(c.u0())
        need.append(g.solve(ui, chi, outer=mgcccs.FGMRES, restart=10, max_it=5000, tol=1e-10).iters)
    limit = (min(need) + max(need)) // 2
    assert min(need) <= limit < max(need), need
    us = [g.from_numpy(c.u0()) for g, c in zip(grids, cases)]
    batch = mgcccs.Batch(grids)
    res = batch.solve(us, chis, inner=mgcccs.FP64, restart=10, max_it=limit, tol=1e-10)
    for r, k in zip(res, need):
        if k <= limit:
            assert r.status == mgcccs.MGC_OK and r.iters == k
        else:
            assert r.status == mgcccs.MGC_ENOCONV and r.iters == limit and r.relres > 1e-10


def test_batch_argument_errors():
    from paper_1412_1953_amd import mgcccs
    g = MIXED[0].grid()
    with pytest.raises(mgcccs.MGCError) as e:
        mgcccs.Batch([g, g])
    assert e.value.status == mgcccs.MGC_EINVAL
    b = mgcccs.Batch([g])
    u, f = g.field(), g.build_rhs_tp(g.field())
    with pytest.raises(mgcccs.MGCError) as e:
        b.solve([u], [f], restart=99)
    assert e.value.status == mgcccs.MGC_EINVAL


def test_batch_of_64_mixed_size_solves():
    """The 64-solve workload: every solve to 1e-10; one solve of each size
    checked by the oracle's operator; batch time against one-by-one solves.
    The host bookkeeping of this batch runs clean under AddressSanitizer
    (tests/test_host_asan.py)."""
    from paper_1412_1953_amd import autotune, mgcccs
    wls = batch_workloads()
    t0 = time.perf_counter()
    grids, chis, us = [], [], []
    for w in wls:
        g = autotune.tuned_grid(w, fp32_cycle=True, max_restart=10, fp32=True)
        grids.append(g)
        chis.append(g.build_rhs_tp(g.field()))
    t_setup = time.perf_counter() - t0
    from paper_1412_1953_amd.workloads import initial_guess
    us = [g.from_numpy(initial_guess(w.n, w.seed)) for g, w in zip(grids, wls)]
    batch = mgcccs.Batch(grids)
    import torch
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    res = batch.solve(us, chis, inner=mgcccs.FP32, restart=10, max_it=20000, tol=1e-10)
    t_batch = time.perf_counter() - t0
    unknowns = sum(w.unknowns for w in wls)
    for w, r in zip(wls, res):
        assert r.status == mgcccs.MGC_OK and r.relres <= 1e-10, (w.name, r.iters, r.relres)
    checked = set()
    for w, u in zip(wls, us):
        if w.n in checked:
            continue
        checked.add(w.n)
        go = Grid1D(w.n, w.L, w.R0, w.theta)
        rel = rel_residual(tp_operator(go, w.Z1, w.Z2, w.lam, w.E), to_np(u),
                           tp_rhs(go, w.Z1, w.Z2, w.lam, w.E))
        assert rel <= 1.001e-10, (w.name, rel)
    # the same solves one after another
    t0 = time.perf_counter()
    single = []
    for g, w, chi in zip(grids, wls, chis):
        ui = g.from_numpy(initial_guess(w.n, w.seed))
        single.append(g.solve(ui, chi, outer=mgcccs.FGMRES, inner=mgcccs.FP32, restart=10, max_it=20000,
                              tol=1e-10))
    torch.cuda.synchronize()
    t_single = time.perf_counter() - t0
    assert [r.iters for r in single] == [r.iters for r in res]
    print(f"64 solves, {unknowns} unknowns, {sum(r.iters for r in res)} iterations: setup {t_setup:.1f} s, "
          f"batch {t_batch:.2f} s ({unknowns / t_batch:.3e} solved unknowns/s), one by one "
          f"{t_single:.2f} s ({unknowns / t_single:.3e})")


def test_batch_of_mixed_sizes_against_one_by_one():
    """Twelve solves of the mixed-size workload (four each of 257^2, 513^2,
    1025^2; FP32 cycle in FP64 FGMRES): every solve to 1e-10 and bit-equal to
    its individual solve; batch wall time against the same solves one by one."""
    import torch
    from paper_1412_1953_amd import autotune, mgcccs
    from paper_1412_1953_amd.workloads import initial_guess
    wls = batch_workloads()
    pick = []
    for n in (256, 512, 1024):
        pick += [w for w in wls if w.n == n][:4]
    grids, chis = [], []
    for w in pick:
        g = autotune.tuned_grid(w, fp32_cycle=True, max_restart=10, fp32=True)
        grids.append(g)
        chis.append(g.build_rhs_tp(g.field()))
    us = [g.from_numpy(initial_guess(w.n, w.seed)) for g, w in zip(grids, pick)]
    batch = mgcccs.Batch(grids)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    res = batch.solve(us, chis, inner=mgcccs.FP32, restart=10, max_it=20000, tol=1e-10)
    t_batch = time.perf_counter() - t0
    for w, r in zip(pick, res):
        assert r.status == mgcccs.MGC_OK and r.relres <= 1e-10, (w.name, r.iters, r.relres)
    t0 = time.perf_counter()
    single = []
    for g, w, chi in zip(grids, pick, chis):
        ui = g.from_numpy(initial_guess(w.n, w.seed))
        single.append((ui, g.solve(ui, chi, outer=mgcccs.FGMRES, inner=mgcccs.FP32, restart=10,
                                   max_it=20000, tol=1e-10)))
    torch.cuda.synchronize()
    t_single = time.perf_counter() - t0
    for u, r, (ui, ri) in zip(us, res, single):
        assert r.iters == ri.iters
        assert np.array_equal(to_np(u), to_np(ui))
    unknowns = sum(w.unknowns for w in pick)
    print(f"12 solves, {unknowns} unknowns, iterations {[r.iters for r in res]}: batch {t_batch:.3f} s "
          f"({unknowns / t_batch:.3e} solved unknowns/s), one by one {t_single:.3f} s "
          f"({unknowns / t_single:.3e})")
