"""GPU parity of the HIP MG-CCCS path against the FP64 CPU oracle.

Every test calls the C ABI through the thin binding and compares element by
element with the oracle on the same seeded inputs.  Tolerances: FP64 kernels
1e-12 relative (max-norm over the field) -- a few hundred ulps of rounding-order
difference; FP32 kernels 2e-5; converged solves 1e-10 relative solution error
against the oracle's direct solve.
"""
import math

import numpy as np
import pytest
import scipy.sparse.linalg as spla

from helpers import Case, rel2, rel_err, to_np
from oracle.grid import rel_residual, tp_rhs

pytestmark = pytest.mark.gpu

GAM = math.radians(5.0)

SMALL = [
    Case(32, 10.0, 0.3, 3, 2),
    Case(64, 20.0, 0.1, 4, 4, pc_gamma=GAM),
    Case(128, 40.0, 0.1, 5, 4),          # the 129^2 workload grid
]


@pytest.mark.parametrize("c", SMALL, ids=lambda c: f"n{c.n}")
def test_rhs(c):
    g = c.grid()
    chi = to_np(g.build_rhs_tp(g.field()))
    o = c.oracle()
    ref = tp_rhs(o.g, c.Z1, c.Z2, c.lam, c.E)
    assert rel_err(chi, ref) < 1e-14


@pytest.mark.parametrize("c", SMALL, ids=lambda c: f"n{c.n}")
@pytest.mark.parametrize("fp32", [False, True], ids=["fp64", "fp32"])
def test_residual(c, fp32):
    g = c.grid()
    u, f = c.rand(1), c.rand(2)
    ut, ft, rt = g.from_numpy(u, fp32), g.from_numpy(f, fp32), g.field(fp32)
    rel = g.residual(ut, ft, rt)
    o = c.oracle()
    ref = o.op.residual(u.astype(np.complex64).astype(complex) if fp32 else u,
                        f.astype(np.complex64).astype(complex) if fp32 else f)
    tol = 2e-5 if fp32 else 1e-13
    assert rel_err(to_np(rt), ref) < tol
    assert abs(rel - np.linalg.norm(ref) / np.linalg.norm(f)) < 1e-5 * rel


@pytest.mark.parametrize("c", SMALL + [Case(64, 20.0, 0.5, 4, 4, pc_gamma=GAM, pc_first_level=1)],
                         ids=lambda c: f"n{c.n}_g{c.pc_gamma:.2f}_f{c.pc_first_level}")
@pytest.mark.parametrize("fp32", [False, True], ids=["fp64", "fp32"])
def test_vcycle(c, fp32):
    g = c.grid()
    o = c.oracle()
    chi = tp_rhs(o.g, c.Z1, c.Z2, c.lam, c.E)
    u = c.u0()
    ut, ft = g.from_numpy(u, fp32), g.from_numpy(chi, fp32)
    g.vcycle(ut, ft)
    ref = o.mg.vcycle(u, chi)
    assert rel_err(to_np(ut), ref) < (5e-5 if fp32 else 1e-12)


@pytest.mark.parametrize("c", SMALL + [Case(64, 20.0, 0.5, 4, 1), Case(64, 20.0, -0.3, 4, 16),
                                       Case(64, 24.0, 0.7, 4, 5, pc_gamma=GAM)],
                         ids=lambda c: f"n{c.n}_M{c.M}_g{c.pc_gamma:.2f}")
@pytest.mark.parametrize("fp32", [False, True], ids=["fp64", "fp32"])
def test_cccs(c, fp32):
    g = c.grid()
    o = c.oracle()
    chi = tp_rhs(o.g, c.Z1, c.Z2, c.lam, c.E)
    u = c.u0()
    ut, ft = g.from_numpy(u, fp32), g.from_numpy(chi, fp32)
    g.cccs(ut, ft)
    ref = o.cc.step(u, chi)
    # compare the correction (u* - u), the part the step computes
    corr = to_np(ut) - (u.astype(np.complex64).astype(complex) if fp32 else u)
    assert rel_err(corr, ref - u) < (1e-4 if fp32 else 1e-10)


def test_cccs_long_interface():
    """513^2 with 16 channels: 32 chunks per channel system, so each interface
    row holds 992 entries and a lane loads its row in more than one round.
    FP64 only: the indexing is shared by both precisions, and the FP32 cycle's
    accuracy at full size is checked through the converged mixed solves."""
    c = Case(512, 40.0, 0.2, 6, 16)
    g = c.grid()
    o = c.oracle()
    chi = tp_rhs(o.g, c.Z1, c.Z2, c.lam, c.E)
    u = c.u0()
    ut, ft = g.from_numpy(u, False), g.from_numpy(chi, False)
    g.cccs(ut, ft)
    ref = o.cc.step(u, chi)
    assert rel_err(to_np(ut) - u, ref - u) < 1e-10


@pytest.mark.parametrize("c", [Case(64, 20.0, -0.4, 4, 4), Case(128, 40.0, 0.1, 5, 4)],
                         ids=lambda c: f"n{c.n}_E{c.E}")
def test_stationary_trajectory(c):
    """K cycles of stationary MG-CCCS from the same seed (exact operator on
    every level): identical iterates up to rounding, whether or not the
    iteration contracts for this energy."""
    from paper_1412_1953_amd import mgcccs
    K = 3
    g = c.grid()
    o = c.oracle()
    chi = tp_rhs(o.g, c.Z1, c.Z2, c.lam, c.E)
    u = c.u0()
    ut, ft = g.from_numpy(u), g.from_numpy(chi)
    res = g.solve(ut, ft, outer=mgcccs.STATIONARY, max_it=K, tol=1e-300)
    assert res.iters == K and res.status == mgcccs.MGC_ENOCONV
    ref = u
    for _ in range(K):
        ref = o.cycle(ref, chi)
    assert rel2(to_np(ut), ref) < 1e-10
    hist_o = [rel_residual(o.op, u, chi)]
    assert abs(res.history[0] - hist_o[0]) < 1e-12 * hist_o[0]


@pytest.mark.parametrize("c", [Case(64, 20.0, 0.3, 4, 4, pc_gamma=GAM),
                               Case(128, 40.0, 0.1, 5, 8, pc_gamma=GAM)],
                         ids=lambda c: f"n{c.n}")
@pytest.mark.parametrize("fp32", [False, True], ids=["fp64", "fp32"])
def test_fgmres_trajectory(c, fp32):
    """The first FGMRES(10) restart cycle from the same seed: same iterate."""
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


@pytest.mark.parametrize("c", [Case(64, 20.0, 0.3, 4, 4, pc_gamma=GAM),
                               Case(128, 40.0, 0.1, 5, 8, pc_gamma=GAM, seed=0)],
                         ids=lambda c: f"n{c.n}")
@pytest.mark.parametrize("fp32", [False, True], ids=["fp64", "fp32"])
def test_fgmres_solution_matches_direct_solve(c, fp32):
    from paper_1412_1953_amd import mgcccs
    g = c.grid()
    o = c.oracle()
    n = c.n
    chi = tp_rhs(o.g, c.Z1, c.Z2, c.lam, c.E)
    ut, ft = g.from_numpy(c.u0()), g.from_numpy(chi)
    res = g.solve(ut, ft, outer=mgcccs.FGMRES, inner=mgcccs.FP32 if fp32 else mgcccs.FP64,
                  restart=10, max_it=2000, tol=1e-12)
    assert res.status == mgcccs.MGC_OK, res
    assert res.relres <= 1e-12
    x = spla.spsolve(o.op.sparse(), chi[1:n, 1:n].ravel()).reshape(n - 1, n - 1)
    err = rel2(to_np(ut)[1:n, 1:n], x)
    assert err < 1e-10, err
    # the oracle's own residual of the GPU solution
    assert rel_residual(o.op, to_np(ut), chi) < 2e-12


# Iterative refinement (MGC_IR): grids on which the stationary cycle contracts
IR_CASES = [Case(32, 10.0, 0.3, 3, 3), Case(64, 16.0, -0.2, 4, 4)]


@pytest.mark.parametrize("c", IR_CASES, ids=lambda c: f"n{c.n}")
@pytest.mark.parametrize("fp32", [False, True], ids=["fp64", "fp32"])
def test_ir_trajectory(c, fp32):
    """Four refinement steps of two MG-CCCS cycles each from the same seed:
    the oracle's refinement iterate (FP64 inner cycles) to 1e-10 in FP64; with
    complex-FP32 inner cycles the corrections carry FP32 rounding, stated
    against the FP64 oracle (1e-5)."""
    from paper_1412_1953_amd import mgcccs
    g = c.grid()
    o = c.oracle()
    chi = tp_rhs(o.g, c.Z1, c.Z2, c.lam, c.E)
    u = c.u0()
    ut, ft = g.from_numpy(u), g.from_numpy(chi)
    res = g.solve(ut, ft, outer=mgcccs.IR, inner=mgcccs.FP32 if fp32 else mgcccs.FP64,
                  max_it=4, inner_cycles=2, tol=1e-300)
    assert res.status == mgcccs.MGC_ENOCONV and res.iters == 4 and res.vcycles == 8
    ref = o.solve_ir(u, chi, 0.0, inner_cycles=2, max_it=4)
    err = rel2(to_np(ut), ref.u)
    assert err < (1e-5 if fp32 else 1e-10), err
    hist = np.array(res.history)
    assert np.all(np.abs(hist - np.array(ref.history)) <= (1e-3 if fp32 else 1e-8) * np.array(ref.history))


@pytest.mark.parametrize("c", IR_CASES, ids=lambda c: f"n{c.n}")
@pytest.mark.parametrize("fp32", [False, True], ids=["fp64", "fp32"])
def test_ir_solution_matches_direct_solve(c, fp32):
    """Refinement to 1e-12 with FP64 or complex-FP32 inner cycles reaches the
    sparse direct solution (the FP64 outer residual removes the FP32 error)."""
    from paper_1412_1953_amd import mgcccs
    g = c.grid()
    o = c.oracle()
    n = c.n
    chi = tp_rhs(o.g, c.Z1, c.Z2, c.lam, c.E)
    ut, ft = g.from_numpy(c.u0()), g.from_numpy(chi)
    res = g.solve(ut, ft, outer=mgcccs.IR, inner=mgcccs.FP32 if fp32 else mgcccs.FP64,
                  max_it=200, inner_cycles=2, tol=1e-12)
    assert res.status == mgcccs.MGC_OK and res.relres <= 1e-12, res
    x = spla.spsolve(o.op.sparse(), chi[1:n, 1:n].ravel()).reshape(n - 1, n - 1)
    assert rel2(to_np(ut)[1:n, 1:n], x) < 1e-10
    assert rel_residual(o.op, to_np(ut), chi) < 2e-12


def test_small_workload_129_as_specified():
    """The 129^2 workload exactly as specified (domain [0,40]^2, ECS beyond 30
    at pi/6, E = 0.1, 5 levels, 4 channels, seed 0, tol 1e-8), FGMRES(10) with
    the FP64 MG-CCCS cycle of the workload's preconditioning hierarchy: the
    oracle's FGMRES reaches the tolerance after the
    same number of iterations, the two iterates agree to 1e-10, and both are
    the sparse direct solution to within the conditioning times 1e-8."""
    from paper_1412_1953_amd import mgcccs
    from paper_1412_1953_amd.workloads import SMALL_129 as w
    from paper_1412_1953_amd import autotune
    c = Case(w.n, w.L, w.E, w.levels, w.M, seed=w.seed, **autotune.hierarchy_of(w))
    g = c.grid()
    o = c.oracle()
    n = c.n
    chi = tp_rhs(o.g, c.Z1, c.Z2, c.lam, c.E)
    u = c.u0()
    ut, ft = g.from_numpy(u), g.from_numpy(chi)
    res = g.solve(ut, ft, outer=mgcccs.FGMRES, restart=10, max_it=2000, tol=w.tol)
    assert res.status == mgcccs.MGC_OK and res.relres <= w.tol, res
    ref = o.solve_fgmres(u, chi, w.tol, restart=10, max_it=2000)
    assert ref.relres <= w.tol and ref.iters == res.iters, (ref.iters, res.iters)
    err = rel2(to_np(ut), ref.u)
    assert err < 1e-10, err
    x = spla.splu(o.op.sparse()).solve(chi[1:n, 1:n].ravel()).reshape(n - 1, n - 1)
    print(f"129^2 workload: {res.iters} iterations, relres {res.relres:.3e}, GPU vs oracle {err:.2e}, "
          f"GPU vs direct {rel2(to_np(ut)[1:n, 1:n], x):.2e}")
    assert rel2(to_np(ut)[1:n, 1:n], x) < 1e-5


def test_coarsest_only_grid_is_a_direct_solve():
    c = Case(8, 4.0, 0.2, 1, 1)
    g = c.grid()
    o = c.oracle()
    chi = tp_rhs(o.g, c.Z1, c.Z2, c.lam, c.E)
    ut, ft = g.from_numpy(c.u0()), g.from_numpy(chi)
    g.vcycle(ut, ft)
    assert rel_residual(o.op, to_np(ut), chi) < 1e-13


def test_solves_are_bitwise_reproducible():
    from paper_1412_1953_amd import mgcccs
    c = Case(64, 20.0, 0.3, 4, 4, pc_gamma=GAM)
    g = c.grid()
    o = c.oracle()
    chi = tp_rhs(o.g, c.Z1, c.Z2, c.lam, c.E)
    outs = []
    for _ in range(2):
        ut, ft = g.from_numpy(c.u0()), g.from_numpy(chi)
        g.solve(ut, ft, outer=mgcccs.FGMRES, restart=10, max_it=25, tol=1e-300)
        outs.append(to_np(ut))
    assert np.array_equal(outs[0], outs[1])


def test_error_paths():
    from paper_1412_1953_amd import mgcccs
    with pytest.raises(mgcccs.MGCError) as e:
        mgcccs.Grid(48, 10.0, 7.5, math.pi / 6, 3, 2)          # n not a power of two
    assert e.value.status == mgcccs.MGC_EINVAL
    with pytest.raises(mgcccs.MGCError) as e:
        mgcccs.Grid(64, 10.0, 7.0, math.pi / 6, 3, 2)          # R0 off the coarse grid
    assert e.value.status == mgcccs.MGC_EINVAL
    g = mgcccs.Grid(32, 10.0, 7.5, math.pi / 6, 3, 2)
    u, f = g.field(), g.field()
    with pytest.raises(mgcccs.MGCError) as e:
        g.vcycle(u, f)                                          # no set_energy yet
    assert e.value.status == mgcccs.MGC_ESTATE
    g.set_potential(1.0, 1.0, 1.0)
    g.set_energy(0.3)
    g.build_rhs_tp(f)
    res = g.solve(u, f, outer=mgcccs.FGMRES, restart=5, max_it=1, tol=1e-12)
    assert res.status == mgcccs.MGC_ENOCONV and res.iters == 1
    assert res.relres < res.history[0]                        # a truncated cycle still helps
    g.set_energy(-0.6)                                          # below the 1s threshold
    with pytest.raises(mgcccs.MGCError) as e:
        g.build_rhs_tp(f)
    assert e.value.status == mgcccs.MGC_EINVAL
    g.set_energy(0.3)
    with pytest.raises(mgcccs.MGCError) as e:
        g.solve(u, f, outer=mgcccs.STATIONARY, max_it=3, tol=1e-8, inner=mgcccs.FP32)
    assert e.value.status == mgcccs.MGC_EINVAL


def test_binding_rejects_fields_the_kernels_would_overrun():
    """Every field is checked before the call: a contiguous (n+1, n+1) tensor
    (the kernels use a row pitch of round16(n+1)), the wrong dtype for the
    call's precision, a mismatched second field, another shape, a view that
    does not reach the end of the buffer."""
    import torch
    from paper_1412_1953_amd import mgcccs
    c = Case(32, 10.0, 0.3, 3, 2)
    g = c.grid()
    n = c.n
    good = g.field()
    chi = g.build_rhs_tp(g.field())
    bad = [torch.zeros((n + 1, n + 1), dtype=torch.complex128, device=g.device),
           g.field(fp32=True),
           g.field()[:n, :n],
           torch.zeros(((n + 1) * g.pitch,), dtype=torch.complex128, device=g.device)[1:].as_strided(
               (n + 1, n + 1), (g.pitch, 1))]
    for b in bad:
        for call in (lambda: g.vcycle(good, b) if b.dtype == good.dtype else g.cross_section(b, chi, 0.5, 0.5),
                     lambda: g.solve(b, chi, max_it=1),
                     lambda: g.cross_section(good, b, 0.5, 0.5)):
            with pytest.raises(mgcccs.MGCError) as e:
                call()
            assert e.value.status == mgcccs.MGC_EINVAL
    with pytest.raises(mgcccs.MGCError) as e:                   # FP32 u with an FP64 f
        g.residual(g.field(fp32=True), chi, g.field(fp32=True))
    assert e.value.status == mgcccs.MGC_EINVAL
    with pytest.raises(mgcccs.MGCError) as e:
        g.vcycle(good, chi.cpu())
    assert e.value.status == mgcccs.MGC_EINVAL


def test_graph_replays_match_eager_launches(monkeypatch):
    """The FGMRES restart cycle runs as a captured hipGraph; several replays
    (with host work and synchronisation between them) must give exactly the
    iterate of the eagerly launched kernels."""
    from paper_1412_1953_amd import mgcccs
    c = Case(64, 20.0, 0.3, 4, 4, pc_gamma=GAM)
    g = c.grid()
    o = c.oracle()
    chi = tp_rhs(o.g, c.Z1, c.Z2, c.lam, c.E)
    outs = {}
    for mode in ("eager", "graph"):
        if mode == "eager":
            monkeypatch.setenv("MGC_NO_GRAPH", "1")
        else:
            monkeypatch.delenv("MGC_NO_GRAPH", raising=False)
        ut, ft = g.from_numpy(c.u0()), g.from_numpy(chi)
        g.solve(ut, ft, outer=mgcccs.FGMRES, restart=10, max_it=40, tol=1e-300)
        outs[mode] = to_np(ut)
    assert np.array_equal(outs["eager"], outs["graph"])


@pytest.mark.parametrize("c", [Case(128, 40.0, 0.3, 5, 4, pc_gamma=GAM),       # pair 128/64, tail 32
                               Case(512, 40.0, 0.2, 7, 8, pc_gamma=GAM),       # pairs 512/256, 128/64
                               Case(256, 20.0, 1.1, 4, 6, pc_gamma=GAM)],      # pair 256/128, tail 32
                         ids=["n128", "n512", "n256"])
@pytest.mark.parametrize("fp32", [False, True], ids=["fp64", "fp32"])
def test_fused_level_passes_match_per_level_launches(c, fp32):
    """Every launch schedule computes, node by node, the same arithmetic: the
    paired-level launches, the coarse tail, one S1 / S2 launch per level with
    a separate coarsest solve, and large or small tiles on any level give the
    same iterate bit for bit over twelve FGMRES steps."""
    from paper_1412_1953_amd import mgcccs
    from oracle.grid import Grid1D
    chi = tp_rhs(Grid1D(c.n, c.L, c.R0, c.theta), c.Z1, c.Z2, c.lam, c.E)
    inner = mgcccs.FP32 if fp32 else mgcccs.FP64
    schedules = [(-1, 1, 1), (-1, 0, 0), (-1, 1, 0), (-1, 0, 1), (0, 1, 1), (-1 & 0x7fffffff, 1, 1), (1, 0, 1),
                 (0b10, 1, 1)]
    outs = []
    g = c.grid()
    for sch in schedules:
        g.set_schedule(*sch)
        assert g.get_schedule() == sch
        ut, ft = g.from_numpy(c.u0()), g.from_numpy(chi)
        r = g.solve(ut, ft, outer=mgcccs.FGMRES, inner=inner, restart=10, max_it=12, tol=1e-300)
        outs.append((to_np(ut), r.history))
    for o in outs[1:]:
        assert o[1] == outs[0][1]
        assert np.array_equal(o[0], outs[0][0])
    with pytest.raises(mgcccs.MGCError) as e:
        g.set_schedule(-2, 1, 1)
    assert e.value.status == mgcccs.MGC_EINVAL
    with pytest.raises(mgcccs.MGCError) as e:
        g.set_schedule(-1, 2, 1)
    assert e.value.status == mgcccs.MGC_EINVAL


@pytest.mark.parametrize("fp32", [False, True], ids=["fp64", "fp32"])
def test_level0_contour_angle(fp32):
    """A hierarchy with level 0 on one contour angle and the coarser levels on
    another: the V-cycle and the CCCS of the library against the oracle's
    hierarchy with the same angles."""
    c = Case(64, 20.0, 0.7, 4, 6, pc_gamma=math.radians(15.0), pc_first_level=1, pc_gamma0=math.radians(10.0))
    g = c.grid()
    o = c.oracle()
    chi = tp_rhs(o.g, c.Z1, c.Z2, c.lam, c.E)
    u = c.u0()
    ut, ft = g.from_numpy(u, fp32), g.from_numpy(chi, fp32)
    g.vcycle(ut, ft)
    ref = o.mg.vcycle(u, chi)
    assert rel_err(to_np(ut), ref) < (5e-5 if fp32 else 1e-12)
    ut = g.from_numpy(u, fp32)
    g.cccs(ut, ft)
    ref = o.cc.step(u, chi)
    corr = to_np(ut) - (u.astype(np.complex64).astype(complex) if fp32 else u)
    assert rel_err(corr, ref - u) < (1e-4 if fp32 else 1e-10)


@pytest.mark.parametrize("graph", [True, False], ids=["graph", "eager"])
@pytest.mark.parametrize("kclass", [1, 2, 3, 4, 5, 6, 7, 8, 9],
                         ids=["apply", "axpy", "s1", "s2", "project", "chain", "s1fine", "s2fine", "expand"])
def test_kernel_timer_counts_launches_and_leaves_results_unchanged(kclass, graph, monkeypatch):
    """Event timing of one kernel class in every fourth restart cycle (the
    first included): launches counted per Arnoldi step (operator pass, first
    axpy pass) or per timed restart cycle (S1/S2: one per level above the
    coarse tail plus the tail launch; CCCS projection/chain 1), the
    algorithmic byte count of each class (FP64 inner cycle), and a
    bitwise-identical iterate."""
    from paper_1412_1953_amd import mgcccs
    if graph:
        monkeypatch.delenv("MGC_NO_GRAPH", raising=False)
    else:
        monkeypatch.setenv("MGC_NO_GRAPH", "1")
    c = Case(64, 20.0, 0.3, 4, 4, pc_gamma=GAM)
    g = c.grid()
    o = c.oracle()
    chi = tp_rhs(o.g, c.Z1, c.Z2, c.lam, c.E)
    its = 43                                   # restart cycles of 10, 10, 10, 10, 3 steps
    u_ref, f = g.from_numpy(c.u0()), g.from_numpy(chi)
    g.solve(u_ref, f, outer=mgcccs.FGMRES, restart=10, max_it=its, tol=1e-300)
    g.set_kernel_timer(kclass)
    u = g.from_numpy(c.u0())
    r = g.solve(u, f, outer=mgcccs.FGMRES, restart=10, max_it=its, tol=1e-300)
    ms, launches, nbytes, floor = g.read_kernel_timer()
    g.set_kernel_timer(mgcccs.KT_NONE)
    assert r.iters == its
    assert np.array_equal(to_np(u), to_np(u_ref))
    # cycles 0 and 4 are timed (10 and 3 steps); classes that do not depend
    # on the Arnoldi step are timed in the first step of a timed cycle
    timed = [10, 3]
    cycles = len(timed)
    # n = 64: level 64 by the fused passes, levels 32 and 16 in the coarse
    # tail (one launch down, one up)
    want_launches = {mgcccs.KT_APPLY_DOT: sum(timed), mgcccs.KT_AXPY: sum(timed),
                     mgcccs.KT_S1: 2 * cycles, mgcccs.KT_S2: 2 * cycles}.get(kclass, cycles)
    assert launches == want_launches
    assert ms > 0 and floor > 0
    n, N = c.n, (c.n - 1) ** 2
    steps = [j for cyc in timed for j in range(cyc)]
    if kclass == mgcccs.KT_APPLY_DOT:
        want = sum(N * (16 + 16 * (j + 1) + 16) for j in steps)
    elif kclass == mgcccs.KT_AXPY:
        want = sum(N * (16 * (j + 1) + 32) for j in steps)
    elif kclass in (mgcccs.KT_S1, mgcccs.KT_S2):
        # every level above the coarsest (4 levels: 64, 32, 16 | 8 coarsest)
        fine = [(m - 1) ** 2 for m in (64, 32, 16)]
        coarse = [(m // 2 - 1) ** 2 for m in (64, 32, 16)]
        k = 1 if kclass == mgcccs.KT_S1 else 2
        want = cycles * sum(k * a + b for a, b in zip(fine, coarse)) * 16
        if kclass == mgcccs.KT_S1:
            # the down launch also reads the coarsest inverse and writes u_c
            Nc = (8 - 1) ** 2
            want += cycles * (Nc * Nc + Nc) * 16
    elif kclass in (mgcccs.KT_CCCS_PROJECT, mgcccs.KT_CCCS_EXPAND):
        want = cycles * (2 * N + (n - 1) * (c.M + c.M)) * 16
    elif kclass in (mgcccs.KT_S1_FINE, mgcccs.KT_S2_FINE):
        # level 64 alone: f in, f_c out (S1); f, e_c in, u out (S2)
        k = 1 if kclass == mgcccs.KT_S1_FINE else 2
        want = cycles * (k * N + (n // 2 - 1) ** 2) * 16
    else:
        want = cycles * 2 * (2 * c.M ** 2 + 4 * c.M) * (n - 1) * 16
    assert nbytes == pytest.approx(want, rel=1e-12)
    assert g.read_kernel_timer() == (0.0, 0, 0.0, 0.0)
