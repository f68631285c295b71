"""GPU parity of the single-ionisation amplitudes s_n(E), the total
double-ionisation cross section sigma_tot(E) (Sec. 3.3) and their batched form
over the energies of a batch, against the oracle on the same seeded fields.
The functionals are linear in (u, chi), so any field serves; the full-size
case uses the converged 1025^2 solution.  Tolerance: 1e-12 of the largest
amplitude (summation order over up to 767^2 terms differs)."""
import math

import numpy as np
import pytest

from helpers import Case, to_np
from oracle import functional as fn
from oracle.grid import tp_rhs

pytestmark = pytest.mark.gpu


def _fields(c, scale=0.1):
    g = c.grid()
    o = c.oracle()
    chi = tp_rhs(o.g, c.Z1, c.Z2, c.lam, c.E)
    u = c.rand(3) * scale
    return g, o, chi, u


@pytest.mark.parametrize("c,nst", [(Case(64, 20.0, 0.6, 4, 2), 4), (Case(128, 40.0, 0.3, 5, 4, Z2=1.3, lam=0.8), 6),
                                   (Case(128, 40.0, -0.05, 5, 4), 3)], ids=["n64", "n128_Z2", "n128_negE"])
def test_single_ionization_matches_oracle(c, nst):
    g, o, chi, u = _fields(c)
    s, kn = g.single_ionization(g.from_numpy(u), g.from_numpy(chi), nst)
    lamB, ks, ref = fn.single_ionization(o.g, c.Z1, c.Z2, c.lam, c.E, u, chi, nst)
    assert np.allclose(kn, ks, rtol=1e-12, atol=0)
    err = np.abs(np.array(s) - ref).max() / np.abs(ref).max()
    assert err < 1e-12, err


@pytest.mark.parametrize("c,nodes", [(Case(64, 20.0, 0.6, 4, 2), 16), (Case(128, 40.0, 1.3, 5, 4), 32),
                                     (Case(128, 40.0, 0.2, 5, 4, Z1=1.2, lam=0.7), 64)],
                         ids=["n64", "n128", "n128_Z1"])
def test_total_double_ionization_matches_oracle(c, nodes):
    g, o, chi, u = _fields(c)
    sig, zs = g.total_double_ionization(g.from_numpy(u), g.from_numpy(chi), nodes)
    ref = fn.sigma_total(o.g, c.Z1, c.lam, c.E, u, chi, nodes)
    assert abs(sig - ref) < 1e-11 * ref, (sig, ref)
    x, _ = np.polynomial.legendre.leggauss(nodes)
    a = (x + 1) * math.pi / 4
    K = math.sqrt(2 * c.E)
    zref = np.array(fn.zeta_sweep(o.g, c.Z1, c.lam, u, chi, K * np.sin(a), K * np.cos(a)))
    assert np.abs(np.array(zs) - zref).max() < 1e-12 * np.abs(zref).max()


def test_batch_cross_sections_equal_single_handle_calls():
    """Four energies (four handles) in one batched call: the same bits as the
    per-handle calls."""
    from paper_1412_1953_amd import mgcccs
    cases = [Case(64, 20.0, E, 4, 3, seed=40 + i) for i, E in enumerate((0.2, 0.7, 1.1, 2.3))]
    gs, us, chis, single = [], [], [], []
    for c in cases:
        g, o, chi, u = _fields(c)
        ut, ct = g.from_numpy(u), g.from_numpy(chi)
        gs.append(g)
        us.append(ut)
        chis.append(ct)
        single.append((g.total_double_ionization(ut, ct, 24)[0], g.single_ionization(ut, ct, 3)[0]))
    b = mgcccs.Batch(gs)
    sigs, ss = b.cross_sections(us, chis, nodes=24, nstates=3)
    for (s1, si1), s2, si2 in zip(single, sigs, ss):
        assert s1 == s2
        assert si1 == si2


def test_cross_section_argument_errors():
    from paper_1412_1953_amd import mgcccs
    c = Case(64, 20.0, -0.2, 4, 2)
    g, o, chi, u = _fields(c)
    ut, ct = g.from_numpy(u), g.from_numpy(chi)
    with pytest.raises(mgcccs.MGCError) as e:
        g.total_double_ionization(ut, ct, 16)            # E <= 0: no double ionisation
    assert e.value.status == mgcccs.MGC_EINVAL
    with pytest.raises(mgcccs.MGCError) as e:
        g.single_ionization(ut, ct, 3)                   # E = -0.2 is below the n = 2 threshold
    assert e.value.status == mgcccs.MGC_EINVAL
    s, _ = g.single_ionization(ut, ct, 1)                # the 1s channel is open
    assert abs(s[0]) > 0
    with pytest.raises(mgcccs.MGCError) as e:
        g.single_ionization(ut, ct, 17)
    assert e.value.status == mgcccs.MGC_EINVAL


def test_total_cross_section_full_size():
    """The 1025^2 workload at E = 0.5 solved to 1e-10: sigma_tot and s_n
    (8 states) against the oracle on the library's solution."""
    from paper_1412_1953_amd import autotune, mgcccs
    from paper_1412_1953_amd.workloads import TP1025
    w = TP1025[0.5]
    c = Case(w.n, w.L, w.E, w.levels, w.M, seed=w.seed, **autotune.hierarchy_of(w))
    g = c.grid()
    chi_t = g.build_rhs_tp(g.field())
    u = g.from_numpy(c.u0())
    r = g.solve(u, chi_t, outer=mgcccs.FGMRES, restart=10, max_it=5000, tol=w.tol)
    assert r.status == mgcccs.MGC_OK
    sig, _ = g.total_double_ionization(u, chi_t, 32)
    s, _ = g.single_ionization(u, chi_t, 8)
    o = c.oracle()
    un, chin = to_np(u), to_np(chi_t)
    ref = fn.sigma_total(o.g, c.Z1, c.lam, c.E, un, chin, 32)
    _, _, sref = fn.single_ionization(o.g, c.Z1, c.Z2, c.lam, c.E, un, chin, 8)
    print(f"1025^2 E=0.5: sigma_tot {sig:.10e} (oracle {ref:.10e}); |s_n| {np.abs(s)}")
    assert abs(sig - ref) < 1e-11 * ref
    assert np.abs(np.array(s) - sref).max() < 1e-11 * np.abs(sref).max()
