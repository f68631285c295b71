"""GPU parity of the cross-section sweep (mgc_cross_section_sweep) against the
oracle's pair-by-pair amplitude: the energy-sharing sweeps of Sec. 3.3 over
many momentum pairs in one pass.  FP64 throughout; tolerance 1e-12 of the
largest amplitude of the sweep (a few hundred ulps of summation-order
difference over up to 767^2 terms)."""
import math

import numpy as np
import pytest

from helpers import Case
from oracle import functional as fn
from oracle.grid import Grid1D, tp_rhs

pytestmark = pytest.mark.gpu


def _fields(c, g, o):
    chi = tp_rhs(o.g, c.Z1, c.Z2, c.lam, c.E)
    u = c.u0()
    return u, chi, g.from_numpy(u), g.from_numpy(chi)


def _sweep_err(za, zb):
    za, zb = np.asarray(za), np.asarray(zb)
    return float(np.abs(za - zb).max() / np.abs(zb).max())


@pytest.mark.parametrize("npairs", [1, 41, 64, 65, 256])
def test_sweep_matches_oracle(npairs):
    c = Case(64, 20.0, 0.3, 4, 2)
    g, o = c.grid(), c.oracle()
    u, chi, ut, ct = _fields(c, g, o)
    from paper_1412_1953_amd import mgcccs
    alphas = np.linspace(0.02, math.pi / 2 - 0.02, npairs)
    k1s, k2s = mgcccs.sharing_momenta(c.E, alphas)
    zs, sig = g.cross_section_sweep(ut, ct, k1s, k2s)
    ref = fn.zeta_sweep(o.g, c.Z1, c.lam, u, chi, k1s, k2s)
    assert _sweep_err(zs, ref) < 1e-12
    sref = [fn.sigma(z, c.E, c.Z1, k1, k2) for z, k1, k2 in zip(ref, k1s, k2s)]
    assert float(np.abs(np.array(sig) - sref).max() / max(sref)) < 1e-11


def test_sweep_matches_oracle_on_the_129_grid():
    c = Case(128, 40.0, 0.1, 5, 4)
    g, o = c.grid(), c.oracle()
    u, chi, ut, ct = _fields(c, g, o)
    from paper_1412_1953_amd import mgcccs
    k1s, k2s = mgcccs.sharing_momenta(0.7, np.linspace(0.05, 1.5, 100))
    zs, _ = g.cross_section_sweep(ut, ct, k1s, k2s)
    ref = fn.zeta_sweep(o.g, c.Z1, c.lam, u, chi, k1s, k2s)
    assert _sweep_err(zs, ref) < 1e-12


def test_sweep_agrees_with_single_pair_calls():
    c = Case(128, 40.0, 0.1, 5, 4)
    g, o = c.grid(), c.oracle()
    _, _, ut, ct = _fields(c, g, o)
    k1s, k2s = [0.3, 0.55, 0.8], [0.9, 0.2, 0.8]
    zs, sig = g.cross_section_sweep(ut, ct, k1s, k2s)
    for z, s, k1, k2 in zip(zs, sig, k1s, k2s):
        z1, s1 = g.cross_section(ut, ct, k1, k2)
        assert abs(z - z1) < 1e-13 * abs(z1)
        assert abs(s - s1) < 1e-12 * s1


def test_sweep_full_size_sampled():
    """1025^2 (the timed grid), the maximal sweep of 256 pairs; eight of them
    checked against the oracle pair by pair."""
    c = Case(1024, 80.0, 0.5, 7, 8)
    g = c.grid(fp32=False)
    g1 = Grid1D(c.n, c.L, c.R0, c.theta)
    chi = tp_rhs(g1, c.Z1, c.Z2, c.lam, c.E)
    u = c.u0()
    ut, ct = g.from_numpy(u), g.from_numpy(chi)
    from paper_1412_1953_amd import mgcccs
    alphas = np.linspace(0.01, math.pi / 2 - 0.01, 256)
    k1s, k2s = mgcccs.sharing_momenta(c.E, alphas)
    zs, _ = g.cross_section_sweep(ut, ct, k1s, k2s)
    pick = [0, 37, 64, 100, 127, 128, 200, 255]
    ref = fn.zeta_sweep(g1, c.Z1, c.lam, u, chi, [k1s[a] for a in pick], [k2s[a] for a in pick])
    assert _sweep_err([zs[a] for a in pick], ref) < 1e-12


def test_sweep_rejects_bad_arguments():
    from paper_1412_1953_amd import mgcccs
    c = Case(32, 10.0, 0.3, 3, 2)
    g = c.grid()
    ut, ct = g.field(), g.field()
    with pytest.raises(mgcccs.MGCError) as e:
        g.cross_section_sweep(ut, ct, [], [])
    assert e.value.status == mgcccs.MGC_EINVAL
    with pytest.raises(mgcccs.MGCError) as e:
        g.cross_section_sweep(ut, ct, [0.5] * 257, [0.5] * 257)
    assert e.value.status == mgcccs.MGC_EINVAL
    with pytest.raises(mgcccs.MGCError) as e:
        g.cross_section_sweep(ut, ct, [0.5, -0.1], [0.5, 0.5])
    assert e.value.status == mgcccs.MGC_EINVAL


def test_sweep_device_test_functions_span_several_rounds():
    """2049^2 (1537 real-region nodes): the device test functions stage the
    potential term in more than one round; the sweep must agree with
    single-pair calls, whose test functions the host computes in the same
    operation order."""
    c = Case(2048, 160.0, 0.1, 8, 8)
    g = c.grid(fp32=False)
    from paper_1412_1953_amd import mgcccs
    u = c.u0()
    chi = c.rand()
    ut, ct = g.from_numpy(u), g.from_numpy(chi)
    alphas = np.linspace(0.05, math.pi / 2 - 0.05, 65)
    k1s, k2s = mgcccs.sharing_momenta(c.E, alphas)
    zs, sig = g.cross_section_sweep(ut, ct, k1s, k2s)
    for a in (0, 31, 64):
        z1, s1 = g.cross_section(ut, ct, k1s[a], k2s[a])
        assert abs(zs[a] - z1) < 1e-13 * abs(z1)
        assert abs(sig[a] - s1) < 1e-12 * s1
