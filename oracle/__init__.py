"""Plain FP64 CPU oracle of the MG-CCCS solver (Cools & Vanroose, arXiv:1412.1953).

TEST INFRASTRUCTURE ONLY.  Nothing in the product path imports this package:
only ``tests/``, ``__graft_entry__.smoke()`` and the ``cpu_baseline`` leg of
``bench.py`` may use it.  It shares no code with the HIP library; the only
common module is ``paper_1412_1953_amd.workloads`` (seeded inputs, no method
arithmetic).

Everything is complex128 and written for readability, not speed: numpy slicing
for the stencil, SciPy's dense/banded LAPACK routines for the direct solves and
the 1D eigenproblem.

Modules
-------
grid        finite-difference grid with exterior complex scaling, operator, rhs
mg          omega-Jacobi, full weighting, bilinear interpolation, V-cycle
cccs        1D bound states, channel potentials, Coupled Channel Correction Step
solvers     stationary MG-CCCS, FGMRES(m), mixed-precision iterative refinement
functional  ionisation amplitude zeta(k1,k2), cross section, adjoint gradient

Parity pins: every function is checked in ``tests/test_oracle_*.py`` against
values the paper prints, closed forms, brute-force direct solves or invariants.
Functions without such a pin say "parity unpinned" in their docstring.
"""
