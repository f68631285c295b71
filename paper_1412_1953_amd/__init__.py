"""MI355X-native MG-CCCS solver for the 2D driven Schroedinger equation.

Cools & Vanroose, arXiv:1412.1953.  The solver is the HIP library
``libmgcccs.so`` (C ABI: ``include/mgcccs.h``); ``mgcccs`` is its Python
binding and ``workloads`` holds the seeded synthetic inputs.
"""
