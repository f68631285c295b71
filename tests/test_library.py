"""CPU checks of the C-ABI library: it builds for gfx950, loads, and exports
every function that include/mgcccs.h declares.  No compute call is made."""
import ctypes
import os
import re
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "mgcccs.h")


def declared_functions():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(mgc_[a-z_]+)\s*\(", text)))


@pytest.fixture(scope="module")
def libpath():
    from paper_1412_1953_amd import build_lib
    if not os.path.exists(build_lib.OUT):
        build_lib.build()
    return build_lib.OUT


def test_header_declares_the_boundary():
    names = declared_functions()
    for required in ["mgc_create_grid", "mgc_set_potential", "mgc_set_energy", "mgc_vcycle",
                     "mgc_cccs", "mgc_solve", "mgc_cross_section"]:
        assert required in names


def test_library_exports_every_declared_symbol(libpath):
    out = subprocess.run(["nm", "-D", "--defined-only", libpath], capture_output=True, text=True,
                         check=True).stdout
    exported = set(re.findall(r"\bT (mgc_[a-z_]+)\b", out))
    missing = [f for f in declared_functions() if f not in exported]
    assert not missing, missing


def test_library_loads_and_binding_matches_header(libpath):
    lib = ctypes.CDLL(libpath)
    for f in declared_functions():
        assert hasattr(lib, f)
    from paper_1412_1953_amd import mgcccs
    assert sorted(mgcccs.EXPORTED) == declared_functions()


def test_gfx950_code_object_present(libpath):
    data = open(libpath, "rb").read()
    assert b"gfx950" in data
