"""The C-ABI library loads on the CPU host and exports every declared symbol.

No compute call is made (there is no GPU here); the GPU tests exercise them.
"""
import ctypes
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "crk.h")


def declared_functions():
    src = open(HEADER).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    names = re.findall(r"\b(crk_[a-z0-9_]+)\s*\(", src)
    return sorted(set(names))


def test_header_declares_the_entry_points():
    names = declared_functions()
    for n in ("crk_create_lattice", "crk_load_gauge", "crk_mg_setup", "crk_mg_solve", "crk_dirac_apply"):
        assert n in names


def test_library_exports_every_declared_symbol():
    import paper_2502_03091_amd as crk
    if not os.path.exists(crk.LIB_PATH):
        pytest.fail("libcrk.so is not built: run __graft_entry__.build()")
    lib = ctypes.CDLL(crk.LIB_PATH)
    missing = [n for n in declared_functions() if not hasattr(lib, n)]
    assert not missing, f"not exported: {missing}"
    assert set(crk.exported_symbols()) <= set(declared_functions())
    crk.lib()  # binding signatures resolve


def test_version_and_error_string_without_gpu():
    import paper_2502_03091_amd as crk
    lib = crk.lib()
    assert lib.crk_version() >= 10000
    assert isinstance(lib.crk_last_error(), bytes)
