"""The C-ABI library loads on a host without a GPU and exports every declared entry point."""
import ctypes
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
LIB = os.path.join(ROOT, "paper_2501_12497_amd", "libmmof.so")


def declared_functions():
    names = set()
    inc = os.path.join(ROOT, "include")
    for f in os.listdir(inc):
        if f.endswith(".h"):
            text = open(os.path.join(inc, f)).read()
            text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
            names |= set(re.findall(r"\b(mmof_[A-Za-z_0-9]+)\s*\(", text))
    return sorted(names)


def test_header_declares_the_boundary_calls():
    names = declared_functions()
    for required in ("mmof_apply_A", "mmof_apply_At", "mmof_apply_grad", "mmof_apply_flow_op",
                     "mmof_flow_update", "mmof_solve_joint"):
        assert required in names


def test_library_exports_every_declared_symbol():
    if not os.path.exists(LIB):
        pytest.fail("libmmof.so is not built (run __graft_entry__.build())")
    lib = ctypes.CDLL(LIB)
    missing = [n for n in declared_functions() if not hasattr(lib, n)]
    assert not missing, missing


def test_binding_signatures_cover_the_header():
    from paper_2501_12497_amd import _lib
    assert set(_lib._SIGS) == set(declared_functions())


def test_version_without_gpu():
    from paper_2501_12497_amd import _lib
    lib = _lib.load()
    assert lib.mmof_version().decode().startswith("mmof-gfx950")
