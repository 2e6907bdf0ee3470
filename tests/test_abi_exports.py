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


def test_solve_joint_rejects_wrong_u0_dtype_before_any_launch():
    """u_inout is read and written as n FP64 values: a float32 u0 must be refused in the
    binding (it would be an out-of-bounds device write), before any GPU work."""
    import torch
    from paper_2501_12497_amd import binding as B

    class _Plan:
        n, m = 16, 8

    b = torch.zeros(8, dtype=torch.float64)
    with pytest.raises(TypeError, match="u0 must be float64"):
        B.solve_joint(_Plan(), b, 0.1, u0=torch.zeros(16, dtype=torch.float32))
    with pytest.raises(TypeError, match="b must be float64"):
        B.solve_joint(_Plan(), b.float(), 0.1)
    with pytest.raises(TypeError, match="u_true must be float64"):
        B.solve_joint(_Plan(), b, 0.1, u_true=torch.zeros(16, dtype=torch.float32))
