"""The C-ABI library loads on a host without a GPU and exports every entry
point that include/mf.h declares; the Python binding covers exactly those."""
import ctypes
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "mf.h")
LIB = os.path.join(ROOT, "paper_2501_18781_amd", "libmf.so")


def declared_functions():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(mf_[a-z0-9_]+)\s*\(", text)))


def test_header_declares_the_boundary():
    names = declared_functions()
    for required in ["mf_operator_apply", "mf_operator_apply_transpose", "mf_cg_solve", "mf_gmres_solve",
                     "mf_mg_vcycle", "mf_heat_coeff_grad", "mf_create", "mf_destroy"]:
        assert required in names


def test_library_exports_every_declared_symbol():
    if not os.path.exists(LIB):
        pytest.fail("libmf.so is not built (run __graft_entry__.build())")
    L = ctypes.CDLL(LIB)
    missing = [n for n in declared_functions() if not hasattr(L, n)]
    assert not missing, missing


def test_binding_matches_header():
    from paper_2501_18781_amd import mf
    assert sorted(mf._SIGS) == declared_functions()


def test_struct_layouts_match_header():
    # offsets the C compiler gives the descriptor structs (natural alignment)
    from paper_2501_18781_amd import mf
    assert ctypes.sizeof(mf.MeshDesc) == 64
    assert mf.OperatorDesc.phi.offset == 16 + 13 * 8
    assert ctypes.sizeof(mf.OperatorDesc) == 16 + 13 * 8 + 4 * 8
    assert ctypes.sizeof(mf.SolveInfo) == 24
    assert mf.MGParams.lambda_max.offset == 32 and ctypes.sizeof(mf.MGParams) == 56
