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


def test_struct_layouts_match_header(tmp_path):
    # every ctypes mirror has the size and field offsets the C compiler gives
    # the header's struct of the same name
    import shutil
    import subprocess
    from paper_2501_18781_amd import mf
    cc = shutil.which("gcc") or shutil.which("cc")
    if cc is None:
        pytest.skip("no C compiler")
    pairs = [("mf_mesh", mf.MeshDesc), ("mf_operator", mf.OperatorDesc), ("mf_solve_info", mf.SolveInfo),
             ("mf_mg_params", mf.MGParams), ("mf_heat_sources", mf.SourcesDesc), ("mf_picard_info", mf.PicardInfo), ("mf_transport_params", mf.TransportDesc)]
    lines = ["#include <stdio.h>", "#include <stddef.h>", '#include "mf.h"', "int main(void) {"]
    expect = []
    for cname, py in pairs:
        lines.append(f'printf("%zu\\n", sizeof({cname}));')
        expect.append(ctypes.sizeof(py))
        for fname, _ in py._fields_:
            lines.append(f'printf("%zu\\n", offsetof({cname}, {fname}));')
            expect.append(getattr(py, fname).offset)
    lines += ["return 0; }"]
    src = tmp_path / "layout.c"
    src.write_text("\n".join(lines) + "\n")
    exe = tmp_path / "layout"
    subprocess.run([cc, "-std=c11", "-I", os.path.join(ROOT, "include"), str(src), "-o", str(exe)], check=True)
    got = [int(v) for v in subprocess.run([str(exe)], check=True, capture_output=True, text=True).stdout.split()]
    assert got == expect


def test_mesh_validation_happens_on_the_host():
    # mf_create rejects an invalid mesh before it touches a device: no cells,
    # an empty box, unknown face bits, or a mesh whose 3 n_nodes reaches 2^31
    # (the largest cube accepted is 446^3 cells; 447^3 is refused)
    from paper_2501_18781_amd import mf
    L = mf.library()

    def create(n, hi=(1.0, 1.0, 1.0), dirichlet=0):
        d = mf.MeshDesc()
        for k in range(3):
            d.n[k], d.lo[k], d.hi[k] = n[k], 0.0, hi[k]
        d.dirichlet = dirichlet
        h = ctypes.c_void_p()
        st = L.mf_create(ctypes.byref(d), ctypes.byref(h))
        assert not h.value
        return st

    err = -1  # MF_ERR_ARG
    assert create((0, 4, 4)) == err
    assert create((4, -3, 4)) == err
    assert create((4, 4, 4), hi=(1.0, 0.0, 1.0)) == err
    assert create((4, 4, 4), dirichlet=64) == err
    assert create((447, 447, 447)) == err
    assert 3 * 895 ** 3 >= 2 ** 31 > 3 * 893 ** 3
    assert L.mf_create(None, ctypes.byref(ctypes.c_void_p())) == err
