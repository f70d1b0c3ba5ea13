"""The C-ABI library loads and exports every entry point the header declares
(no GPU needed; no compute calls)."""
import os
import re

import paper_2110_13778_amd as F
from paper_2110_13778_amd import _lib

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def declared():
    src = open(os.path.join(ROOT, "include", "fagbi.h")).read()
    return sorted(set(re.findall(r"\b(fagbi_[a-z_0-9]+)\s*\(", src)))


def test_header_and_binding_agree():
    assert declared() == sorted(_lib.EXPORTS)


def test_library_exports_every_declared_symbol():
    lib = F.load()
    for name in declared():
        assert hasattr(lib, name), name


def test_params_struct_size_matches_header_layout():
    import ctypes
    # 8 doubles + 11 int32 with natural alignment (see include/fagbi.h): the
    # last int32 (basis) at 128, padded to 136
    assert ctypes.sizeof(_lib.Params) == 136
    p = F.default_params()
    assert p.eps_out == 80.0 and p.p_leaf == 4 and p.quad_duffy == 7


def test_struct_layouts_match_c_compiler(tmp_path):
    """every field offset and struct size of the ctypes mirrors equals what a
    C compiler gives for include/fagbi.h"""
    import ctypes
    import shutil
    import subprocess
    import pytest
    if shutil.which("gcc") is None:
        pytest.skip("no C compiler")
    structs = {"fagbi_params": _lib.Params, "fagbi_tree_info": _lib.TreeInfo,
               "fagbi_solve_info": _lib.SolveInfo, "fagbi_profile": _lib.Profile}
    lines = ["#include <stdio.h>", "#include <stddef.h>", '#include "fagbi.h"', "int main(void) {"]
    for cname, py in structs.items():
        lines.append('printf("%s %%zu\\n", sizeof(%s));' % (cname, cname))
        for fname, _ in py._fields_:
            lines.append('printf("%s.%s %%zu\\n", offsetof(%s, %s));' % (cname, fname, cname, fname))
    lines += ["return 0;", "}"]
    src = tmp_path / "layout.c"
    src.write_text("\n".join(lines) + "\n")
    exe = tmp_path / "layout"
    subprocess.run(["gcc", "-std=c99", "-I", os.path.join(ROOT, "include"), str(src), "-o", str(exe)], check=True)
    out = dict(l.split() for l in subprocess.run([str(exe)], check=True, capture_output=True,
                                                 text=True).stdout.splitlines())
    for cname, py in structs.items():
        assert int(out[cname]) == ctypes.sizeof(py), cname
        for fname, _ in py._fields_:
            assert int(out[cname + "." + fname]) == getattr(py, fname).offset, (cname, fname)
