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
    # 8 doubles + 10 int32 with natural alignment (see include/fagbi.h)
    assert ctypes.sizeof(_lib.Params) == 112
    p = F.default_params()
    assert p.eps_out == 80.0 and p.p_leaf == 4 and p.quad_duffy == 7
