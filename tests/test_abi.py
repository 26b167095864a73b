"""The C-ABI library loads on the CPU host and exports every call gap.h declares.

No compute call is made here (there is no GPU in this check).
"""
import ctypes
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "gap.h")
LIB = os.path.join(ROOT, "paper_2310_03921_amd", "libgap.so")


def declared_symbols():
    text = open(HEADER).read()
    return sorted(set(re.findall(r"^\s*(?:gap_status|const char \*|int)\s*(gap_\w+)\s*\(", text, re.M)))


def test_header_declares_the_verbs():
    names = declared_symbols()
    for verb in ("gap_create", "gap_build_kmm", "gap_build_knm", "gap_fit", "gap_predict",
                 "gap_predict_backward", "gap_forces", "gap_pair_transpose", "gap_lstsq"):
        assert verb in names


@pytest.mark.skipif(not os.path.exists(LIB), reason="libgap.so not built (run __graft_entry__.build())")
def test_library_exports_every_declared_symbol():
    lib = ctypes.CDLL(LIB)
    missing = [n for n in declared_symbols() if not hasattr(lib, n)]
    assert not missing, missing


def test_binding_structs_match_header_layout():
    import paper_2310_03921_amd as g
    # gap_atoms: 4 int64, 2 pointers, enum (+pad), int64, 3 pointers, enum (+pad), int64
    assert ctypes.sizeof(g.gap_atoms) == 4 * 8 + 2 * 8 + 8 + 8 + 3 * 8 + 8 + 8
    assert ctypes.sizeof(g.gap_sparse) == 3 * 8 + 8 + 8 + 8
    assert ctypes.sizeof(g.gap_fit_info) == 8 * 8 + 8 + 8 + 8
