"""The C-ABI library loads on the CPU host and exports every entry point
declared in include/cutbddc.h (no compute calls: there is no GPU here)."""
import ctypes
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "cutbddc.h")
LIB = os.path.join(ROOT, "paper_1703_06323_amd", "libcutbddc.so")


def declared_symbols():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(cb_[a-z_]+)\s*\(", text)))


def test_header_declares_the_boundary():
    names = declared_symbols()
    for required in ("cb_setup", "cb_factor", "cb_solve", "cb_solve_rhs", "cb_grad",
                     "cb_query", "cb_destroy", "cb_last_error"):
        assert required in names


@pytest.mark.skipif(not os.path.exists(LIB), reason="library not built")
def test_library_exports_every_declared_symbol():
    lib = ctypes.CDLL(LIB)
    missing = [n for n in declared_symbols() if not hasattr(lib, n)]
    assert not missing, missing


@pytest.mark.skipif(not os.path.exists(LIB), reason="library not built")
def test_binding_signatures_load():
    from paper_1703_06323_amd import cutbddc
    lib = cutbddc.load_library()
    assert lib.cb_last_error() is not None
