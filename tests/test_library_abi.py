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


def _setup_status(problem):
    """cb_setup's status for a problem that argument validation must reject
    before any device work (so it runs without a GPU)."""
    from paper_1703_06323_amd import cutbddc
    lib = cutbddc.load_library()
    p, keep = cutbddc._problem_struct(problem)
    ctx = ctypes.c_void_p()
    rc = lib.cb_setup(ctypes.byref(p), None, ctypes.byref(ctx))
    return rc, lib.cb_last_error().decode(), ctx


@pytest.mark.skipif(not os.path.exists(LIB), reason="library not built")
@pytest.mark.parametrize("s", [24, 32])
def test_setup_rejects_blocks_too_large_for_lds(s):
    """Subdomain blocks whose cell tables and one assembly row exceed the
    160 KB of LDS of a workgroup are an argument error at setup, not a
    launch failure inside factor or solve (blocks up to 16 cells per side
    take the large-subdomain kernels)."""
    import workloads as W
    from paper_1703_06323_amd import cutbddc
    rc, msg, ctx = _setup_status(W.uncut(2 * s, s))
    assert rc == cutbddc.CB_ERR_ARG and "LDS" in msg, (rc, msg)
    assert not ctx.value


@pytest.mark.skipif(not os.path.exists(LIB), reason="library not built")
def test_setup_argument_errors():
    import numpy as np

    import workloads as W
    from paper_1703_06323_amd import cutbddc
    assert _setup_status(W.uncut(10, 4))[0] == cutbddc.CB_ERR_ARG                 # s does not divide N
    assert _setup_status(W.uncut(8, 4).with_options(weighting=3))[0] == cutbddc.CB_ERR_ARG
    assert _setup_status(W.uncut(8, 4).with_options(coarse_variant=7))[0] == cutbddc.CB_ERR_ARG
    assert _setup_status(W.uncut(8, 4).with_options(cut_boundary=2))[0] == cutbddc.CB_ERR_ARG
    bad = W.Problem(n=8, s=4, centres=np.array([[0.5, 0.5, 0.5]]), radii=np.array([-0.1]))
    assert _setup_status(bad)[0] == cutbddc.CB_ERR_ARG


@pytest.mark.skipif(not os.path.exists(LIB), reason="library not built")
def test_null_context_errors():
    from paper_1703_06323_amd import cutbddc
    lib = cutbddc.load_library()
    assert lib.cb_factor(None) == cutbddc.CB_ERR_ARG
    assert lib.cb_query(None, None) == cutbddc.CB_ERR_ARG
    x0 = (ctypes.c_double * 3)(0.0, 0.0, 0.0)
    assert lib.cb_manufactured_load(None, x0, 1.0, None) == cutbddc.CB_ERR_ARG
    assert lib.cb_manufactured_errors(None, x0, 1.0, None, None, None) == cutbddc.CB_ERR_ARG
    n = ctypes.c_int32(0)
    assert lib.cb_pcg_history(None, 0, 0, None, None, None, ctypes.byref(n), None, None) == cutbddc.CB_ERR_ARG
    assert lib.cb_lanczos_extremes(-1, None, None, None, None) == cutbddc.CB_ERR_ARG
