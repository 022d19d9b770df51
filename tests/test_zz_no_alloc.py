"""The allocation-free batched SPD inverse (cb_dense_spd_inverse_noalloc)
against the allocating entry point (cb_dense_spd_inverse), both through the
C ABI, in FP64 and FP32: two calls in a row on the shared scratch array, the
second with a smaller input, then the error paths (a request beyond the
scratch size, a matrix that is not positive definite)."""
import ctypes as C

import numpy as np
import pytest

pytestmark = pytest.mark.gpu


def _lib():
    from paper_1703_06323_amd import cutbddc
    lib = cutbddc.load_library()
    lib.cb_dense_spd_inverse_noalloc.argtypes = [C.c_int32, C.c_int32, C.c_int32, C.c_void_p, C.c_void_p]
    lib.cb_dense_spd_inverse_noalloc.restype = C.c_int
    return lib


def _spd(n, batch, seed):
    rng = np.random.default_rng(seed)
    X = rng.standard_normal((batch, n, n))
    return X @ np.transpose(X, (0, 2, 1)) / n + np.eye(n)[None]


def _noalloc(A, precision):
    lib = _lib()
    A = np.ascontiguousarray(A, dtype=np.float64)
    out = np.full_like(A, np.nan)
    rc = lib.cb_dense_spd_inverse_noalloc(A.shape[1], A.shape[0], precision, A.ctypes.data_as(C.c_void_p),
                                          out.ctypes.data_as(C.c_void_p))
    return rc, out, lib.cb_last_error().decode()


@pytest.mark.parametrize("precision", [0, 1])
def test_noalloc_matches_allocating_entry_point(precision):
    from paper_1703_06323_amd.cutbddc import dense_spd_inverse
    # FP64: both run the same blocked algorithm (the allocating one overlaps
    # its triangular inverse on side streams), so they agree to rounding;
    # FP32: within the FP32 bar of the building block's own test
    tol = 1e-12 if precision == 0 else 1e-4
    for n, batch, seed in ((300, 5, 1), (70, 3, 2)):   # the second call is smaller
        A = _spd(n, batch, seed)
        print(f"[gpu] noalloc spd inverse n={n} batch={batch} precision={precision}", flush=True)
        ref = dense_spd_inverse(A, precision)
        rc, out, msg = _noalloc(A, precision)
        assert rc == 0, msg
        err = np.abs(out - ref).max() / np.abs(ref).max()
        print(f"  max |noalloc - alloc| / max |alloc| = {err:.2e}")
        assert err < tol, err


def test_noalloc_errors():
    from paper_1703_06323_amd.cutbddc import CB_ERR_ARG, CB_ERR_NOT_SPD
    print("[gpu] noalloc error paths", flush=True)
    rc, _, msg = _noalloc(np.zeros((64, 300, 300)), 0)     # ~150 MB of scratch: over the limit
    assert rc == CB_ERR_ARG and "scratch" in msg, (rc, msg)
    A = _spd(40, 3, 5)
    A[1] -= 50.0 * np.eye(40)                                # matrix 1 indefinite
    rc, _, msg = _noalloc(A, 0)
    assert rc == CB_ERR_NOT_SPD and "matrix 1" in msg, (rc, msg)
    # a later valid call on the same array is unaffected
    B = _spd(40, 2, 6)
    rc, out, msg = _noalloc(B, 0)
    assert rc == 0, msg
    assert np.abs(out - np.linalg.inv(B)).max() / np.abs(np.linalg.inv(B)).max() < 1e-12
