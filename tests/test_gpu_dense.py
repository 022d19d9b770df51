"""GPU parity of the batched SPD inverse building block (blocked Cholesky,
triangular inverse, Y^T Y on MFMA) against numpy on random SPD matrices,
sizes spanning several 32-wide tiles and a ragged tail."""
import sys

import numpy as np
import pytest

pytestmark = pytest.mark.gpu


@pytest.mark.parametrize("n,batch", [(1, 1), (31, 2), (32, 1), (33, 3), (100, 2), (257, 2), (300, 3), (700, 1)])
@pytest.mark.parametrize("precision", [0, 1])
def test_spd_inverse(n, batch, precision):
    from paper_1703_06323_amd.cutbddc import dense_spd_inverse
    rng = np.random.default_rng(n * 7 + batch)
    X = rng.standard_normal((batch, n, n))
    A = X @ np.transpose(X, (0, 2, 1)) / n + np.eye(n)[None]
    print(f"[gpu] spd_inverse n={n} batch={batch} precision={precision}", flush=True)
    Ai = dense_spd_inverse(A, precision)
    ref = np.linalg.inv(A)
    err = np.abs(Ai - ref).max() / np.abs(ref).max()
    assert err < (1e-12 if precision == 0 else 1e-4), err
