"""Lanczos eigenvalue estimates from CG coefficients (cb_lanczos_extremes,
host code of the library; used by cb_pcg_history and cb_query): against the
spectrum that CG explores exactly on a small diagonal system, and against
the oracle's dense tridiagonal eigensolver on random coefficients."""
import os

import numpy as np
import pytest

from oracle import pcg

LIB = os.path.join(os.path.dirname(os.path.dirname(os.path.abspath(__file__))), "paper_1703_06323_amd",
                   "libcutbddc.so")
pytestmark = pytest.mark.skipif(not os.path.exists(LIB), reason="library not built")


def _cg_coefficients(diag, b, steps):
    """Plain CG (M = I) on diag(diag) x = b: the alphas and betas."""
    x = np.zeros_like(b)
    r = b.copy()
    p = r.copy()
    rho = r @ r
    al, be = [], []
    for k in range(steps):
        q = diag * p
        a = rho / (p @ q)
        x += a * p
        r -= a * q
        al.append(a)
        if k + 1 == steps:
            break
        rn = r @ r
        be.append(rn / rho)
        rho = rn
        p = r + be[-1] * p
    return np.array(al), np.array(be)


def test_full_krylov_space_gives_the_exact_extremes():
    """After n steps on an n x n SPD matrix with distinct eigenvalues, the
    Lanczos matrix has exactly the matrix's eigenvalues."""
    from paper_1703_06323_amd.cutbddc import lanczos_extremes
    diag = np.arange(1.0, 11.0)
    al, be = _cg_coefficients(diag, np.ones(10), 10)
    lo, hi = lanczos_extremes(al, be)
    assert abs(lo - 1.0) <= 1e-8 and abs(hi - 10.0) <= 1e-8


@pytest.mark.parametrize("n,seed", [(1, 0), (2, 1), (7, 2), (60, 3), (400, 4)])
def test_matches_the_oracle_on_random_coefficients(n, seed):
    from paper_1703_06323_amd.cutbddc import lanczos_extremes
    rng = np.random.default_rng(seed)
    al = rng.uniform(0.05, 2.0, n)
    be = rng.uniform(0.0, 0.9, max(n - 1, 0))
    lo, hi = lanczos_extremes(al, be)
    wlo, whi = pcg.lanczos_condition(list(al), list(be))
    assert abs(lo - wlo) <= 1e-12 * abs(whi) and abs(hi - whi) <= 1e-12 * abs(whi)


def test_no_step_and_bad_coefficients():
    from paper_1703_06323_amd import cutbddc
    assert cutbddc.lanczos_extremes([], []) == (1.0, 1.0)
    with pytest.raises(cutbddc.CBError):
        cutbddc.lanczos_extremes([1.0, -0.5], [0.1])
    with pytest.raises(cutbddc.CBError):
        cutbddc.lanczos_extremes([1.0, 0.5], [-0.1])
