"""Pins for occupied-pair screening with localised orbitals (Conclusion:
localised orbitals and the screening of occupied pairs) and for the
synthetic localised orbitals it runs on."""
import numpy as np
import pytest

import workloads
from conftest import rel
from oracle.fmm import Setup, band_ends, band_mask, far_K, pair_bound, pair_screen


@pytest.fixture(scope="module")
def chain40():
    wl = workloads.alkane_chain(n_carbon=40, depth=5)
    C = workloads.localized_orbitals(wl.system, 7)
    return wl, C, Setup(wl.system, wl.params)


def test_localized_orbitals_orthonormal_and_local(chain40):
    wl, C, st = chain40
    S = workloads.overlap_matrix(wl.system)
    assert np.abs(C.T @ S @ C - np.eye(C.shape[1])).max() < 1e-12
    assert C.shape[1] == wl.system.nocc
    # every orbital keeps nearly all its weight within a few bohr of its centroid
    xyz = st.fn.center
    axis = int(np.argmax(np.ptp(wl.system.xyz, 0)))
    w = C * (S @ C)                            # Mulliken-like weights, columns sum to 1
    x = xyz[:, axis]
    centroid = (w * x[:, None]).sum(0)
    far = (np.abs(x[:, None] - centroid[None]) > 10.0)
    assert np.abs((w * far).sum(0)).max() < 1e-2
    # columns follow the chain
    assert np.all(np.diff(centroid) > -3.0)


def test_bound_dominates_brute_force(chain40):
    """b_ij >= sum over the screened pairs (t, u) of K_tu |C_tj| |C_ui|,
    brute force over every pair of functions."""
    wl, C, st = chain40
    fn, r, s = st.fn, st.r, st.s
    a, b = fn.exp[r], fn.exp[s]
    A = np.zeros((st.nbasis, st.nbasis))
    A[r, s] = np.exp(-(a * b / (a + b)) * ((fn.center[r] - fn.center[s]) ** 2).sum(1))
    brute = np.abs(C).T @ A @ np.abs(C)
    B = pair_bound(st, C)
    assert np.all(B >= brute * (1 - 1e-12))
    # and is not loose by orders of magnitude where it matters
    big = brute > 1e-6
    assert np.median(B[big] / brute[big]) < 20.0


def test_screening_keeps_a_band(chain40):
    wl, C, st = chain40
    n = C.shape[1]
    m = pair_screen(st, C, 1e-3)
    assert np.array_equal(m, m.T) and m.diagonal().all()
    assert m.mean() < 0.5
    ii, jj = np.nonzero(m)
    assert np.abs(ii - jj).max() < n // 3
    assert pair_screen(st, C, 0.0).all()


def test_screened_error_falls_with_the_threshold(chain40):
    """Dropping the occupied pairs below tau changes K^ff by less than tau
    (relative), and by less for a smaller tau; keeping every pair changes
    nothing."""
    wl, C, st = chain40
    K0 = far_K(st, C)
    assert np.array_equal(far_K(st, C, pair_mask=pair_screen(st, C, 0.0)), K0)
    errs = []
    for tau in (1e-2, 1e-3, 1e-5):
        e = rel(far_K(st, C, pair_mask=pair_screen(st, C, tau)), K0)
        assert e < tau
        errs.append(e)
    assert errs[0] > errs[1] > errs[2] > 0


def test_band_mask_covers_the_screen(chain40):
    """The banded schedule evaluates every pair the screen keeps, and its
    bands are the tightest that do: each batch ends at its own last j or
    one past a kept pair."""
    wl, C, st = chain40
    n = C.shape[1]
    tau = 1e-4
    m = pair_screen(st, C, tau)
    for jb in (7, 16, 64, n):
        ends = band_ends(st, C, tau, jb)
        assert len(ends) == (n + jb - 1) // jb
        bm = band_mask(n, jb, ends)
        assert np.array_equal(bm, bm.T)
        assert bm[m].all()
        for k, e in enumerate(ends):
            j0, j1 = k * jb, min(n, (k + 1) * jb)
            assert e == j1 or m[e - 1, j0:j1].any()
        if jb == n:
            assert bm.all()
    assert np.array_equal(band_ends(st, C, 0.0, 16), np.full((n + 15) // 16, n))
