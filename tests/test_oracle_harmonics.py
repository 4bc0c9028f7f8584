"""Pins for the oracle's solid harmonics and translation operators.

They check Eq. (3)-(4) and the translation identities against facts fixed by
the mathematics, not against the oracle's own formulas: scipy's associated
Legendre routine, the Coulomb potential 1/r12, the addition theorem of the
regular harmonics and exact re-centring of polynomials.
"""
import math

import numpy as np
import pytest
from scipy.special import lpmv

from oracle import harmonics as H
from oracle.fmm import l2l_matrix, m2l_matrix, m2m_matrix


def _sph(v):
    r = np.linalg.norm(v, axis=-1)
    return r, np.arccos(v[..., 2] / r), np.arctan2(v[..., 1], v[..., 0])


@pytest.mark.parametrize("L", [0, 3, 8, 16])
def test_eq4_against_scipy_lpmv(L):
    rng = np.random.default_rng(10 + L)
    v = rng.standard_normal((7, 3)) * 3.0
    O, M = H.regular(L, v), H.irregular(L, v)
    r, th, ph = _sph(v)
    for l in range(L + 1):
        for m in range(-l, l + 1):
            am = abs(m)
            eps = 1.0 if m >= 0 else (-1.0) ** m
            P = lpmv(am, l, np.cos(th))
            o = eps * r ** l / math.factorial(l + am) * P * np.exp(-1j * m * ph)
            mm = eps * math.factorial(l - am) / r ** (l + 1) * P * np.exp(1j * m * ph)
            assert np.allclose(O[:, H.idx(l, m)], o, rtol=1e-11, atol=1e-14 * np.abs(o).max())
            assert np.allclose(M[:, H.idx(l, m)], mm, rtol=1e-11, atol=1e-14 * np.abs(mm).max())


def test_regular_on_axis_and_origin():
    O = H.regular(4, np.array([[0.0, 0.0, 2.0], [0.0, 0.0, 0.0]]))
    # on the z axis only m = 0 survives: O_l0 = z^l / l!
    for l in range(5):
        assert O[0, H.idx(l, 0)] == pytest.approx(2.0 ** l / math.factorial(l))
        for m in range(1, l + 1):
            assert abs(O[0, H.idx(l, m)]) < 1e-15 and abs(O[0, H.idx(l, -m)]) < 1e-15
    assert O[1, 0] == 1.0 and np.all(O[1, 1:] == 0)


def test_symmetries():
    rng = np.random.default_rng(3)
    v = rng.standard_normal((5, 3))
    L = 6
    O, M = H.regular(L, v), H.irregular(L, v)
    On, Mn = H.regular(L, -v), H.irregular(L, -v)
    for l in range(L + 1):
        for m in range(-l, l + 1):
            # conjugate symmetry X_{l,-m} = (-1)^m conj(X_{l,m})
            assert np.allclose(O[:, H.idx(l, -m)], (-1) ** m * np.conj(O[:, H.idx(l, m)]), atol=1e-14)
            assert np.allclose(M[:, H.idx(l, -m)], (-1) ** m * np.conj(M[:, H.idx(l, m)]), atol=1e-14)
            # parity
            assert np.allclose(On[:, H.idx(l, m)], (-1) ** l * O[:, H.idx(l, m)], atol=1e-14)
            assert np.allclose(Mn[:, H.idx(l, m)], (-1) ** l * M[:, H.idx(l, m)], atol=1e-14)


def test_addition_theorem_regular():
    """O_lm(a+b) = sum_{l'm'} O_{l-l',m-m'}(a) O_{l'm'}(b) (exact)."""
    rng = np.random.default_rng(4)
    a, b = rng.standard_normal(3), rng.standard_normal(3)
    L = 7
    lhs = H.regular(L, a + b)
    Oa, Ob = H.regular(L, a), H.regular(L, b)
    for l in range(L + 1):
        for m in range(-l, l + 1):
            s = 0
            for lp in range(l + 1):
                for mp in range(-lp, lp + 1):
                    if abs(m - mp) <= l - lp:
                        s += Oa[H.idx(l - lp, m - mp)] * Ob[H.idx(lp, mp)]
            assert abs(s - lhs[H.idx(l, m)]) < 1e-13 * max(1.0, abs(lhs[H.idx(l, m)]))


def _expansion(L, a, b, R):
    """Eq. (3): sum (-1)^l O_lm(a) M_{l+l',m+m'}(R) O_l'm'(b), square truncation."""
    Oa, Ob, MR = H.regular(L, a), H.regular(L, b), H.irregular(2 * L, R)
    s = 0
    for l in range(L + 1):
        for m in range(-l, l + 1):
            for lp in range(L + 1):
                for mp in range(-lp, lp + 1):
                    s += (-1) ** l * Oa[H.idx(l, m)] * MR[H.idx(l + lp, m + mp)] * Ob[H.idx(lp, mp)]
    return s


def test_eq3_converges_to_coulomb():
    """Eq. (3) -> 1/|r1 - r2| geometrically for |a| + |b| < |R|."""
    X = np.zeros(3)
    Xp = np.array([5.0, 3.0, -2.0])
    a = np.array([0.5, -0.3, 0.4])
    b = np.array([-0.2, 0.6, 0.1])
    exact = 1.0 / np.linalg.norm((X + a) - (Xp + b))
    ratio = (np.linalg.norm(a) + np.linalg.norm(b)) / np.linalg.norm(X - Xp)
    errs = []
    for L in (1, 2, 4, 8, 12):
        s = _expansion(L, a, b, X - Xp)
        assert abs(s.imag) < 1e-15
        err = abs(s.real - exact) / exact
        errs.append(err)
        assert err <= 2.0 * ratio ** (L + 1) + 1e-15
    assert errs[-1] < 1e-12
    assert all(e2 < e1 for e1, e2 in zip(errs, errs[1:]))


def test_eq3_sign_on_the_source_index_fails():
    """The parity factor belongs to the r1 (X) index: moving it to the r2 index
    (a plausible mistake) gives a wrong potential."""
    a = np.array([0.5, -0.3, 0.4])
    b = np.array([-0.2, 0.6, 0.1])
    R = np.array([5.0, 3.0, -2.0])
    exact = 1.0 / np.linalg.norm(R + a - b)
    L = 8
    Oa, Ob, MR = H.regular(L, a), H.regular(L, b), H.irregular(2 * L, R)
    wrong = 0
    for l in range(L + 1):
        for m in range(-l, l + 1):
            for lp in range(L + 1):
                for mp in range(-lp, lp + 1):
                    wrong += (-1) ** lp * Oa[H.idx(l, m)] * MR[H.idx(l + lp, m + mp)] * Ob[H.idx(lp, mp)]
    assert abs(_expansion(L, a, b, R).real - exact) / exact < 1e-8
    assert abs(wrong.real - exact) / exact > 1e-2


def test_m2m_matrix_shifts_point_multipoles_exactly():
    """Multipoles of point charges about Xc, translated by Eq. (11), equal the
    multipoles taken directly about Xp (exact for every l <= L)."""
    rng = np.random.default_rng(5)
    Xc, Xp = np.array([0.3, -0.2, 0.5]), np.array([1.0, 1.0, -1.0])
    pts = Xc + rng.uniform(-0.5, 0.5, (6, 3))
    q = rng.standard_normal(6)
    L = 6
    oc = (q[:, None] * H.regular(L, pts - Xc)).sum(0)
    op = (q[:, None] * H.regular(L, pts - Xp)).sum(0)
    assert np.allclose(m2m_matrix(L, Xc - Xp) @ oc, op, rtol=1e-12, atol=1e-13)


def test_l2l_matrix_recentres_exactly():
    """sum O_lm(r-Xp) Mp_lm == sum O_lm(r-Xc) (T Mp)_lm for any coefficients."""
    rng = np.random.default_rng(6)
    L = 5
    Q = H.ncomp(L)
    Mp = rng.standard_normal(Q) + 1j * rng.standard_normal(Q)
    Xp, Xc = np.array([0.0, 0.0, 0.0]), np.array([0.7, -0.4, 0.2])
    Mc = l2l_matrix(L, Xc - Xp) @ Mp
    for r in rng.standard_normal((4, 3)):
        v1 = H.regular(L, r - Xp) @ Mp
        v2 = H.regular(L, r - Xc) @ Mc
        assert abs(v1 - v2) < 1e-12 * max(1, abs(v1))


def test_m2l_potential_of_point_charges():
    """Eq. (12) local expansion evaluated near X reproduces sum q/|r - x| as L grows."""
    rng = np.random.default_rng(7)
    X, Xs = np.zeros(3), np.array([6.0, -2.0, 3.0])
    src = Xs + rng.uniform(-0.8, 0.8, (5, 3))
    q = rng.uniform(0.5, 1.5, 5)
    r = X + np.array([0.4, 0.3, -0.5])
    exact = np.sum(q / np.linalg.norm(r - src, axis=1))
    prev = None
    for L in (2, 4, 8):
        om = (q[:, None] * H.regular(L, src - Xs)).sum(0)
        loc = m2l_matrix(L, X - Xs) @ om
        val = H.regular(L, r - X) @ loc
        err = abs(val - exact) / exact
        assert abs(val.imag) < 1e-14
        if prev is not None:
            assert err < prev
        prev = err
    assert prev < 1e-6


@pytest.mark.parametrize("L", [2, 4])
def test_axis_aligned_translations_are_block_diagonal(L):
    """A displacement on the x axis is unchanged by the reflections y -> -y
    and z -> -z, one in the xy plane by z -> -z.  The translation operators
    commute with them, so for x-axis displacements every M2M, M2L and L2L
    matrix is real and couples (l, m) to (l', m') only when l + m and l' + m'
    have the same parity; for xy-plane displacements the parity rule holds.
    The zeros are exact (a zero y or z stays zero through the harmonics'
    recurrences), which is what lets the library skip them."""
    Q = H.ncomp(L)
    par = np.array([(l + m) & 1 for l in range(L + 1) for m in range(-l, l + 1)])
    cross = par[:, None] != par[None, :]
    for d in ([2.7, 0.0, 0.0], [-5.1, 0.0, 0.0], [3.3, -1.9, 0.0], [0.0, 4.2, 0.0]):
        d = np.array(d)
        for T in (m2m_matrix(L, d), l2l_matrix(L, d), m2l_matrix(L, 4.0 * d)):
            assert T.shape == (Q, Q)
            assert np.all(T[cross] == 0), d
            if d[1] == 0.0:
                assert np.all(T.imag == 0), d
    # a generic displacement has no such zeros
    T = m2l_matrix(L, np.array([2.1, -1.3, 0.7]))
    assert np.count_nonzero(T[cross]) == np.count_nonzero(cross)
