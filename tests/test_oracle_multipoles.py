"""Pins for the oracle's AO multipole integrals, Eq. (8).

* s-type: a product of two s Gaussians is spherically symmetric about P and
  O_lm is a harmonic polynomial, so by the mean-value property
  O^{rs,X}_lm = S_rs O_lm(P - X) exactly; S_rs is the closed-form overlap.
* p-type: (x - A_x) exp(-a|r-A|^2) = (1/2a) d/dA_x exp(-a|r-A|^2), so a p
  multipole is a centre derivative of an s multipole; checked by a
  Richardson-extrapolated central difference of the s-type closed form.
* quadrature order: exact, so adding nodes changes nothing.
* re-centring: the multipoles of one pair about two centres are related by
  the addition theorem (Eq. 11) exactly.
"""
import math

import numpy as np
import pytest

import workloads
from oracle import harmonics as H
from oracle.basis import Functions, ao_multipoles, function_pairs
from oracle.fmm import m2m_matrix


def _ss_closed(a, A, b, B, X, L):
    p = a + b
    P = (a * A + b * B) / p
    Na, Nb = (2 * a / math.pi) ** 0.75, (2 * b / math.pi) ** 0.75
    S = Na * Nb * (math.pi / p) ** 1.5 * math.exp(-a * b / p * np.dot(A - B, A - B))
    return S * H.regular(L, P - X)


def test_s_type_mean_value_property(tiny):
    wl, C, st = tiny
    fn = st.fn
    rng = np.random.default_rng(0)
    k = rng.choice(len(st.r), 50, replace=False)
    X = np.array([3.0, 0.5, -0.4])
    L = 6
    got = ao_multipoles(fn, st.r[k], st.s[k], X, L)
    for n, kk in enumerate(k):
        r, s = st.r[kk], st.s[kk]
        ref = _ss_closed(fn.exp[r], fn.center[r], fn.exp[s], fn.center[s], X, L)
        assert np.allclose(got[n], ref, rtol=1e-12, atol=1e-14 * max(1e-300, np.abs(ref).max()))


def _unnorm_ss(a, A, b, B, X, L):
    p = a + b
    P = (a * A + b * B) / p
    return (math.pi / p) ** 1.5 * math.exp(-a * b / p * np.dot(A - B, A - B)) * H.regular(L, P - X)


def _p_by_derivative(a, A, d, b, B, X, L):
    """integral N_p (x_d - A_d) e^{-a|r-A|^2} N_s e^{-b|r-B|^2} O_lm(r - X)."""
    Np = (2 * a / math.pi) ** 0.75 * 2 * math.sqrt(a)
    Ns = (2 * b / math.pi) ** 0.75

    def f(hh):
        e = np.zeros(3)
        e[d] = hh
        return (_unnorm_ss(a, A + e, b, B, X, L) - _unnorm_ss(a, A - e, b, B, X, L)) / (2 * hh)
    h = 1e-3
    deriv = (4 * f(h / 2) - f(h)) / 3.0        # Richardson, O(h^4)
    return Np * Ns * deriv / (2 * a)


def test_p_type_against_centre_derivative():
    wl = workloads.graphene_flake(n=2, nocc=12, depth=3)
    fn = Functions(wl.system)
    r, s, P = function_pairs(wl.system, fn, wl.params.pair_log_thresh)
    sel = np.nonzero((fn.pow[r].sum(1) == 1) & (fn.pow[s].sum(1) == 0) & (fn.exp[r] < 30) & (fn.exp[s] < 30))[0]
    rng = np.random.default_rng(1)
    k = rng.choice(sel, 40, replace=False)
    L = 4
    X = np.array([1.0, -2.0, 0.3])
    got = ao_multipoles(fn, r[k], s[k], X, L)
    for n, kk in enumerate(k):
        rr, ss = r[kk], s[kk]
        d = int(np.argmax(fn.pow[rr]))
        ref = _p_by_derivative(fn.exp[rr], fn.center[rr], d, fn.exp[ss], fn.center[ss], X, L)
        scale = np.abs(ref).max()
        assert np.allclose(got[n], ref, rtol=0, atol=1e-7 * scale)


def test_quadrature_order_independent():
    wl = workloads.graphene_flake(n=2, nocc=12, depth=3)
    fn = Functions(wl.system)
    r, s, P = function_pairs(wl.system, fn, wl.params.pair_log_thresh)
    k = np.random.default_rng(2).choice(len(r), 60, replace=False)
    X = np.array([0.5, 0.5, 0.5])
    a = ao_multipoles(fn, r[k], s[k], X, 5)
    b = ao_multipoles(fn, r[k], s[k], X, 5, nquad=9)
    assert np.allclose(a, b, rtol=1e-11, atol=1e-14 * np.abs(a).max())


def test_multipole_recentring_is_m2m():
    wl = workloads.graphene_flake(n=2, nocc=12, depth=3)
    fn = Functions(wl.system)
    r, s, P = function_pairs(wl.system, fn, wl.params.pair_log_thresh)
    k = np.random.default_rng(3).choice(len(r), 30, replace=False)
    Xc, Xp = np.array([0.2, 0.1, 0.0]), np.array([2.0, -1.5, 0.0])
    L = 4
    oc = ao_multipoles(fn, r[k], s[k], Xc, L)
    op = ao_multipoles(fn, r[k], s[k], Xp, L)
    T = m2m_matrix(L, Xc - Xp)
    assert np.allclose(oc @ T.T, op, rtol=1e-11, atol=1e-13 * np.abs(op).max())


def test_overlap_matches_input_overlap():
    """The l=0 multipole is the overlap; compare with the workloads' S (another
    closed form written for input preparation)."""
    wl = workloads.graphene_flake(n=2, nocc=12, depth=3)
    fn = Functions(wl.system)
    S = workloads.overlap_matrix(wl.system)
    r, s, P = function_pairs(wl.system, fn, wl.params.pair_log_thresh)
    k = np.random.default_rng(4).choice(len(r), 200, replace=False)
    got = ao_multipoles(fn, r[k], s[k], np.zeros(3), 0)[:, 0].real
    assert np.allclose(got, S[r[k], s[k]], rtol=1e-12, atol=1e-15)
