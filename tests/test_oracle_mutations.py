"""Planted mistakes in the oracle (on the CPU) must be caught by the pins.

Each case patches one oracle routine with a plausible error and checks that the
corresponding pin (hierarchical == direct, or convergence to the point-charge
limit) no longer holds.
"""
import numpy as np
import pytest

from oracle import fmm
from oracle.exact import far_K_exact_s

from conftest import rel


def _hier_vs_direct(st, C):
    return rel(fmm.far_K(st, C), fmm.far_K_direct(st, C))


def test_transposed_m2m_is_caught(tiny, monkeypatch):
    wl, C, st = tiny
    orig = fmm.m2m_matrix
    monkeypatch.setattr(fmm, "m2m_matrix", lambda L, d: orig(L, d).T.copy())
    assert _hier_vs_direct(st, C) > 1e-3


def test_l2l_wrong_displacement_sign_is_caught(tiny, monkeypatch):
    wl, C, st = tiny
    orig = fmm.l2l_matrix
    monkeypatch.setattr(fmm, "l2l_matrix", lambda L, d: orig(L, -d))
    assert _hier_vs_direct(st, C) > 1e-3


def test_m2l_missing_parity_is_caught(tiny, monkeypatch):
    wl, C, st = tiny
    Kp = far_K_exact_s(st, C, "pc")
    good = rel(fmm.far_K(st, C), Kp)
    orig = fmm.m2l_matrix

    def no_parity(L, R):
        T = orig(L, R)
        for l in range(L + 1):
            T[l * l:(l + 1) * (l + 1)] *= (-1) ** l
        return T
    monkeypatch.setattr(fmm, "m2l_matrix", no_parity)
    bad = rel(fmm.far_K(st, C), Kp)
    assert good < 2e-2 and bad > 10 * good


def test_truncation_keeping_p_squared_components_is_caught(tiny, monkeypatch):
    """Rank truncation that keeps p^2 instead of (p+1)^2 components (drops the
    whole order l = p) breaks the rank-p == lmax-p pin."""
    from oracle.fmm import Setup
    from conftest import with_params
    wl, C, st = tiny
    st3 = Setup(wl.system, with_params(wl, lmax=3))
    st2 = Setup(wl.system, with_params(wl, lmax=2))
    good = rel(fmm.far_K(st3, C, m2l_rank=2), fmm.far_K(st2, C))

    def short(T, p):
        n = p * p
        out = np.zeros_like(T)
        out[:n, :n] = T[:n, :n]
        return out
    monkeypatch.setattr(fmm, "truncate", short)
    bad = rel(fmm.far_K(st3, C, m2l_rank=2), fmm.far_K(st2, C))
    assert good < 1e-13 and bad > 1e-3


def test_coulomb_missing_parity_is_caught(tiny, monkeypatch):
    """(-1)^l dropped from the M2L operator: J^ff no longer converges to the
    point-charge far field."""
    from oracle.exact import far_J_exact_s
    wl, C, st = tiny
    Dm = 2.0 * C @ C.T
    Jp = far_J_exact_s(st, Dm, "pc")
    good = rel(fmm.far_J(st, Dm), Jp)
    orig = fmm.m2l_matrix

    def no_parity(L, R):
        T = orig(L, R)
        for l in range(L + 1):
            T[l * l:(l + 1) * (l + 1)] *= (-1) ** l
        return T
    monkeypatch.setattr(fmm, "m2l_matrix", no_parity)
    bad = rel(fmm.far_J(st, Dm), Jp)
    assert good < 2e-2 and bad > 10 * good


def test_coulomb_transposed_m2m_is_caught(tiny, monkeypatch):
    wl, C, st = tiny
    Dm = 2.0 * C @ C.T
    orig = fmm.m2m_matrix
    monkeypatch.setattr(fmm, "m2m_matrix", lambda L, d: orig(L, d).T.copy())
    assert rel(fmm.far_J(st, Dm), fmm.far_J_direct(st, Dm)) > 1e-3
