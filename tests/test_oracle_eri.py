"""Pins for the oracle's exact integrals and near-field exchange (oracle/eri.py).

* s-type integrals equal the Boys-F0 closed form of oracle/exact.py.
* p-type integrals equal derivatives of s-type ones with respect to the
  centre (x - A_x) e^{-a|r-A|^2} = (1/2a) d/dA_x e^{-a|r-A|^2}, by central
  finite differences (one and two derivatives).
* For two distributions far apart, every integral (up to (pp|pp)) equals
  its multipole expansion (the oracle's AO multipoles by quadrature and its
  M2L matrix, Eq. 3) at high rank: the Gaussian penetration is negligible.
* Permutation symmetries (rs|tu) = (sr|tu) = (rs|ut) = (tu|rs).
* Near field + far field = the whole exchange: with the extent criterion
  (penetration below 1e-8) and L = 10, K^nf + K^ff equals the exchange with
  every pair integral exact.
"""
import math
from types import SimpleNamespace

import numpy as np
import pytest

import workloads
from oracle import fmm
from oracle.basis import Functions, ao_multipoles
from oracle.eri import all_K, eri, near_K, near_K_rows
from oracle.exact import eri_s

from conftest import rel, with_params


def _fn(funcs):
    """Functions-like object from (centre, exponent, powers) tuples."""
    c = np.array([f[0] for f in funcs], dtype=float)
    e = np.array([f[1] for f in funcs], dtype=float)
    pw = np.array([f[2] for f in funcs], dtype=np.int64)
    lsum = pw.sum(1)
    norm = (2 * e / math.pi) ** 0.75 * np.where(lsum == 1, 2 * np.sqrt(e), 1.0)
    return SimpleNamespace(center=c, exp=e, pow=pw, norm=norm, n=len(e))


def test_s_type_equals_boys_closed_form(tiny):
    wl, C, st = tiny
    fn = st.fn
    rng = np.random.default_rng(0)
    r, s, t, u = (rng.integers(0, fn.n, 400) for _ in range(4))
    v = eri(fn, r, s, t, u)
    a, b, c, d = fn.exp[r], fn.exp[s], fn.exp[t], fn.exp[u]
    p, q = a + b, c + d
    Kab = np.exp(-(a * b / p) * ((fn.center[r] - fn.center[s]) ** 2).sum(1))
    Kcd = np.exp(-(c * d / q) * ((fn.center[t] - fn.center[u]) ** 2).sum(1))
    P = (a[:, None] * fn.center[r] + b[:, None] * fn.center[s]) / p[:, None]
    Q = (c[:, None] * fn.center[t] + d[:, None] * fn.center[u]) / q[:, None]
    ref = eri_s(p, q, fn.norm[r] * fn.norm[s] * Kab, fn.norm[t] * fn.norm[u] * Kcd, np.linalg.norm(P - Q, axis=1))
    assert np.abs(v - ref).max() <= 1e-13 * np.abs(ref).max()


X = np.eye(3)
CENTRES = [np.array([0.1, -0.2, 0.3]), np.array([1.3, 0.4, -0.5]), np.array([-0.6, 1.1, 0.2]),
           np.array([0.7, -0.9, 1.4])]
EXPS = [0.9, 1.7, 0.6, 1.2]


@pytest.mark.parametrize("slot,dim", [(0, 0), (1, 1), (2, 2), (3, 0)])
def test_one_p_equals_centre_derivative(slot, dim):
    """(.. p_dim ..) at slot = (1/sqrt(a)) d/dA_dim of the s integral."""
    h = 1e-4
    funcs = [(CENTRES[k], EXPS[k], (0, 0, 0)) for k in range(4)]
    fp = list(funcs)
    fp[slot] = (CENTRES[slot], EXPS[slot], tuple(int(v) for v in X[dim]))
    got = eri(_fn(fp), [0], [1], [2], [3])[0]
    vals = []
    for sgn in (1, -1):
        f2 = list(funcs)
        f2[slot] = (CENTRES[slot] + sgn * h * X[dim], EXPS[slot], (0, 0, 0))
        vals.append(eri(_fn(f2), [0], [1], [2], [3])[0])
    ref = (vals[0] - vals[1]) / (2 * h) / math.sqrt(EXPS[slot])
    assert got == pytest.approx(ref, rel=1e-7, abs=1e-12)


@pytest.mark.parametrize("s1,d1,s2,d2", [(0, 0, 1, 0), (0, 1, 2, 2), (2, 0, 3, 1), (1, 2, 3, 2)])
def test_two_p_equal_mixed_centre_derivative(s1, d1, s2, d2):
    h = 1e-3
    funcs = [(CENTRES[k], EXPS[k], (0, 0, 0)) for k in range(4)]
    fp = list(funcs)
    fp[s1] = (CENTRES[s1], EXPS[s1], tuple(int(v) for v in X[d1]))
    fp[s2] = (CENTRES[s2], EXPS[s2], tuple(int(v) for v in X[d2]))
    got = eri(_fn(fp), [0], [1], [2], [3])[0]
    acc = 0.0
    for e1 in (1, -1):
        for e2 in (1, -1):
            f2 = list(funcs)
            f2[s1] = (CENTRES[s1] + e1 * h * X[d1], EXPS[s1], (0, 0, 0))
            f2[s2] = (CENTRES[s2] + e2 * h * X[d2], EXPS[s2], (0, 0, 0))
            acc += e1 * e2 * eri(_fn(f2), [0], [1], [2], [3])[0]
    ref = acc / (4 * h * h) / math.sqrt(EXPS[s1] * EXPS[s2])
    assert got == pytest.approx(ref, rel=1e-5, abs=1e-12)


def test_far_apart_integrals_equal_multipole_expansion():
    """Every (ab|cd) type up to (pp|pp), distributions 14 bohr apart: the
    exact integral equals sum (-1)^l O^{ab}_lm M_{l+l',m+m'} O^{cd}_l'm' at L = 16."""
    L = 16
    Xa, Xb = np.array([0.2, -0.1, 0.3]), np.array([13.5, 3.0, -2.0])
    shells = [(0, 0, 0), (1, 0, 0), (0, 1, 0), (0, 0, 1)]
    funcs = []
    for cen in (Xa, Xa + [0.6, 0.2, -0.3], Xb, Xb + [-0.4, 0.5, 0.1]):
        for pw in shells:
            funcs.append((cen, 1.1, pw))
    fn = _fn(funcs)
    T = fmm.m2l_matrix(L, Xa - Xb)
    bra = [(a, b) for a in range(0, 8) for b in range(0, 8)]
    ket = [(c, d) for c in range(8, 16) for d in range(8, 16)]
    Ob = ao_multipoles(fn, np.array([x[0] for x in bra]), np.array([x[1] for x in bra]), Xa, L)
    Ok = ao_multipoles(fn, np.array([x[0] for x in ket]), np.array([x[1] for x in ket]), Xb, L)
    approx = (Ob @ T @ Ok.T).real
    R, S = np.meshgrid(np.arange(len(bra)), np.arange(len(ket)), indexing="ij")
    br, kt = np.array(bra), np.array(ket)
    exact = eri(fn, br[R.ravel(), 0], br[R.ravel(), 1], kt[S.ravel(), 0], kt[S.ravel(), 1]).reshape(approx.shape)
    assert np.abs(exact - approx).max() <= 1e-10 * np.abs(exact).max()


def test_permutation_symmetry():
    wl = workloads.sp_chain(n=4)
    fn = Functions(wl.system)
    rng = np.random.default_rng(1)
    r, s, t, u = (rng.integers(0, fn.n, 300) for _ in range(4))
    v = eri(fn, r, s, t, u)
    for perm in ((s, r, t, u), (r, s, u, t), (t, u, r, s), (u, t, s, r)):
        assert np.abs(eri(fn, *perm) - v).max() <= 1e-13 * np.abs(v).max()


def test_near_plus_far_is_the_whole_exchange():
    """Extent criterion (penetration of far pairs below 1e-8), L = 10:
    K^nf (exact integrals, near leaf pairs) + K^ff (multipoles) equals the
    exchange with every integral exact."""
    from oracle.fmm import Setup
    wl = workloads.sp_chain(n=8)
    p = with_params(wl, near_rule=1, ext_ws=0.0, ext_tau=1e-8, lmax=10)
    st = Setup(wl.system, p)
    assert st.tree.lmin is not None
    C = wl.orbitals()
    Kn = near_K(st, C)
    Kf = fmm.far_K(st, C)
    Ka = all_K(st, C)
    assert np.abs(Kf).max() > 1e-6 * np.abs(Ka).max()    # the far field is not empty
    assert rel(Kn + Kf, Ka) <= 1e-7
    assert rel(Kn, Ka) > 1e-5                             # the near field alone is not the whole


def test_sampled_rows_equal_the_full_near_field():
    from oracle.fmm import Setup
    wl = workloads.sp_chain(n=8)
    st = Setup(wl.system, with_params(wl, lmax=0))
    C = wl.orbitals()
    K = near_K(st, C)
    rows = [0, 7, 21, 39]
    assert rel(near_K_rows(st, C, rows), K[rows]) <= 1e-13
