"""Pins for the oracle's step-by-step occ-FMM-K far field (Eqs. 15-18).

* Hierarchical translations == direct ancestor-centred sum (exact identity:
  M2M and L2L are exact for truncated expansions), on a 1-D s-only chain and
  a 2-D s+p sheet.  Catches a transposed or mis-signed M2M/L2L operator.
* L = 0 reduces to monopoles: K_ri = 2 sum S_rs C_sj S_tu C_tj C_ui / |Xa - Xb|.
* s-type chain: as L grows K_FMM(L) converges to the point-charge far field;
  the point-charge far field differs from the exact (Boys F0) far field only
  by the tiny Gaussian-penetration term.  Catches a wrong factor (e.g. the 2
  of Eq. 5) or a wrong sign/placement of (-1)^l.
* The Boys closed form itself is checked against an independent Fourier-space
  quadrature.
* Invariants: K_ij = C^T K symmetric; additivity over j and i ranges; rigid
  shift; atom permutation.
"""
import copy
import math

import numpy as np
import pytest
from scipy.integrate import quad

import workloads
from oracle.exact import eri_s, far_K_exact_s
from oracle.fmm import Setup, far_K, far_K_direct

from conftest import rel, small_sheet, with_params


@pytest.fixture(scope="module")
def sheet():
    wl = small_sheet(lmax=3, depth=3)
    return wl, wl.orbitals(), Setup(wl.system, wl.params)


def test_hierarchical_equals_direct_chain(tiny):
    wl, C, st = tiny
    K = far_K(st, C, jblock=7)
    Kd = far_K_direct(st, C)
    assert rel(K, Kd) < 1e-13


def test_hierarchical_equals_direct_sheet(sheet):
    wl, C, st = sheet
    assert st.tree.lmin < st.tree.depth      # translations are exercised
    K, im = far_K(st, C, return_imag=True)
    Kd = far_K_direct(st, C)
    assert rel(K, Kd) < 1e-12
    assert im < 1e-12 * np.abs(K).max()


def test_L0_is_monopole_sum(tiny):
    wl, C, st = tiny
    st0 = Setup(wl.system, with_params(wl, lmax=0))
    K = far_K(st0, C)
    t = st0.tree
    S = workloads.overlap_matrix(wl.system)
    n = wl.system.nbasis
    Kref = np.zeros_like(K)
    for b1 in range(st0.nleaf):
        for b2 in range(st0.nleaf):
            lev = t.far_level(b1, b2)
            if lev is None:
                continue
            Xa = t.centre(lev, t.boxes[lev][t.ancestor(lev, b1)])
            Xb = t.centre(lev, t.boxes[lev][t.ancestor(lev, b2)])
            k1, k2 = st0.leaf_pairs[b1], st0.leaf_pairs[b2]
            r, s = st0.r[k1], st0.s[k1]
            tt, u = st0.r[k2], st0.s[k2]
            # sum_{tu} S_tu C_tj C_ui -> (j, i)
            om = np.einsum("k,kj,ki->ji", S[tt, u], C[tt], C[u])
            h = S[r, s][:, None] * C[s]                    # (k, j)
            contrib = 2.0 * (h @ om) / np.linalg.norm(Xa - Xb)
            np.add.at(Kref, r, contrib)
    assert rel(K, Kref) < 1e-12


def test_boys_closed_form_vs_fourier_quadrature():
    """(ab|cd) = S_ab S_cd (2/pi) int_0^inf sin(kR)/(kR) exp(-k^2/(4 alpha)) dk."""
    for p, q, R in [(0.2, 0.3, 3.0), (2.0, 0.25, 1.3), (20.0, 5.0, 0.4), (0.2, 0.2, 9.0)]:
        alpha = p * q / (p + q)
        f = lambda k: (np.sinc(k * R / math.pi)) * math.exp(-k * k / (4 * alpha))
        val, _ = quad(f, 0, np.inf, limit=400, epsabs=1e-14, epsrel=1e-12)
        ref = (2 / math.pi) * val
        # S_ab = pref (pi/p)^1.5 with pref = N_a N_b K_ab; use pref = (p/pi)^1.5 -> S = 1
        got = eri_s(p, q, (p / math.pi) ** 1.5, (q / math.pi) ** 1.5, R)
        assert got == pytest.approx(ref, rel=1e-10)


@pytest.fixture(scope="module")
def chain_refs(tiny):
    wl, C, st = tiny
    return far_K_exact_s(st, C, "exact"), far_K_exact_s(st, C, "pc")


def test_fmm_converges_to_point_charge_limit(tiny, chain_refs):
    wl, C, st = tiny
    Ke, Kp = chain_refs
    errs = []
    for L in (2, 4, 6, 8):
        stL = st if L == 2 else Setup(wl.system, with_params(wl, lmax=L))
        errs.append(rel(far_K(stL, C), Kp))
    assert all(b < 0.1 * a for a, b in zip(errs, errs[1:])), errs
    assert errs[-1] < 1e-6


def test_fmm_matches_exact_boys_far_field(tiny, chain_refs):
    """|K_FMM(L) - K_exact| is within truncation + penetration; the penetration
    part (point charge vs Boys) is small for this chain."""
    wl, C, st = tiny
    Ke, Kp = chain_refs
    assert rel(Kp, Ke) < 1e-5
    K2 = far_K(st, C)
    assert rel(K2, Ke) < 2e-2
    st8 = Setup(wl.system, with_params(wl, lmax=8))
    K8 = far_K(st8, C)
    assert rel(K8, Ke) < 5e-6
    # half of it (a dropped factor 2) is far outside
    assert rel(0.5 * K8, Ke) > 0.4


def test_symmetry_of_Kij(sheet):
    wl, C, st = sheet
    K = far_K(st, C)
    Kij = C.T @ K
    assert np.abs(Kij - Kij.T).max() < 1e-12 * np.abs(Kij).max()


def test_column_additivity(sheet):
    wl, C, st = sheet
    n = C.shape[1]
    K = far_K(st, C)
    Kj = far_K(st, C, j_range=(0, 5)) + far_K(st, C, j_range=(5, n))
    assert rel(Kj, K) < 1e-13
    Ki = np.hstack([far_K(st, C, i_range=(0, 7)), far_K(st, C, i_range=(7, n))])
    assert rel(Ki, K) < 1e-13


def test_rigid_shift_invariance(tiny):
    wl, C, st = tiny
    sysm = copy.deepcopy(wl.system)
    sysm.xyz = sysm.xyz + np.array([3.25, -1.5, 0.75])
    st2 = Setup(sysm, wl.params)
    assert rel(far_K(st2, C), far_K(st, C)) < 1e-12


def test_atom_permutation(sheet):
    wl, C, st = sheet
    sysm = wl.system
    perm = np.random.default_rng(9).permutation(sysm.natoms)
    inv = np.argsort(perm)
    sp = [sysm.species[k] for k in perm]
    new = workloads._build("perm", sysm.xyz[perm], sp, sysm.nocc)
    # function index map old -> new
    def firsts(s):
        f = {}
        n = 0
        for sh in range(s.nshell):
            f.setdefault(int(s.shell_atom[sh]), []).extend(range(n, n + 2 * int(s.shell_l[sh]) + 1))
            n += 2 * int(s.shell_l[sh]) + 1
        return f
    fo, fnw = firsts(sysm), firsts(new)
    rowmap = np.zeros(sysm.nbasis, dtype=int)     # new function -> old function
    for a_new, a_old in enumerate(perm):
        for x, y in zip(fnw[a_new], fo[a_old]):
            rowmap[x] = y
    p = copy.copy(wl.params)
    st2 = Setup(new, p)
    K2 = far_K(st2, C[rowmap])
    assert rel(K2, far_K(st, C)[rowmap]) < 1e-12
    del inv


@pytest.mark.parametrize("which", ["chain", "sheet"])
def test_rank_truncated_m2l_equals_lower_lmax(which, tiny):
    """Interaction-list truncation to l, l' <= p (Eq. 12 at rank p) inside an
    L = 4 expansion equals the whole method run at lmax = p: M2M (Eq. 11) gives
    order l only from orders l' <= l, so the rank-p multipoles are the lmax = p
    ones; the truncated M2L leaves every local component above p at zero and
    L2L (Eq. 13) keeps them at zero, so L2P sees exactly the lmax = p locals."""
    if which == "chain":
        wl, C, _ = tiny
    else:
        wl = small_sheet(lmax=4, depth=3)
        C = wl.orbitals()
    st4 = Setup(wl.system, with_params(wl, lmax=4))
    for p in range(4):
        stp = Setup(wl.system, with_params(wl, lmax=p))
        Kp = far_K(stp, C)
        Kt = far_K(st4, C, m2l_rank=p)
        assert rel(Kt, Kp) < 1e-13, (which, p)
    # the truncation is not a no-op: rank 3 differs from the full rank 4
    assert rel(far_K(st4, C, m2l_rank=3), far_K(st4, C)) > 1e-6
