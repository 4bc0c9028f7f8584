"""Pins for the oracle's far-field Coulomb matrix J^ff (the Coulomb passage of
the Theory section, Eq. 10, through the same tree as K).

* Hierarchical translations == direct ancestor-centred sum (M2M and L2L are
  exact for truncated expansions), on the s-only chain and the s+p sheet.
* L = 0 reduces to monopoles: J_rs = S_rs sum_far S_tu D_tu / |Xa - Xb|.
* s-type chain: J_FMM(L) converges to the point-charge far field as L grows;
  the point-charge and the exact (Boys F0) far fields differ only by the
  Gaussian penetration term; at L = 10 (the paper's L^J) J_FMM matches the
  exact far field within that.
* One occupied orbital c with D = 2 c c^T: K^ff_r0 = sum_s J^ff_rs c_s, an
  identity between the exchange and Coulomb far fields (same pairs, same
  far partition), checked against the separately pinned far_K.
* J^ff is symmetric; it is linear in D.
"""
import numpy as np
import pytest

import workloads
from oracle.exact import far_J_exact_s
from oracle.fmm import Setup, far_J, far_J_direct, far_K

from conftest import rel, small_sheet, with_params


def _density(C):
    return 2.0 * C @ C.T


@pytest.fixture(scope="module")
def sheet3():
    wl = small_sheet(lmax=3, depth=3)
    return wl, wl.orbitals(), Setup(wl.system, wl.params)


def test_hierarchical_equals_direct_chain(tiny):
    wl, C, st = tiny
    Dm = _density(C)
    J = far_J(st, Dm)
    assert np.abs(J).max() > 0
    assert rel(J, far_J_direct(st, Dm)) < 1e-13


def test_hierarchical_equals_direct_sheet(sheet3):
    wl, C, st = sheet3
    assert st.tree.lmin < st.tree.depth
    Dm = _density(C)
    J, im = far_J(st, Dm, return_imag=True)
    assert rel(J, far_J_direct(st, Dm)) < 1e-12
    assert im < 1e-12 * np.abs(J).max()


def test_L0_is_monopole_sum(tiny):
    wl, C, st = tiny
    st0 = Setup(wl.system, with_params(wl, lmax=0))
    Dm = _density(C)
    J = far_J(st0, Dm)
    t = st0.tree
    S = workloads.overlap_matrix(wl.system)
    Jref = np.zeros_like(J)
    for b1 in range(st0.nleaf):
        for b2 in range(st0.nleaf):
            lev = t.far_level(b1, b2)
            if lev is None:
                continue
            Xa = t.centre(lev, t.boxes[lev][t.ancestor(lev, b1)])
            Xb = t.centre(lev, t.boxes[lev][t.ancestor(lev, b2)])
            k1, k2 = st0.leaf_pairs[b1], st0.leaf_pairs[b2]
            q = (S[st0.r[k2], st0.s[k2]] * Dm[st0.r[k2], st0.s[k2]]).sum()
            Jref[st0.r[k1], st0.s[k1]] += S[st0.r[k1], st0.s[k1]] * q / np.linalg.norm(Xa - Xb)
    assert rel(J, Jref) < 1e-12


@pytest.fixture(scope="module")
def chain_J_refs(tiny):
    wl, C, st = tiny
    Dm = _density(C)
    return Dm, far_J_exact_s(st, Dm, "exact"), far_J_exact_s(st, Dm, "pc")


@pytest.fixture(scope="module")
def chain_L10(tiny):
    wl, C, st = tiny
    return Setup(wl.system, with_params(wl, lmax=10))


def test_fmm_converges_to_point_charge_limit(tiny, chain_J_refs, chain_L10):
    wl, C, st = tiny
    Dm, Je, Jp = chain_J_refs
    errs = [rel(far_J(st if L == 2 else Setup(wl.system, with_params(wl, lmax=L)), Dm), Jp) for L in (2, 4, 6)]
    errs.append(rel(far_J(chain_L10, Dm), Jp))
    assert all(b < 0.1 * a for a, b in zip(errs, errs[1:])), errs
    assert errs[-1] < 1e-7


def test_fmm_at_LJ10_matches_exact_boys_far_field(tiny, chain_J_refs, chain_L10):
    wl, C, st = tiny
    Dm, Je, Jp = chain_J_refs
    pen = rel(Jp, Je)                      # Gaussian penetration: point charge vs exact
    assert pen < 1e-5
    J10 = far_J(chain_L10, Dm)
    assert rel(J10, Je) < 2 * pen + 1e-8
    assert rel(0.5 * J10, Je) > 0.4       # a dropped factor of the density is far outside


@pytest.mark.parametrize("which", ["chain", "sheet"])
def test_exchange_coulomb_identity_one_orbital(which, tiny, sheet3):
    """With one occupied orbital c and D = 2 c c^T, K^ff_r0 = sum_s J^ff_rs c_s."""
    wl, C, st = tiny if which == "chain" else sheet3
    for col in (0, C.shape[1] - 1):
        c = C[:, col:col + 1]
        K = far_K(st, c)
        J = far_J(st, _density(c))
        assert rel(J @ c, K) < 1e-12, (which, col)


def test_symmetric_and_linear(sheet3):
    wl, C, st = sheet3
    D1 = _density(C[:, :4])
    D2 = _density(C[:, 4:])
    J1, J2 = far_J(st, D1), far_J(st, D2)
    assert np.abs(J1 - J1.T).max() < 1e-12 * np.abs(J1).max()
    assert rel(far_J(st, D1 + 0.5 * D2), J1 + 0.5 * J2) < 1e-13
