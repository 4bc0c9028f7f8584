"""Brute-force far-field exchange for s-type primitives (no multipole expansion).

For normalised s primitives (exponents a, b, c, d; p = a+b, q = c+d) the
two-electron integral has the textbook Boys-function closed form

  (ab|cd) = 2 pi^{5/2} / (p q sqrt(p+q)) K_ab K_cd N_a N_b N_c N_d F0(alpha R^2),
  K_ab = exp(-ab/p |A-B|^2),  alpha = pq/(p+q),  R = |P - Q|,
  F0(T) = (1/2) sqrt(pi/T) erf(sqrt(T)).

Its large-separation limit is the point-charge interaction S_ab S_cd / R,
which is exactly what the multipole expansion converges to as L grows.

  K^ff_ri = 2 sum_j sum_{(r,s) in B, (t,u) in B', B and B' far} (rs|tu) C_sj C_tj C_ui,

Eq. (1)/(5) restricted to the far leaf pairs of the tree (Setup.tree), and
likewise the far-field Coulomb matrix

  J^ff_rs = sum_{(t,u) in B', B and B' far} (rs|tu) D_tu   for (r,s) in B.
"""
from __future__ import annotations

import math

import numpy as np
from scipy.special import erf


def _boys_f0(T: np.ndarray) -> np.ndarray:
    Ts = np.where(T > 0, T, 1.0)
    return np.where(T > 1e-15, 0.5 * np.sqrt(math.pi / Ts) * erf(np.sqrt(Ts)), 1.0 - T / 3.0)


def eri_s(p, q, pref_ab, pref_cd, R):
    """(ab|cd) for normalised s primitives; pref = N_a N_b K_ab (broadcasts)."""
    alpha = p * q / (p + q)
    return (2 * math.pi ** 2.5 / (p * q * np.sqrt(p + q)) * pref_ab * pref_cd
            * _boys_f0(alpha * R * R))


def _far_pair_matrix(setup, kind: str) -> np.ndarray:
    """V[k, k'] = (r_k s_k | r_k' s_k') for far leaf pairs, 0 otherwise."""
    fn = setup.fn
    if np.any(fn.pow.sum(1) != 0):
        raise ValueError("s-type primitives only")
    r, s, P = setup.r, setup.s, setup.P
    a, b = fn.exp[r], fn.exp[s]
    p = a + b
    Kab = np.exp(-(a * b / p) * ((fn.center[r] - fn.center[s]) ** 2).sum(1))
    Nab = fn.norm[r] * fn.norm[s]
    S = Nab * Kab * (math.pi / p) ** 1.5
    t = setup.tree
    leaf = t.pair_leaf
    nl = setup.nleaf
    far = np.zeros((nl, nl), dtype=bool)
    for b1 in range(nl):
        for b2 in range(nl):
            far[b1, b2] = t.far_level(b1, b2) is not None
    pab = Nab * Kab
    V = np.empty((len(r), len(r)))
    for k0 in range(0, len(r), 512):
        k1 = min(len(r), k0 + 512)
        R = np.sqrt(((P[k0:k1, None, :] - P[None, :, :]) ** 2).sum(-1))
        if kind == "exact":
            blk = eri_s(p[k0:k1, None], p[None, :], pab[k0:k1, None], pab[None, :], R)
        elif kind == "pc":
            blk = S[k0:k1, None] * S[None, :] / np.where(R > 0, R, np.inf)
        else:
            raise ValueError(kind)
        V[k0:k1] = np.where(far[leaf[k0:k1, None], leaf[None, :]], blk, 0.0)
    return V


def far_J_exact_s(setup, Dm: np.ndarray, kind: str = "exact") -> np.ndarray:
    """J^ff (dense nbasis x nbasis, zero outside the pairs) by brute force;
    kind = 'exact' (Boys F0) or 'pc' (point charges)."""
    V = _far_pair_matrix(setup, kind)
    r, s = setup.r, setup.s
    J = np.zeros((setup.fn.n, setup.fn.n))
    J[r, s] = V @ Dm[r, s]
    return J


def far_K_exact_s(setup, C: np.ndarray, kind: str = "exact", i_range=None, j_range=None):
    """kind = 'exact' (Boys F0) or 'pc' (point charges S_ab S_cd / R)."""
    fn = setup.fn
    if np.any(fn.pow.sum(1) != 0):
        raise ValueError("s-type primitives only")
    nocc = C.shape[1]
    i0, i1 = (0, nocc) if i_range is None else i_range
    j0, j1 = (0, nocc) if j_range is None else j_range
    r, s, P = setup.r, setup.s, setup.P
    a, b = fn.exp[r], fn.exp[s]
    p = a + b
    Kab = np.exp(-(a * b / p) * ((fn.center[r] - fn.center[s]) ** 2).sum(1))
    Nab = fn.norm[r] * fn.norm[s]
    S = Nab * Kab * (math.pi / p) ** 1.5
    t = setup.tree
    leaf = t.pair_leaf
    nl = setup.nleaf
    far = np.zeros((nl, nl), dtype=bool)
    for b1 in range(nl):
        for b2 in range(nl):
            far[b1, b2] = t.far_level(b1, b2) is not None
    pab = Nab * Kab
    V = np.empty((len(r), len(r)))
    for k0 in range(0, len(r), 512):
        k1 = min(len(r), k0 + 512)
        R = np.sqrt(((P[k0:k1, None, :] - P[None, :, :]) ** 2).sum(-1))
        if kind == "exact":
            blk = eri_s(p[k0:k1, None], p[None, :], pab[k0:k1, None], pab[None, :], R)
        elif kind == "pc":
            blk = S[k0:k1, None] * S[None, :] / np.where(R > 0, R, np.inf)
        else:
            raise ValueError(kind)
        V[k0:k1] = np.where(far[leaf[k0:k1, None], leaf[None, :]], blk, 0.0)
    # Xm[(t,u), (j,i)] = C_tj C_ui over the pair list (t,u) = (r_k, s_k)
    Ct = C[r][:, j0:j1]
    Cu = C[s][:, i0:i1]          # C_ui
    Xm = np.einsum("kj,ki->kji", Ct, Cu).reshape(len(r), -1)
    Y = (V @ Xm).reshape(len(r), j1 - j0, i1 - i0)          # Y[(r,s), j, i]
    Cs = C[s][:, j0:j1]
    contrib = 2.0 * np.einsum("kj,kji->ki", Cs, Y)
    K = np.zeros((fn.n, i1 - i0))
    np.add.at(K, r, contrib)
    return K
