"""Exact two-electron repulsion integrals over normalised s/p Cartesian
primitives, and the near-field part of the occupied exchange.

TEST INFRASTRUCTURE ONLY (see the package docstring).

  (rs|tu) = integral phi_r(1) phi_s(1) 1/r12 phi_t(2) phi_u(2)      (Introduction, the ERI definition)

computed with the Obara-Saika recurrences (vertical recurrence on the bra
and ket angular momentum from [00|00]^(m), then the horizontal transfer
(a, b+1_i| = (a+1_i, b| + (A_i - B_i)(a, b| on both sides) for unnormalised
Cartesian Gaussians, times the functions' normalisation.  The Boys function
is F_m(T) = Gamma(m+1/2) P(m+1/2, T) / (2 T^(m+1/2)) with the regularised
lower incomplete gamma P of scipy, and 1/(2m+1) - T/(2m+3) + ... at T -> 0.

Near field (the Theory section: the pairs of distributions whose leaf boxes
are near, where the multipole expansion is not used):

  K^nf_ri = 2 sum_j sum_{(r,s) in B, (t,u) in B', B near B'} (rs|tu) C_sj C_tj C_ui

with B, B' leaves that are near (the leaf-level near relation of the tree,
B = B' included); together with K^ff it gives the whole exchange.
"""
from __future__ import annotations

import math

import numpy as np
from scipy.special import gamma, gammainc


def boys(m: int, T: np.ndarray) -> np.ndarray:
    T = np.asarray(T, dtype=np.float64)
    small = T < 1e-10
    Ts = np.where(small, 1.0, T)
    a = m + 0.5
    big = gamma(a) * gammainc(a, Ts) / (2.0 * Ts ** a)
    series = 1.0 / (2 * m + 1) - T / (2 * m + 3) + T * T / (2.0 * (2 * m + 5))
    return np.where(small, series, big)


def _unit(i: int):
    e = [0, 0, 0]
    e[i] = 1
    return tuple(e)


def _sub(v, i):
    w = list(v)
    w[i] -= 1
    return tuple(w)


def _add(v, i):
    w = list(v)
    w[i] += 1
    return tuple(w)


class _Quartets:
    """Obara-Saika recurrences, vectorised over N primitive quartets that share
    their Cartesian powers."""

    def __init__(self, A, a, B, b, C, c, D, d):
        self.A, self.B, self.C, self.D = A, B, C, D
        z, e = a + b, c + d
        self.z, self.e = z, e
        self.P = (a[:, None] * A + b[:, None] * B) / z[:, None]
        self.Q = (c[:, None] * C + d[:, None] * D) / e[:, None]
        self.W = (z[:, None] * self.P + e[:, None] * self.Q) / (z + e)[:, None]
        self.rho = z * e / (z + e)
        Kab = np.exp(-(a * b / z) * ((A - B) ** 2).sum(1))
        Kcd = np.exp(-(c * d / e) * ((C - D) ** 2).sum(1))
        self.T = self.rho * ((self.P - self.Q) ** 2).sum(1)
        self.pre = 2.0 * math.pi ** 2.5 / (z * e * np.sqrt(z + e)) * Kab * Kcd
        self.memo = {}

    def vrr(self, ea, ec, m):
        """[ea 0 | ec 0]^(m)."""
        key = (ea, ec, m)
        if key in self.memo:
            return self.memo[key]
        if any(v < 0 for v in ea + ec):
            out = 0.0
        elif sum(ea) == 0 and sum(ec) == 0:
            out = self.pre * boys(m, self.T)
        elif sum(ea) > 0:
            i = next(k for k in range(3) if ea[k] > 0)
            e1 = _sub(ea, i)
            z, e = self.z, self.e
            out = ((self.P[:, i] - self.A[:, i]) * self.vrr(e1, ec, m)
                   + (self.W[:, i] - self.P[:, i]) * self.vrr(e1, ec, m + 1))
            if e1[i] > 0:
                e2 = _sub(e1, i)
                out = out + e1[i] / (2 * z) * (self.vrr(e2, ec, m) - self.rho / z * self.vrr(e2, ec, m + 1))
            if ec[i] > 0:
                out = out + ec[i] / (2 * (z + e)) * self.vrr(e1, _sub(ec, i), m + 1)
        else:
            i = next(k for k in range(3) if ec[k] > 0)
            c1 = _sub(ec, i)
            z, e = self.z, self.e
            out = ((self.Q[:, i] - self.C[:, i]) * self.vrr(ea, c1, m)
                   + (self.W[:, i] - self.Q[:, i]) * self.vrr(ea, c1, m + 1))
            if c1[i] > 0:
                c2 = _sub(c1, i)
                out = out + c1[i] / (2 * e) * (self.vrr(ea, c2, m) - self.rho / e * self.vrr(ea, c2, m + 1))
            if ea[i] > 0:
                out = out + ea[i] / (2 * (z + e)) * self.vrr(_sub(ea, i), c1, m + 1)
        self.memo[key] = out
        return out

    def ket(self, ea, ec, ed):
        """[ea 0 | ec ed] by the horizontal transfer on the ket."""
        if sum(ed) == 0:
            return self.vrr(ea, ec, 0)
        i = next(k for k in range(3) if ed[k] > 0)
        d1 = _sub(ed, i)
        return self.ket(ea, _add(ec, i), d1) + (self.C[:, i] - self.D[:, i]) * self.ket(ea, ec, d1)

    def eri(self, ea, eb, ec, ed):
        """(ea eb | ec ed) by the horizontal transfer on the bra."""
        if sum(eb) == 0:
            return self.ket(ea, ec, ed)
        i = next(k for k in range(3) if eb[k] > 0)
        b1 = _sub(eb, i)
        return self.eri(_add(ea, i), b1, ec, ed) + (self.A[:, i] - self.B[:, i]) * self.eri(ea, b1, ec, ed)


def eri(fn, r, s, t, u) -> np.ndarray:
    """(r_k s_k | t_k u_k) for arrays of function indices (normalised functions)."""
    r, s, t, u = (np.atleast_1d(np.asarray(x, dtype=np.int64)) for x in (r, s, t, u))
    out = np.empty(len(r))
    pw = fn.pow
    key = np.stack([pw[r] @ [1, 2, 4], pw[s] @ [1, 2, 4], pw[t] @ [1, 2, 4], pw[u] @ [1, 2, 4]], 1)
    for kk in np.unique(key, axis=0):
        sel = np.nonzero((key == kk).all(1))[0]
        for c0 in range(0, len(sel), 200000):
            idx = sel[c0:c0 + 200000]
            q = _Quartets(fn.center[r[idx]], fn.exp[r[idx]], fn.center[s[idx]], fn.exp[s[idx]],
                          fn.center[t[idx]], fn.exp[t[idx]], fn.center[u[idx]], fn.exp[u[idx]])
            val = q.eri(tuple(pw[r[idx[0]]]), tuple(pw[s[idx[0]]]), tuple(pw[t[idx[0]]]), tuple(pw[u[idx[0]]]))
            out[idx] = val * fn.norm[r[idx]] * fn.norm[s[idx]] * fn.norm[t[idx]] * fn.norm[u[idx]]
    return out


def near_K(setup, C: np.ndarray, i_range=None, j_range=None) -> np.ndarray:
    """K^nf[:, i0:i1] = 2 sum_{j in [j0,j1)} sum over near leaf pairs of
    (rs|tu) C_sj C_tj C_ui, with exact integrals."""
    t = setup.tree
    nocc = C.shape[1]
    i0, i1 = (0, nocc) if i_range is None else i_range
    j0, j1 = (0, nocc) if j_range is None else j_range
    K = np.zeros((setup.nbasis, i1 - i0))
    r, s = setup.r, setup.s
    for b1 in range(setup.nleaf):
        k1 = setup.leaf_pairs[b1]
        for b2 in t.near_leaves(b1):
            k2 = setup.leaf_pairs[b2]
            R, T = np.meshgrid(k1, k2, indexing="ij")
            V = eri(setup.fn, r[R.ravel()], s[R.ravel()], r[T.ravel()], s[T.ravel()]).reshape(len(k1), len(k2))
            X = np.einsum("kj,ki->kji", C[r[k2], j0:j1], C[s[k2], i0:i1]).reshape(len(k2), -1)
            Y = (V @ X).reshape(len(k1), j1 - j0, i1 - i0)
            np.add.at(K, r[k1], 2.0 * np.einsum("kj,kji->ki", C[s[k1], j0:j1], Y))
    return K


def near_K_rows(setup, C: np.ndarray, rows) -> np.ndarray:
    """Rows r of K^nf (all i, all j): only the pairs (r, s) with that r and the
    pairs of the leaves near theirs; for sampling a large system."""
    t = setup.tree
    r_all, s_all = setup.r, setup.s
    out = np.zeros((len(rows), C.shape[1]))
    for n, rr in enumerate(rows):
        k1_all = np.nonzero(r_all == rr)[0]
        for b1 in np.unique(t.pair_leaf[k1_all]):
            k1 = k1_all[t.pair_leaf[k1_all] == b1]
            for b2 in t.near_leaves(int(b1)):
                k2 = setup.leaf_pairs[b2]
                R, T = np.meshgrid(k1, k2, indexing="ij")
                V = eri(setup.fn, r_all[R.ravel()], s_all[R.ravel()], r_all[T.ravel()],
                        s_all[T.ravel()]).reshape(len(k1), len(k2))
                # sum_j C_sj sum_(t,u) V C_tj C_ui
                W = V.T @ C[s_all[k1]]                       # (k2, j)
                out[n] += 2.0 * np.einsum("kj,kj,ki->i", W, C[r_all[k2]], C[s_all[k2]])
    return out


def all_K(setup, C: np.ndarray) -> np.ndarray:
    """The whole exchange K_ri = 2 sum_j (rj|ji) with exact integrals over
    every pair of screened distributions (no tree; for small systems)."""
    r, s = setup.r, setup.s
    n = len(r)
    K = np.zeros((setup.nbasis, C.shape[1]))
    for k0 in range(0, n, 512):
        kk = np.arange(k0, min(n, k0 + 512))
        R, T = np.meshgrid(kk, np.arange(n), indexing="ij")
        V = eri(setup.fn, r[R.ravel()], s[R.ravel()], r[T.ravel()], s[T.ravel()]).reshape(len(kk), n)
        # sum_j sum_(t,u) V (C_sj C_tj C_ui)
        X = np.einsum("kj,ki->kji", C[r], C[s]).reshape(n, -1)
        Y = (V @ X).reshape(len(kk), C.shape[1], C.shape[1])
        np.add.at(K, r[kk], 2.0 * np.einsum("kj,kji->ki", C[s[kk]], Y))
    return K
