"""Step-by-step occ-FMM-K far field, complex128 (Theory section, Eqs. 11-18).

Steps, in the paper's order:
  1. AO multipoles O^{rs,X} of every pair about the centre X of its leaf, Eq. (8).
  2. MO transforms, Eq. (15a,b):  O^{rj,X} = sum_s O^{rs,X} C_sj,
     O^{ij,X} = sum_r O^{rj,X} C_ri  (the occupied-pair multipole, "Omega").
  3. Upward pass, Eq. (17a) / (11):  O^{ij,Xp}_{lm} = sum O_{l-l',m-m'}(Xc-Xp) O^{ij,Xc}_{l'm'}.
  4. Interaction lists, Eq. (17b) / (12):
     Mloc^{ij}_{lm}(X) = (-1)^l sum M_{l+l',m+m'}(X-X') O^{ij,X'}_{l'm'}.
  5. Downward pass, Eq. (17c) / (13):  Mloc_{lm}(Xc) = sum Mloc_{l'm'}(Xp) O_{l'-l,m'-m}(Xc-Xp)
     (the printed M_{l'm'}(Xp) is read as the parent's local expansion).
  6. K^ff_ri = 2 sum_X sum_j sum_lm O^{rj,X}_{lm} Mloc^{ij}_{lm}(X), Eq. (18) with the
     factor 2 of Eq. (5) and the sum over leaf boxes X made explicit.

``pair_bound`` / ``pair_screen`` give the occupied-pair screening for
localised orbitals (the Conclusion's proposal): keep (i, j) when the bound
b_ij on sum_(t,u) K_tu |C_tj| |C_ui| over the screened pairs reaches the
threshold; ``band_ends`` / ``band_mask`` give the pairs a banded j-batch
schedule evaluates, and ``far_K(pair_mask=...)`` the far field of a pair set.

``far_J`` is the far-field Coulomb matrix through the same tree and
translations, with one density-contracted column (the Coulomb passage of the
Theory section, Eq. 10).

Truncation: l <= L and l' <= L everywhere (the irregular harmonics are
therefore needed to 2L).  Optional i and j ranges restrict the output
columns and the summed occupied index.

``far_K_direct`` evaluates the same truncated quantity without translations:
for every far leaf pair it expands both pairs about the centres of the
ancestors whose interaction lists contain each other and applies the M2L
kernel once.  M2M is exact for multipoles truncated at L and L2L is an exact
re-centring of a degree-L polynomial, so both must agree to rounding.
"""
from __future__ import annotations

import numpy as np
from scipy import sparse
from scipy.special import erfcinv

from . import harmonics as H
from .basis import Functions, ao_multipoles, function_pairs
from .tree import Tree


def m2m_matrix(L: int, d: np.ndarray) -> np.ndarray:
    """T[lm, l'm'] = O_{l-l', m-m'}(d), d = Xc - Xp (Eq. 11)."""
    Od = H.regular(L, d)
    Q = H.ncomp(L)
    T = np.zeros((Q, Q), dtype=np.complex128)
    for l in range(L + 1):
        for m in range(-l, l + 1):
            for lp in range(l + 1):
                for mp in range(-lp, lp + 1):
                    if abs(m - mp) <= l - lp:
                        T[H.idx(l, m), H.idx(lp, mp)] = Od[H.idx(l - lp, m - mp)]
    return T


def m2l_matrix(L: int, R: np.ndarray) -> np.ndarray:
    """T[lm, l'm'] = (-1)^l M_{l+l', m+m'}(R), R = X - X' (Eq. 12)."""
    MR = H.irregular(2 * L, R)
    Q = H.ncomp(L)
    T = np.zeros((Q, Q), dtype=np.complex128)
    for l in range(L + 1):
        for m in range(-l, l + 1):
            for lp in range(L + 1):
                for mp in range(-lp, lp + 1):
                    T[H.idx(l, m), H.idx(lp, mp)] = (-1) ** l * MR[H.idx(l + lp, m + mp)]
    return T


def l2l_matrix(L: int, d: np.ndarray) -> np.ndarray:
    """T[lm, l'm'] = O_{l'-l, m'-m}(d), d = Xc - Xp (Eq. 13)."""
    Od = H.regular(L, d)
    Q = H.ncomp(L)
    T = np.zeros((Q, Q), dtype=np.complex128)
    for l in range(L + 1):
        for m in range(-l, l + 1):
            for lp in range(l, L + 1):
                for mp in range(-lp, lp + 1):
                    if abs(mp - m) <= lp - l:
                        T[H.idx(l, m), H.idx(lp, mp)] = Od[H.idx(lp - l, mp - m)]
    return T


def _leaf_multipoles(args):
    fn, r, s, X, L, nquad = args
    return ao_multipoles(fn, r, s, X, L, nquad)


class Setup:
    """Step 1: pairs, tree and the leaf AO multipoles (per geometry).

    workers > 1 evaluates the leaves' multipole integrals in that many
    processes; each leaf's integrals are the same computation either way."""

    def __init__(self, system, params, nquad: int | None = None, workers: int = 1):
        self.system, self.params = system, params
        self.L = int(params.lmax)
        self.fn = Functions(system)
        self.r, self.s, self.P = function_pairs(system, self.fn, params.pair_log_thresh)
        if getattr(params, "near_rule", 0) == 1:
            # extent of a pair distribution of exponent p = a + b: erfc^-1(tau) / sqrt(p)
            pe = self.fn.exp[self.r] + self.fn.exp[self.s]
            ext = erfcinv(params.ext_tau) / np.sqrt(pe)
            self.tree = Tree(self.P, params.split_mask, params.depth, params.ext_ws, extents=ext)
        else:
            self.tree = Tree(self.P, params.split_mask, params.depth, params.ws)
        t = self.tree
        self.nleaf = len(t.boxes[t.depth])
        self.leaf_pairs = [np.nonzero(t.pair_leaf == b)[0] for b in range(self.nleaf)]
        jobs = [(self.fn, self.r[k], self.s[k], t.centre(t.depth, t.boxes[t.depth][b]), self.L, nquad)
                for b, k in enumerate(self.leaf_pairs)]
        if workers > 1:
            import multiprocessing as mp
            with mp.get_context("fork").Pool(workers) as pool:
                mps = pool.map(_leaf_multipoles, jobs, chunksize=1)
        else:
            mps = map(_leaf_multipoles, jobs)
        # per leaf: its sorted functions, the local (row, column) of each of
        # its pairs and the pairs' multipoles (npairs_B, Q)
        self.leaf_funcs, self.leaf_ra, self.leaf_sa, self.leaf_pm = [], [], [], []
        for b, om in enumerate(mps):
            k = self.leaf_pairs[b]
            f = np.unique(np.concatenate([self.r[k], self.s[k]]))
            self.leaf_funcs.append(f)
            self.leaf_ra.append(np.searchsorted(f, self.r[k]))
            self.leaf_sa.append(np.searchsorted(f, self.s[k]))
            self.leaf_pm.append(om)

    def dense_block(self, b: int) -> np.ndarray:
        """O^{rs,X}_q of leaf b as a dense (Q, nb, nb) block over its functions
        (zero where (r, s) is not one of the leaf's pairs)."""
        nb = len(self.leaf_funcs[b])
        dense = np.zeros((nb, nb, self.leaf_pm[b].shape[1]), dtype=np.complex128)
        np.add.at(dense, (self.leaf_ra[b], self.leaf_sa[b]), self.leaf_pm[b])
        return np.ascontiguousarray(dense.transpose(2, 0, 1))

    def half(self, b: int, Cj: np.ndarray) -> np.ndarray:
        """Eq. (15a) in leaf b: O^{rj}_q = sum_s O^{rs}_q C_sj, the s-sum running
        over the pairs (r, s) assigned to b.  Cj: (nbasis, nj) -> (Q, nb, nj)."""
        f = self.leaf_funcs[b]
        om, ra, sa = self.leaf_pm[b], self.leaf_ra[b], self.leaf_sa[b]
        CB = Cj[f]
        out = np.empty((om.shape[1], len(f), Cj.shape[1]), dtype=np.complex128)
        for q in range(om.shape[1]):
            out[q] = sparse.csr_matrix((om[:, q], (ra, sa)), shape=(len(f), len(f))) @ CB
        return out

    @property
    def nbasis(self) -> int:
        return self.fn.n


def _ranges(nocc, i_range, j_range):
    i0, i1 = (0, nocc) if i_range is None else i_range
    j0, j1 = (0, nocc) if j_range is None else j_range
    return i0, i1, j0, j1


def truncate(T: np.ndarray, p: int) -> np.ndarray:
    """Rank-p truncation of a square translation: only l <= p and l' <= p kept."""
    n = (p + 1) * (p + 1)
    out = np.zeros_like(T)
    out[:n, :n] = T[:n, :n]
    return out


def _operators(setup: Setup, m2l_rank=None):
    """Translation matrices of the tree: M2M (Eq. 11) and L2L (Eq. 13) per
    child box, M2L (Eq. 12) per interaction-list pair, optionally truncated."""
    t, L, D = setup.tree, setup.L, setup.tree.depth
    up = {}
    for lev in range(t.lmin + 1, D + 1):
        for b, c in enumerate(t.boxes[lev]):
            p = t.parent(lev, b)
            up[(lev, b)] = m2m_matrix(L, t.centre(lev, c) - t.centre(lev - 1, t.boxes[lev - 1][p]))
    down = {k: None for k in up}
    for (lev, b) in up:
        c = t.boxes[lev][b]
        p = t.parent(lev, b)
        down[(lev, b)] = l2l_matrix(L, t.centre(lev, c) - t.centre(lev - 1, t.boxes[lev - 1][p]))
    m2l = {}
    for lev in range(t.lmin, D + 1):
        for b, c in enumerate(t.boxes[lev]):
            for b2 in t.il[lev][b]:
                T = m2l_matrix(L, t.centre(lev, c) - t.centre(lev, t.boxes[lev][b2]))
                m2l[(lev, b, b2)] = T if m2l_rank is None else truncate(T, int(m2l_rank))
    return up, down, m2l


def far_J(setup: Setup, Dm: np.ndarray, return_imag: bool = False):
    """Far-field Coulomb matrix J^ff_rs = sum_lm O^{rs,X}_lm Mloc_lm(X) (Theory
    section, the Coulomb passage with Eq. 10), for the pairs (r, s) of every
    leaf X; dense (nbasis, nbasis), zero outside the screened pairs.

    Steps: density-contracted multipoles of each leaf,
    O^X_lm = sum_{(t,u) in X} D_tu O^{tu,X}_lm; upward translations (Eq. 11);
    interaction lists (Eq. 12, i.e. Eq. 10 summed hierarchically); downward
    translations (Eq. 13); the contraction with each pair's multipoles."""
    t = setup.tree
    n = setup.nbasis
    J = np.zeros((n, n), dtype=np.complex128)
    if t.lmin is None:
        return (J.real, 0.0) if return_imag else J.real
    D = t.depth
    up, down, m2l = _operators(setup)
    Om = {D: [setup.leaf_pm[b].T @ Dm[setup.r[k], setup.s[k]] for b, k in enumerate(setup.leaf_pairs)]}
    for lev in range(D - 1, t.lmin - 1, -1):
        acc = [np.zeros_like(Om[D][0]) for _ in t.boxes[lev]]
        for b in range(len(t.boxes[lev + 1])):
            acc[t.parent(lev + 1, b)] += up[(lev + 1, b)] @ Om[lev + 1][b]
        Om[lev] = acc
    Ml = {}
    for lev in range(t.lmin, D + 1):
        cur = []
        for b in range(len(t.boxes[lev])):
            acc = np.zeros_like(Om[D][0])
            for b2 in t.il[lev][b]:
                acc += m2l[(lev, b, b2)] @ Om[lev][b2]
            if lev > t.lmin:
                acc += down[(lev, b)] @ Ml[lev - 1][t.parent(lev, b)]
            cur.append(acc)
        Ml[lev] = cur
    for b, k in enumerate(setup.leaf_pairs):
        J[setup.r[k], setup.s[k]] += setup.leaf_pm[b] @ Ml[D][b]
    if return_imag:
        return J.real, float(np.abs(J.imag).max())
    return J.real


def far_J_direct(setup: Setup, Dm: np.ndarray, nquad=None):
    """The same truncated J^ff from ancestor-centred expansions, one M2L per
    far leaf pair (no translations)."""
    t, L = setup.tree, setup.L
    n = setup.nbasis
    J = np.zeros((n, n), dtype=np.complex128)
    if t.lmin is None:
        return J.real
    cache = {}

    def mult(leaf, lev):   # pair multipoles of a leaf about its level-lev ancestor's centre
        if (leaf, lev) not in cache:
            X = t.centre(lev, t.boxes[lev][t.ancestor(lev, leaf)])
            k = setup.leaf_pairs[leaf]
            cache[(leaf, lev)] = (ao_multipoles(setup.fn, setup.r[k], setup.s[k], X, L, nquad), X)
        return cache[(leaf, lev)]

    for b1 in range(setup.nleaf):
        for b2 in range(setup.nleaf):
            lev = t.far_level(b1, b2)
            if lev is None:
                continue
            O1, X1 = mult(b1, lev)
            O2, X2 = mult(b2, lev)
            k1, k2 = setup.leaf_pairs[b1], setup.leaf_pairs[b2]
            om = O2.T @ Dm[setup.r[k2], setup.s[k2]]
            J[setup.r[k1], setup.s[k1]] += O1 @ (m2l_matrix(L, X1 - X2) @ om)
    return J.real


def far_K(setup: Setup, C: np.ndarray, i_range=None, j_range=None, jblock: int = 64,
          return_imag: bool = False, m2l_rank=None, pair_mask=None):
    """K^ff[:, i0:i1] = 2 sum_{j in [j0,j1)} (rj|ji)_ff by the hierarchical FMM.

    m2l_rank: optional int p (0 <= p <= L) applied to every interaction-list
    translation (l, l' <= p), the uniform version of a per-interaction rank.
    pair_mask: optional boolean (nocc, nocc) array, symmetric: only the
    occupied pairs (i, j) it keeps contribute (occupied-pair screening; the
    pair's multipoles, and so everything translated from them, are dropped)."""
    t, L = setup.tree, setup.L
    nocc = C.shape[1]
    i0, i1, j0, j1 = _ranges(nocc, i_range, j_range)
    K = np.zeros((setup.nbasis, i1 - i0), dtype=np.complex128)
    if t.lmin is None or j1 <= j0 or i1 <= i0:
        return (K.real, 0.0) if return_imag else K.real
    D = t.depth
    up, down, m2l = _operators(setup, m2l_rank)
    for jb0 in range(j0, j1, jblock):
        jb1 = min(j1, jb0 + jblock)
        # Step 2: MO transforms at the leaves
        Hb, Om = [], {D: []}
        for b in range(setup.nleaf):
            h = setup.half(b, C[:, jb0:jb1])                                     # O^{rj}_q = O^{rs}_q C_sj
            Hb.append(h)
            om = np.matmul(C[setup.leaf_funcs[b], i0:i1].T, h)                   # O^{ij}_q = sum_r C_ri O^{rj}_q
            if pair_mask is not None:
                om = om * pair_mask[i0:i1, jb0:jb1][None]
            Om[D].append(om)
        # Step 3: upward
        for lev in range(D - 1, t.lmin - 1, -1):
            acc = [np.zeros_like(Om[D][0]) for _ in t.boxes[lev]]
            for b in range(len(t.boxes[lev + 1])):
                p = t.parent(lev + 1, b)
                acc[p] += np.tensordot(up[(lev + 1, b)], Om[lev + 1][b], axes=(1, 0))
            Om[lev] = acc
        # Steps 4-5: interaction lists and downward
        Ml = {}
        for lev in range(t.lmin, D + 1):
            cur = []
            for b in range(len(t.boxes[lev])):
                acc = np.zeros_like(Om[D][0])
                for b2 in t.il[lev][b]:
                    acc += np.tensordot(m2l[(lev, b, b2)], Om[lev][b2], axes=(1, 0))
                if lev > t.lmin:
                    p = t.parent(lev, b)
                    acc += np.tensordot(down[(lev, b)], Ml[lev - 1][p], axes=(1, 0))
                cur.append(acc)
            Ml[lev] = cur
        # Step 6: K^ff
        for b in range(setup.nleaf):
            # sum_j sum_q O^{rj}_q Mloc^{ij}_q
            K[setup.leaf_funcs[b]] += 2.0 * np.matmul(Hb[b], Ml[D][b].transpose(0, 2, 1)).sum(0)
    if return_imag:
        return K.real, float(np.abs(K.imag).max())
    return K.real


def pair_bound(setup: Setup, C: np.ndarray) -> np.ndarray:
    """Bound b_ij for occupied-pair screening with localised orbitals
    (Conclusion: localised orbitals and the screening of occupied pairs).

    Every function has a home leaf, the leaf holding its centre (that of its
    pair with itself).  With n_Ai = sum of |C_ti| over the functions t of home
    leaf A, and W_AA' = the largest Gaussian product factor
    K_tu = exp(-a_t a_u / (a_t + a_u) |A_t - A_u|^2) over the screened pairs
    (t, u) with t at home in A and u in A',

        b_ij = sum_(A, A') n_Aj W_AA' n_A'i  >=  sum_(t,u) K_tu |C_tj| |C_ui|,

    the sum on the right running over the screened pairs."""
    fn, r, s = setup.fn, setup.r, setup.s
    nl = setup.nleaf
    home = np.full(setup.nbasis, -1, dtype=np.int64)
    self_pair = r == s
    home[r[self_pair]] = setup.tree.pair_leaf[self_pair]
    if (home < 0).any():
        raise ValueError("a function without its pair with itself")
    a, b = fn.exp[r], fn.exp[s]
    Ktu = np.exp(-(a * b / (a + b)) * ((fn.center[r] - fn.center[s]) ** 2).sum(1))
    W = np.zeros((nl, nl))
    np.maximum.at(W, (home[r], home[s]), Ktu)
    N = np.zeros((nl, C.shape[1]))
    np.add.at(N, home, np.abs(C))
    return N.T @ W @ N          # [j, i]


def pair_screen(setup: Setup, C: np.ndarray, thresh: float) -> np.ndarray:
    """Occupied-pair mask: (i, j) kept when b_ij >= thresh or b_ji >= thresh
    (pair_bound)."""
    B = pair_bound(setup, C)
    return (B >= thresh) | (B.T >= thresh)


def band_ends(setup: Setup, C: np.ndarray, thresh: float, jblock: int) -> np.ndarray:
    """i end (exclusive) of every j batch of a banded schedule: batch k,
    j in [k jblock, (k+1) jblock), carries every i below one past the last
    i > j whose pair bound b_ji (pair_bound) reaches thresh, and at least
    up to its own last j."""
    B = pair_bound(setup, C)
    n = C.shape[1]
    ends = []
    for j0 in range(0, n, jblock):
        j1 = min(n, j0 + jblock)
        e = j1
        for j in range(j0, j1):
            kept = np.nonzero(B[j, j + 1:] >= thresh)[0]
            if kept.size:
                e = max(e, j + 1 + int(kept[-1]) + 1)
        ends.append(e)
    return np.array(ends, dtype=np.int64)


def band_mask(nocc: int, jblock: int, band_end) -> np.ndarray:
    """The (i, j) pairs a banded schedule evaluates: j batch k = [k jblock,
    (k+1) jblock) carries i < band_end[k], and the pair (i, j) is evaluated
    once, by the batch of min(i, j)."""
    m = np.zeros((nocc, nocc), dtype=bool)
    for k, e in enumerate(band_end):
        j0, j1 = k * jblock, min(nocc, (k + 1) * jblock)
        m[j0:j1, j0:int(e)] = True
    return m | m.T


def far_K_direct(setup: Setup, C: np.ndarray, i_range=None, j_range=None, nquad=None):
    """Same truncated K^ff from ancestor-centred expansions, one M2L per far leaf pair."""
    t, L = setup.tree, setup.L
    nocc = C.shape[1]
    i0, i1, j0, j1 = _ranges(nocc, i_range, j_range)
    K = np.zeros((setup.nbasis, i1 - i0), dtype=np.complex128)
    if t.lmin is None:
        return K.real
    D = t.depth
    cache = {}

    def mult(leaf, lev):
        key = (leaf, lev)
        if key not in cache:
            a = t.ancestor(lev, leaf)
            X = t.centre(lev, t.boxes[lev][a])
            k = setup.leaf_pairs[leaf]
            f = setup.leaf_funcs[leaf]
            loc = {int(v): n for n, v in enumerate(f)}
            om = ao_multipoles(setup.fn, setup.r[k], setup.s[k], X, L, nquad)
            dense = np.zeros((len(f), len(f), H.ncomp(L)), dtype=np.complex128)
            np.add.at(dense, (np.searchsorted(f, setup.r[k]), np.searchsorted(f, setup.s[k])), om)
            dense = np.ascontiguousarray(dense.transpose(2, 0, 1))
            del loc
            cache[key] = (dense, X)
        return cache[key]

    for b1 in range(setup.nleaf):
        for b2 in range(setup.nleaf):
            lev = t.far_level(b1, b2)
            if lev is None:
                continue
            O1, X1 = mult(b1, lev)
            O2, X2 = mult(b2, lev)
            C1, C2 = C[setup.leaf_funcs[b1]], C[setup.leaf_funcs[b2]]
            h = np.einsum("qrs,sj->qrj", O1, C1[:, j0:j1])
            om = np.einsum("ui,qtu->qti", C2[:, i0:i1], O2)
            om = np.einsum("qti,tj->qij", om, C2[:, j0:j1])
            T = m2l_matrix(L, X1 - X2)
            Mloc = np.tensordot(T, om, axes=(1, 0))                         # (q, i, j)
            K[setup.leaf_funcs[b1]] += 2.0 * np.einsum("qrj,qij->ri", h, Mloc)
    return K.real
