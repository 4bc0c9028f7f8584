"""Basis functions, screened AO pairs and AO multipole integrals, Eq. (8).

  O^{rs,X}_{l,m} = integral phi_r(r) O_{l,m}(r - X) phi_s(r) d^3r

Basis: normalised uncontracted Cartesian primitives, s and p (x, y, z).  The
product of two Gaussians is a Gaussian of exponent p = a + b centred at
P = (aA + bB)/p times exp(-ab/p |A-B|^2) (Gaussian product theorem), so

  integral f(r) exp(-p|r-P|^2) d^3r = p^{-3/2} sum_{ijk} w_i w_j w_k f(P + t_ijk/sqrt(p))

with tensor-product Gauss-Hermite nodes t and weights w.  The integrand's
polynomial part has degree <= L + 2 in each coordinate, so n >= (L+3)/2 nodes
per dimension integrate it exactly.

Pairs: every ordered pair of shells (A, a), (B, b) with
(ab/(a+b)) |A-B|^2 <= pair_log_thresh is kept (prefactor >= e^-thresh); all
function pairs of a kept shell pair share the centre P, which is the pair's
position for box assignment (the expansion centre is the box centre, Theory
section).
"""
from __future__ import annotations

import math

import numpy as np

from . import harmonics as H


class Functions:
    """Per-function arrays built from a workloads.System-like object."""

    def __init__(self, system):
        cen, ex, pw, shell = [], [], [], []
        for s in range(len(system.shell_l)):
            A = np.asarray(system.xyz[system.shell_atom[s]], dtype=np.float64)
            comps = [(0, 0, 0)] if system.shell_l[s] == 0 else [(1, 0, 0), (0, 1, 0), (0, 0, 1)]
            for c in comps:
                cen.append(A)
                ex.append(float(system.shell_exp[s]))
                pw.append(c)
                shell.append(s)
        self.center = np.array(cen)
        self.exp = np.array(ex)
        self.pow = np.array(pw, dtype=np.int64)
        self.shell = np.array(shell, dtype=np.int64)
        lsum = self.pow.sum(1)
        # normalisation of x^i y^j z^k exp(-a r^2) for total degree 0 or 1
        self.norm = (2 * self.exp / math.pi) ** 0.75 * np.where(lsum == 1, 2 * np.sqrt(self.exp), 1.0)
        self.n = len(self.exp)


def shell_pairs(system, thresh: float):
    """Ordered shell pairs kept by the screening rule; raises on a near-tie."""
    xyz = np.asarray(system.xyz, dtype=np.float64)
    A = xyz[system.shell_atom]
    a = np.asarray(system.shell_exp, dtype=np.float64)
    mu = a[:, None] * a[None, :] / (a[:, None] + a[None, :])
    d2 = ((A[:, None, :] - A[None, :, :]) ** 2).sum(-1)
    val = mu * d2
    if math.isfinite(thresh):
        close = np.abs(val - thresh) <= 1e-9 * thresh
        if np.any(close):
            raise ValueError("pair screening value within 1e-9 of the threshold")
        keep = val <= thresh
    else:
        keep = np.ones_like(val, dtype=bool)
    s1, s2 = np.nonzero(keep)
    return s1, s2


def function_pairs(system, fn: Functions, thresh: float):
    """(r, s, P) for every ordered function pair of every kept shell pair, in
    the order (shell pair, function of the first shell, function of the second)."""
    s1, s2 = shell_pairs(system, thresh)
    nf = 2 * np.asarray(system.shell_l, dtype=np.int64) + 1
    first = np.zeros(len(nf) + 1, dtype=np.int64)
    first[1:] = np.cumsum(nf)
    na, nb = nf[s1], nf[s2]
    cnt = na * nb
    start = np.repeat(np.cumsum(cnt) - cnt, cnt)
    k = np.arange(int(cnt.sum()), dtype=np.int64) - start       # index inside the shell pair
    nbr = np.repeat(nb, cnt)
    r = np.repeat(first[s1], cnt) + k // nbr
    s = np.repeat(first[s2], cnt) + k % nbr
    ea, eb = fn.exp[r], fn.exp[s]
    P = (ea[:, None] * fn.center[r] + eb[:, None] * fn.center[s]) / (ea + eb)[:, None]
    return r, s, P


def ao_multipoles(fn: Functions, r: np.ndarray, s: np.ndarray, X: np.ndarray, L: int,
                  nquad: int | None = None, points_per_chunk: int = 100000) -> np.ndarray:
    """O^{rs,X}_{lm} for function pairs (r[k], s[k]) about centres X[k] (k, 3).

    Returns complex (npairs, (L+1)^2).
    """
    n = (L + 4) // 2 if nquad is None else nquad
    t, w = np.polynomial.hermite.hermgauss(n)
    T = np.stack(np.meshgrid(t, t, t, indexing="ij"), -1).reshape(-1, 3)
    Wt = np.einsum("i,j,k->ijk", w, w, w).reshape(-1)
    out = np.zeros((len(r), H.ncomp(L)), dtype=np.complex128)
    chunk = max(1, points_per_chunk // len(Wt))
    X = np.broadcast_to(np.asarray(X, dtype=np.float64), (len(r), 3))
    for k0 in range(0, len(r), chunk):
        k1 = min(len(r), k0 + chunk)
        rr, ss = r[k0:k1], s[k0:k1]
        a, b = fn.exp[rr], fn.exp[ss]
        A, B = fn.center[rr], fn.center[ss]
        p = a + b
        P = (a[:, None] * A + b[:, None] * B) / p[:, None]
        pref = fn.norm[rr] * fn.norm[ss] * np.exp(-(a * b / p) * ((A - B) ** 2).sum(1)) * p ** -1.5
        pts = P[:, None, :] + T[None, :, :] / np.sqrt(p)[:, None, None]      # (k, n^3, 3)
        poly = np.ones(pts.shape[:2])
        for d in range(3):
            poly = poly * np.where(fn.pow[rr, d][:, None] == 1, pts[..., d] - A[:, None, d], 1.0)
            poly = poly * np.where(fn.pow[ss, d][:, None] == 1, pts[..., d] - B[:, None, d], 1.0)
        harm = H.regular(L, pts - X[k0:k1, None, :])                        # (k, n^3, Q)
        out[k0:k1] = pref[:, None] * np.einsum("kp,kpq->kq", poly * Wt[None, :], harm)
    return out


def overlap_pairs(fn: Functions, r: np.ndarray, s: np.ndarray) -> np.ndarray:
    """S_rs for the given pairs: the l = 0 multipole, by the same quadrature."""
    return ao_multipoles(fn, r, s, np.zeros(3), 0)[:, 0].real
