"""Scaled regular (O) and irregular (M) solid harmonics, Eq. (4a,b).

  O_{l,m}(r) = eps_m r^l / (l+|m|)!  P_{l,|m|}(cos t) exp(-i m phi)
  M_{l,m}(r) = eps_m (l-|m|)! / r^(l+1) P_{l,|m|}(cos t) exp(+i m phi)
  eps_m = 1 for m >= 0, (-1)^m for m < 0.

P_{l,m} is the associated Legendre function with the Condon-Shortley phase
(the paper does not fix the phase; every identity of the method carries
matching phase factors, so the result does not depend on it).  It is computed
by the textbook three-term recurrence in l at fixed m.  To stay regular at
r = 0 and on the z axis, (1-x^2)^{m/2} e^{-+ i m phi} is written as
((x -+ i y)/r)^m, i.e. the recurrence runs on Pbar_{l,m} = P_{l,m}/(1-x^2)^{m/2}.

Components are stored flat at index l*l + l + m (m = -l..l); (L+1)^2 of them.
"""
from __future__ import annotations

import math

import numpy as np


def idx(l: int, m: int) -> int:
    return l * l + l + m


def ncomp(L: int) -> int:
    return (L + 1) * (L + 1)


def _powers(w: np.ndarray, n: int) -> list:
    out = [np.ones_like(w)]
    for _ in range(n):
        out.append(out[-1] * w)
    return out


def _pbar(lmax: int, x: np.ndarray) -> np.ndarray:
    """Pbar[l, m] = P_{l,m}(x) / (1-x^2)^{m/2} for 0 <= m <= l <= lmax."""
    out = np.zeros((lmax + 1, lmax + 1) + x.shape)
    for m in range(lmax + 1):
        dfact = 1.0
        for k in range(1, 2 * m, 2):
            dfact *= k
        out[m, m] = (-1) ** m * dfact
        if m + 1 <= lmax:
            out[m + 1, m] = x * (2 * m + 1) * out[m, m]
        for l in range(m + 2, lmax + 1):
            out[l, m] = ((2 * l - 1) * x * out[l - 1, m] - (l + m - 1) * out[l - 2, m]) / (l - m)
    return out


def regular(L: int, v: np.ndarray) -> np.ndarray:
    """O_{l,m}(v) for l <= L; v (..., 3) -> complex (..., (L+1)^2)."""
    v = np.asarray(v, dtype=np.float64)
    x, y, z = v[..., 0], v[..., 1], v[..., 2]
    r = np.sqrt(x * x + y * y + z * z)
    safe = np.where(r > 0, r, 1.0)
    pb = _pbar(L, np.where(r > 0, z / safe, 0.0))
    out = np.zeros(v.shape[:-1] + (ncomp(L),), dtype=np.complex128)
    wm = _powers(x - 1j * y, L)       # (r sin(t) e^{-i phi})^m
    wp = _powers(x + 1j * y, L)
    rp = _powers(r, L)
    for l in range(L + 1):
        for m in range(l + 1):
            radial = rp[l - m] * pb[l, m] / math.factorial(l + m)
            out[..., idx(l, m)] = radial * wm[m]
            if m > 0:
                out[..., idx(l, -m)] = (-1) ** m * radial * wp[m]
    return out


def irregular(L: int, v: np.ndarray) -> np.ndarray:
    """M_{l,m}(v) for l <= L; v (..., 3) with |v| > 0 -> complex (..., (L+1)^2)."""
    v = np.asarray(v, dtype=np.float64)
    x, y, z = v[..., 0], v[..., 1], v[..., 2]
    r = np.sqrt(x * x + y * y + z * z)
    if np.any(r == 0):
        raise ValueError("irregular harmonic at r = 0")
    pb = _pbar(L, z / r)
    out = np.zeros(v.shape[:-1] + (ncomp(L),), dtype=np.complex128)
    wm = _powers(x - 1j * y, L)
    wp = _powers(x + 1j * y, L)
    for l in range(L + 1):
        for m in range(l + 1):
            radial = math.factorial(l - m) * pb[l, m] / r ** (l + 1 + m)
            out[..., idx(l, m)] = radial * wp[m]
            if m > 0:
                out[..., idx(l, -m)] = (-1) ** m * radial * wm[m]
    return out
