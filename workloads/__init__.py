"""Seeded synthetic workloads for the far-field occupied exchange.

This module only *generates inputs*: geometries, uncontracted s/p Gaussian
basis sets, occupied orbital coefficients C and the tree parameters of each
workload.  It holds none of the multipole method's arithmetic and is shared by
the CPU oracle (``oracle/``), the tests and the benchmark; the HIP library
receives its outputs through the C ABI.

The paper's systems (def2-SVP basis, the C400H802 / C150H30 / (H2O)100 /
Crambin geometries of its Table II) are not available, so each workload is a
rule-generated stand-in with the same atom counts, function counts, occupied
counts and spatial dimensionality (1-D chain, 2-D sheet, 3-D clusters, 3-D
globule).  Units are bohr.  Random numbers come from numpy's PCG64
(``numpy.random.default_rng``) with fixed seeds.

Orbitals: a dense random Gaussian matrix orthonormalised in the overlap metric
(C^T S C = I).  The paper's canonical MOs are dense and delocalised and it makes
no density-sparsity assumption (Conclusion), so a dense C is the faithful
stand-in.  The overlap matrix S is input preparation, not part of the method.
"""
from __future__ import annotations

import math
from dataclasses import dataclass, field

import numpy as np

__all__ = [
    "System", "TreeParams", "Workload",
    "tiny_chain", "alkane_chain", "graphene_flake", "water_cluster",
    "water_batch", "protein_blob", "overlap_matrix", "occupied_orbitals",
    "function_table", "SPLIT_X", "SPLIT_XY", "SPLIT_XYZ",
]

SPLIT_X, SPLIT_XY, SPLIT_XYZ = 1, 3, 7
ANGSTROM = 1.0 / 0.529177210903  # bohr per angstrom (used only for cfg-2's C-C bond)

# ----------------------------------------------------------------------------
# basis rules (synthetic; chosen to reproduce the function counts of the
# paper's systems: C/N/O-like 14, S-like 18, H-like 5 functions)
# ----------------------------------------------------------------------------


def _geometric(hi: float, lo: float, n: int) -> list[float]:
    r = (lo / hi) ** (1.0 / (n - 1))
    return [hi * r ** k for k in range(n)]


def site_shells(kind: str) -> list[tuple[int, float]]:
    """(l, exponent) list of the uncontracted primitive shells on one site."""
    if kind in ("C", "N", "O"):
        s = _geometric(3000.0, 0.15, 5)
        return [(0, e) for e in s] + [(1, e) for e in s[-3:]]
    if kind == "S":
        s = _geometric(3000.0, 0.15, 6)
        return [(0, e) for e in s] + [(1, e) for e in s[-4:]]
    if kind == "H":
        return [(0, 13.0), (0, 0.12), (1, math.sqrt(0.12 * 13.0))]
    if kind == "X":  # tiny-chain site: 4 s shells, geometric 0.1 .. 10
        return [(0, 0.1 * 100.0 ** (k / 3.0)) for k in range(4)]
    if kind == "Y":  # small s+p test site: 2 s shells and one p shell, compact
        return [(0, 4.0), (0, 1.2), (1, 1.5)]
    raise ValueError(kind)


ELECTRONS = {"C": 6, "N": 7, "O": 8, "S": 16, "H": 1}


@dataclass
class System:
    """Atoms plus an uncontracted s/p Cartesian Gaussian basis.

    Functions are ordered by shell; a p shell contributes x, y, z in that
    order.  Every primitive is normalised.
    """
    name: str
    xyz: np.ndarray                 # (natoms, 3) float64, bohr
    species: list[str]
    shell_atom: np.ndarray          # (nshell,) int32
    shell_l: np.ndarray             # (nshell,) int32, 0 or 1
    shell_exp: np.ndarray           # (nshell,) float64
    nocc: int

    @property
    def natoms(self) -> int:
        return int(self.xyz.shape[0])

    @property
    def nshell(self) -> int:
        return int(self.shell_l.shape[0])

    @property
    def nbasis(self) -> int:
        return int(np.sum(2 * self.shell_l + 1))


@dataclass
class TreeParams:
    split_mask: int          # bit0 x, bit1 y, bit2 z
    depth: int               # number of subdivisions: 2**depth boxes per split dimension
    ws: int                  # near iff Chebyshev box-index distance <= ws (same level)
    lmax: int                # multipole rank L (l <= L and l' <= L)
    pair_log_thresh: float = math.log(1e12)  # keep pair iff (ab/(a+b))|A-B|^2 <= thresh
    near_rule: int = 0       # 0: box-index ws above; 1: extents of the charge distributions
    ext_ws: float = 0.0      # extent rule: far iff |Xa - Xb| > (1 + ext_ws)(ext_a + ext_b)
    ext_tau: float = 1e-8    # extent of a distribution of exponent p: erfc^-1(ext_tau) / sqrt(p)


@dataclass
class Workload:
    system: System
    params: TreeParams
    seed: int
    C: np.ndarray | None = field(default=None, repr=False)

    def orbitals(self) -> np.ndarray:
        if self.C is None:
            self.C = occupied_orbitals(self.system, self.seed)
        return self.C


def _build(name, xyz, species, nocc) -> System:
    sa, sl, se = [], [], []
    for a, sp in enumerate(species):
        for l, e in site_shells(sp):
            sa.append(a)
            sl.append(l)
            se.append(e)
    return System(name, np.ascontiguousarray(xyz, dtype=np.float64), list(species),
                  np.asarray(sa, np.int32), np.asarray(sl, np.int32),
                  np.asarray(se, np.float64), int(nocc))


# ----------------------------------------------------------------------------
# geometries
# ----------------------------------------------------------------------------


def tiny_chain() -> Workload:
    """20 sites on the x axis, 2 bohr apart, 4 s shells each (nbasis 80, nocc 20)."""
    xyz = np.zeros((20, 3))
    xyz[:, 0] = 2.0 * np.arange(20)
    sysm = _build("tiny_chain", xyz, ["X"] * 20, 20)
    return Workload(sysm, TreeParams(SPLIT_X, 3, 2, 2, math.inf), seed=1)


def sp_chain(n: int = 10, spacing: float = 2.4, lmax: int = 2, depth: int = 3) -> Workload:
    """n compact s+p sites (2 s shells, 1 p shell) on the x axis, slightly
    zig-zag in y; nbasis 5n, nocc n; no pair screening (small tests of the
    near field, which needs exact integrals over every function type)."""
    xyz = np.zeros((n, 3))
    xyz[:, 0] = spacing * np.arange(n)
    xyz[:, 1] = 0.3 * (np.arange(n) % 2)
    sysm = _build(f"sp_chain_{n}", xyz, ["Y"] * n, n)
    return Workload(sysm, TreeParams(SPLIT_X, depth, 1, lmax, math.inf), seed=11)


def alkane_chain(n_carbon: int = 400, lmax: int = 2, depth: int = 8) -> Workload:
    """All-trans zig-zag CnH(2n+2) along x (C400H802: nbasis 9610, nocc 1601).

    C-C 1.54 angstrom at the tetrahedral angle; each carbon carries two
    hydrogens at 2.06 bohr, outward along the zig-zag bisector and split +-z at
    the tetrahedral angle; each terminal carbon carries one more along the
    chain axis.
    """
    bond = 1.54 * ANGSTROM
    tet = math.acos(-1.0 / 3.0)
    dx = bond * math.sin(tet / 2)
    dy = bond * math.cos(tet / 2) / 2
    ch = 2.06
    xyz, sp = [], []
    for k in range(n_carbon):
        s = 1.0 if k % 2 == 0 else -1.0
        xyz.append((dx * k, s * dy, 0.0))
        sp.append("C")
    for k in range(n_carbon):
        s = 1.0 if k % 2 == 0 else -1.0
        c = np.array(xyz[k])
        for sz in (1.0, -1.0):
            v = np.array([0.0, s * math.cos(tet / 2), sz * math.sin(tet / 2)])
            xyz.append(tuple(c + ch * v))
            sp.append("H")
    xyz.append(tuple(np.array(xyz[0]) + ch * np.array([-1.0, 0, 0])))
    sp.append("H")
    xyz.append(tuple(np.array(xyz[n_carbon - 1]) + ch * np.array([1.0, 0, 0])))
    sp.append("H")
    nel = sum(ELECTRONS[s] for s in sp)
    sysm = _build(f"alkane_C{n_carbon}H{2 * n_carbon + 2}", np.array(xyz), sp, nel // 2)
    return Workload(sysm, TreeParams(SPLIT_X, depth, 2, lmax), seed=2)


def graphene_flake(n: int = 5, lmax: int = 2, nocc: int | None = 480, depth: int = 4) -> Workload:
    """Hexagonal flake C(6n^2)H(6n) in the xy plane (n=5: C150H30, nbasis 2250).

    Rings whose hexagonal distance from the centre ring is < n; C-C 2.68 bohr;
    every two-coordinated carbon carries one hydrogen at 2.06 bohr on the
    outward bisector.  nocc defaults to 480 (the paper's 930 electrons give 465).
    """
    d = 2.68
    a = math.sqrt(3.0) * d
    a1 = np.array([a, 0.0])
    a2 = np.array([a / 2, a * math.sqrt(3.0) / 2])
    verts: dict[tuple[int, int], np.ndarray] = {}
    for i in range(-n + 1, n):
        for j in range(-n + 1, n):
            if max(abs(i), abs(j), abs(i + j)) > n - 1:
                continue
            c = i * a1 + j * a2
            for k in range(6):
                ang = math.radians(30 + 60 * k)
                v = c + d * np.array([math.cos(ang), math.sin(ang)])
                key = (int(round(v[0] * 1e6)), int(round(v[1] * 1e6)))
                verts[key] = v
    carb = np.array(sorted(verts.values(), key=lambda v: (round(v[1], 6), round(v[0], 6))))
    dist = np.linalg.norm(carb[:, None, :] - carb[None, :, :], axis=-1)
    nbr = (dist < d * 1.1) & (dist > 1e-6)
    hyd = []
    for k in range(len(carb)):
        idx = np.nonzero(nbr[k])[0]
        if len(idx) == 2:
            out = (carb[k] - carb[idx[0]]) + (carb[k] - carb[idx[1]])
            hyd.append(carb[k] + 2.06 * out / np.linalg.norm(out))
    xyz = np.zeros((len(carb) + len(hyd), 3))
    xyz[: len(carb), :2] = carb
    xyz[len(carb):, :2] = np.array(hyd)
    sp = ["C"] * len(carb) + ["H"] * len(hyd)
    nel = sum(ELECTRONS[s] for s in sp)
    sysm = _build(f"graphene_C{len(carb)}H{len(hyd)}", xyz, sp,
                  nel // 2 if nocc is None else nocc)
    return Workload(sysm, TreeParams(SPLIT_XY, depth, 2, lmax), seed=3)


def _random_rotation(rng) -> np.ndarray:
    q = rng.standard_normal(4)
    q /= np.linalg.norm(q)
    w, x, y, z = q
    return np.array([
        [1 - 2 * (y * y + z * z), 2 * (x * y - z * w), 2 * (x * z + y * w)],
        [2 * (x * y + z * w), 1 - 2 * (x * x + z * z), 2 * (y * z - x * w)],
        [2 * (x * z - y * w), 2 * (y * z + x * w), 1 - 2 * (x * x + y * y)],
    ])


def water_cluster(nmol: int, seed: int, lmax: int = 2, depth: int = 3) -> Workload:
    """nmol waters: O uniform in a sphere at 1 g/cm^3 (201.9 bohr^3 per molecule),
    O-O >= 4.5 bohr by rejection, O-H 1.81 bohr, H-O-H 104.5 deg, random
    orientation.  nbasis 24*nmol, nocc 5*nmol."""
    rng = np.random.default_rng([seed, 0])
    radius = (3.0 * 201.9 * nmol / (4.0 * math.pi)) ** (1.0 / 3.0)
    oxy: list[np.ndarray] = []
    while len(oxy) < nmol:
        p = rng.uniform(-radius, radius, 3)
        if np.dot(p, p) > radius * radius:
            continue
        if all(np.linalg.norm(p - q) >= 4.5 for q in oxy):
            oxy.append(p)
    half = math.radians(104.5) / 2
    h1 = 1.81 * np.array([math.sin(half), 0.0, math.cos(half)])
    h2 = 1.81 * np.array([-math.sin(half), 0.0, math.cos(half)])
    xyz, sp = [], []
    for o in oxy:
        R = _random_rotation(rng)
        xyz += [o, o + R @ h1, o + R @ h2]
        sp += ["O", "H", "H"]
    sysm = _build(f"water_{nmol}", np.array(xyz), sp, 5 * nmol)
    return Workload(sysm, TreeParams(SPLIT_XYZ, depth, 2, lmax), seed=seed)


def water_batch() -> list[Workload]:
    """16 clusters of 20 + round(80k/15) molecules (20 .. 100), seeds 40..55."""
    return [water_cluster(20 + int(round(80 * k / 15)), 40 + k) for k in range(16)]


def protein_blob(seed: int = 5, lmax: int = 8, nocc: int | None = 1261, depth: int = 3,
                 scale: float = 1.0) -> Workload:
    """644 sites (202 C, 317 H, 64 O, 55 N, 6 S; nbasis 6187) uniform in a sphere
    of radius 20.36 bohr (4732 amu at 1.5 g/cm^3), minimum distance 1.9 bohr.

    scale < 1 keeps the density and the composition ratios with about
    scale * 644 sites (smaller globules for training the rank selector);
    nocc=None then takes half the electrons."""
    rng = np.random.default_rng([seed, 0])
    counts = {"C": 202, "H": 317, "O": 64, "N": 55, "S": 6}
    if scale != 1.0:
        counts = {k: max(1, int(round(v * scale))) for k, v in counts.items()}
    comp = [k for k, v in counts.items() for _ in range(v)]
    comp = [comp[k] for k in rng.permutation(len(comp))]
    radius = 20.36 * (len(comp) / 644.0) ** (1.0 / 3.0)
    pts: list[np.ndarray] = []
    while len(pts) < len(comp):
        p = rng.uniform(-radius, radius, 3)
        if np.dot(p, p) > radius * radius:
            continue
        if pts and np.min(np.linalg.norm(np.array(pts) - p, axis=1)) < 1.9:
            continue
        pts.append(p)
    if nocc is None:
        nocc = sum(ELECTRONS[s] for s in comp) // 2
    sysm = _build("protein_blob" if scale == 1.0 else f"protein_blob_{len(comp)}", np.array(pts), comp, nocc)
    return Workload(sysm, TreeParams(SPLIT_XYZ, depth, 2, lmax), seed=seed)


# ----------------------------------------------------------------------------
# overlap matrix and orthonormal occupied orbitals (input preparation)
# ----------------------------------------------------------------------------


def function_table(sysm: System):
    """Per-function arrays: centre (nbf,3), exponent, Cartesian powers (nbf,3)."""
    cen, ex, pw = [], [], []
    for s in range(sysm.nshell):
        A = sysm.xyz[sysm.shell_atom[s]]
        if sysm.shell_l[s] == 0:
            cen.append(A); ex.append(sysm.shell_exp[s]); pw.append((0, 0, 0))
        else:
            for d in range(3):
                p = [0, 0, 0]
                p[d] = 1
                cen.append(A); ex.append(sysm.shell_exp[s]); pw.append(tuple(p))
    return np.array(cen), np.array(ex), np.array(pw, dtype=np.int64)


def overlap_matrix(sysm: System) -> np.ndarray:
    """S_rs for normalised Cartesian s/p primitives (closed form, products of
    1-D Gaussian moments)."""
    cen, ex, pw = function_table(sysm)
    norm = (2 * ex / math.pi) ** 0.75 * np.where(pw.sum(1) == 1, 2 * np.sqrt(ex), 1.0)
    n = len(ex)
    S = np.empty((n, n))
    blk = 1024
    for r0 in range(0, n, blk):
        r1 = min(n, r0 + blk)
        a = ex[r0:r1, None]
        b = ex[None, :]
        p = a + b
        val = norm[r0:r1, None] * norm[None, :] * (math.pi / p) ** 1.5
        for d in range(3):
            A = cen[r0:r1, None, d]
            B = cen[None, :, d]
            P = (a * A + b * B) / p
            ia = pw[r0:r1, None, d]
            ib = pw[None, :, d]
            fac = np.exp(-a * b / p * (A - B) ** 2)
            PA, PB = P - A, P - B
            poly = np.where(ia == 1, PA, 1.0) * np.where(ib == 1, PB, 1.0)
            poly = poly + np.where((ia == 1) & (ib == 1), 0.5 / p, 0.0)
            val = val * fac * poly
        S[r0:r1] = val
    return 0.5 * (S + S.T)


def occupied_orbitals(sysm: System, seed: int, nocc: int | None = None) -> np.ndarray:
    """C (nbasis x nocc, row-major float64) with C^T S C = I.

    G ~ N(0,1); Q = qr(G); S = L L^T; C = L^-T Q.  If the Cholesky factorisation
    fails, canonical orthogonalisation (eigenvalues < 1e-10 dropped) is used.
    """
    from scipy.linalg import cholesky, solve_triangular
    nocc = sysm.nocc if nocc is None else nocc
    rng = np.random.default_rng([seed, 1])
    S = overlap_matrix(sysm)
    n = S.shape[0]
    try:
        Lc = cholesky(S, lower=True)
        G = rng.standard_normal((n, nocc))
        Q, _ = np.linalg.qr(G)
        C = solve_triangular(Lc.T, Q, lower=False)
    except np.linalg.LinAlgError:
        w, U = np.linalg.eigh(S)
        keep = w > 1e-10
        X = U[:, keep] / np.sqrt(w[keep])
        G = rng.standard_normal((int(keep.sum()), nocc))
        Q, _ = np.linalg.qr(G)
        C = X @ Q
    return np.ascontiguousarray(C)


def localized_orbitals(sysm: System, seed: int, nocc: int | None = None) -> np.ndarray:
    """Occupied orbitals localised by construction (input for occupied-pair
    screening): the nocc orbitals are dealt to the sites in proportion to
    their function counts, each a seeded N(0,1) combination of its own site's
    functions (orthonormalised within the site); the columns are then
    orthonormalised symmetrically in the overlap metric,
    C = G (G^T S G)^{-1/2}, which keeps every orbital on its site up to tails
    that decay with distance.  Columns are ordered along the system's longest
    direction."""
    nocc = sysm.nocc if nocc is None else nocc
    rng = np.random.default_rng([seed, 3])
    S = overlap_matrix(sysm)
    xyz = sysm.xyz
    axis = int(np.argmax(xyz.max(0) - xyz.min(0)))
    order = np.argsort(xyz[:, axis], kind="stable")
    funcs = [[] for _ in range(len(xyz))]
    f = 0
    for sh in range(sysm.nshell):
        nf = 1 if sysm.shell_l[sh] == 0 else 3
        funcs[int(sysm.shell_atom[sh])].extend(range(f, f + nf))
        f += nf
    total = sum(len(v) for v in funcs)
    share = np.array([len(funcs[a]) * nocc / total for a in order])
    count = np.floor(share).astype(int)
    for a in np.argsort(-(share - count), kind="stable")[: nocc - count.sum()]:
        count[a] += 1
    G = np.zeros((S.shape[0], nocc))
    k = 0
    for a, m in zip(order, count):
        if m == 0:
            continue
        rows = np.array(funcs[a])
        Q, _ = np.linalg.qr(rng.standard_normal((len(rows), m)))
        G[rows, k:k + m] = Q
        k += m
    M = G.T @ S @ G
    w, U = np.linalg.eigh(M)
    C = G @ (U / np.sqrt(w)) @ U.T
    return np.ascontiguousarray(C)
