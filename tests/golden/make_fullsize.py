"""Writes the oracle's K^ff for sampled output columns of the full-size
workloads (tests/golden/fullsize_<name>.npz), for the GPU parity tests at
sizes where the oracle takes minutes to tens of minutes.

Calls only the oracle (oracle/) and the seeded input generators (workloads/).
Each file holds, for its workload: the sampled i ranges, the summed j range,
the oracle's K columns (nbasis x sampled columns, float64) and a fingerprint
of the orthonormal orbitals C (the first 4x4 block and the Frobenius norm),
so that a test can check that it regenerated the same inputs.

    python tests/golden/make_fullsize.py [name ...] [--workers N]

names: alkane_L4 graphene_L8 water_batch protein_L8_1261 protein_L8_1700
(default: all).
"""
from __future__ import annotations

import argparse
import os
import sys
import time

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(os.path.dirname(HERE))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

import workloads  # noqa: E402
from oracle.fmm import Setup, far_K  # noqa: E402


def _ends(n: int, w: int = 2):
    return [(0, w), (n - w, n)]


# name -> (workload factory, i samples (from nocc), j range (None = all), oracle j batch)
CASES = {
    "alkane_L4": (lambda: workloads.alkane_chain(lmax=4), _ends, None, 64),
    "graphene_L8": (lambda: workloads.graphene_flake(lmax=8), _ends, None, 32),
    "protein_L8_1261": (lambda: workloads.protein_blob(nocc=1261), _ends, (0, 64), 16),
    "protein_L8_1700": (lambda: workloads.protein_blob(nocc=1700), _ends, (0, 64), 16),
}


def fingerprint(C: np.ndarray) -> np.ndarray:
    return np.concatenate([C[:4, :4].ravel(), [np.linalg.norm(C)]])


def _columns(st, C, samples, jr, jblock):
    return np.hstack([far_K(st, C, i_range=s, j_range=jr, jblock=jblock) for s in samples])


def make_case(name: str, workers: int, setups: dict):
    factory, samp, jr, jblock = CASES[name]
    t0 = time.time()
    wl = factory()
    C = wl.orbitals()
    key = (wl.system.name, wl.params.lmax)
    if key not in setups:
        setups.clear()
        setups[key] = Setup(wl.system, wl.params, workers=workers)
    st = setups[key]
    samples = samp(C.shape[1])
    K = _columns(st, C, samples, jr, jblock)
    np.savez(os.path.join(HERE, f"fullsize_{name}.npz"), K=K, samples=np.array(samples),
             j_range=np.array(jr if jr is not None else (0, C.shape[1])), fingerprint=fingerprint(C))
    print(f"{name}: {K.shape} in {time.time() - t0:.0f} s", flush=True)


def make_water_batch(workers: int):
    t0 = time.time()
    out = {}
    for k, wl in enumerate(workloads.water_batch()):
        C = wl.orbitals()
        st = Setup(wl.system, wl.params, workers=workers)
        samples = _ends(C.shape[1])
        out[f"K{k}"] = _columns(st, C, samples, None, 64)
        out[f"samples{k}"] = np.array(samples)
        out[f"fingerprint{k}"] = fingerprint(C)
    np.savez(os.path.join(HERE, "fullsize_water_batch.npz"), **out)
    print(f"water_batch: 16 systems in {time.time() - t0:.0f} s", flush=True)


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("names", nargs="*")
    ap.add_argument("--workers", type=int, default=os.cpu_count() or 1)
    a = ap.parse_args()
    names = a.names or ["alkane_L4", "graphene_L8", "water_batch", "protein_L8_1261", "protein_L8_1700"]
    setups: dict = {}
    for n in names:
        if n == "water_batch":
            make_water_batch(a.workers)
        else:
            make_case(n, a.workers, setups)


if __name__ == "__main__":
    main()
