"""Near-field exchange with exact integrals on the GPU (occk_near_K) against
the oracle (Obara-Saika integrals over the near leaf pairs), and near + far
on the GPU against the oracle's near + far.

Gates (normwise, max|dK|/max|K|): 1e-10 on the small systems (FP64
integrals; X is summed with atomic adds, so only the order of the last bits
differs between runs); 1e-8 on sampled rows of the full alkane chain.
"""
import time

import numpy as np
import pytest

import workloads
from oracle.eri import near_K as oracle_near_K, near_K_rows
from oracle.fmm import Setup, far_K as oracle_far_K

from conftest import rel, with_params

pytestmark = pytest.mark.gpu


def _occk():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_1708_05353_amd import occk
    return occk


def _gpu_near(occk, wl, p, C, tr=None):
    import torch
    own = tr is None
    tr = tr or occk.Tree(wl.system, p)
    Cd = torch.from_numpy(C).cuda()
    K = torch.full((wl.system.nbasis, C.shape[1]), 3.0, dtype=torch.float64, device="cuda")
    occk.near_K(tr, Cd, K)
    torch.cuda.synchronize()
    out = K.cpu().numpy()
    if own:
        tr.free()
    return out


CASES = {
    "chain_box": (workloads.tiny_chain, {}),
    "sp_chain_box": (lambda: workloads.sp_chain(n=10), {}),
    "sp_chain_extent": (lambda: workloads.sp_chain(n=10), dict(near_rule=1, ext_ws=0.0, ext_tau=1e-8)),
    "water2": (lambda: workloads.water_cluster(2, 40), {}),
}


@pytest.mark.parametrize("name", list(CASES))
def test_near_K_matches_oracle(name):
    occk = _occk()
    make, kw = CASES[name]
    wl = make()
    p = with_params(wl, lmax=0, **kw)
    C = wl.orbitals()
    print(f"[near] {name}: nbasis {wl.system.nbasis}", flush=True)
    ref = oracle_near_K(Setup(wl.system, p), C)
    got = _gpu_near(occk, wl, p, C)
    e = rel(got, ref)
    print(f"[near] {name}: eps_max {e:.3e}", flush=True)
    assert np.abs(ref).max() > 0
    assert e <= 1e-10


def test_near_plus_far_on_the_gpu():
    """sp chain, extent rule, L = 6: near + far from the two GPU entry points
    against the oracle's near + far (whose sum is pinned to the all-exact
    exchange on the CPU)."""
    import torch
    occk = _occk()
    wl = workloads.sp_chain(n=10)
    p = with_params(wl, lmax=6, near_rule=1, ext_ws=0.0, ext_tau=1e-8)
    C = wl.orbitals()
    st = Setup(wl.system, p)
    ref = oracle_near_K(st, C) + oracle_far_K(st, C)
    tr = occk.Tree(wl.system, p)
    Cd = torch.from_numpy(C).cuda()
    K = torch.zeros((wl.system.nbasis, C.shape[1]), dtype=torch.float64, device="cuda")
    occk.far_K(tr, Cd, K)
    occk.near_K(tr, Cd, K, accumulate=True)
    torch.cuda.synchronize()
    assert rel(K.cpu().numpy(), ref) <= 1e-10
    tr.free()


def test_alkane_near_field_sampled_rows():
    """The full alkane chain (nbasis 9610, nocc 1601, depth 8, ws 2): every
    column of sampled rows (an s and a p function) against the oracle."""
    import torch
    occk = _occk()
    wl = workloads.alkane_chain()
    C = wl.orbitals()
    tr = occk.Tree(wl.system, wl.params)
    Cd = torch.from_numpy(C).cuda()
    K = torch.zeros((wl.system.nbasis, C.shape[1]), dtype=torch.float64, device="cuda")
    t0 = time.perf_counter()
    occk.near_K(tr, Cd, K)
    torch.cuda.synchronize()
    tasks, quartets = occk.near_info(tr)
    print(f"[near] alkane: {time.perf_counter() - t0:.2f} s first call, {quartets} shell quartets", flush=True)
    st = Setup(wl.system, with_params(wl, lmax=0))
    rows = [int(np.nonzero(st.fn.pow.sum(1) == 0)[0][2000]), int(np.nonzero(st.fn.pow.sum(1) == 1)[0][3001])]
    ref = near_K_rows(st, C, rows)
    e = rel(K.cpu().numpy()[rows], ref)
    print(f"[near] alkane rows {rows}: eps_max {e:.3e}", flush=True)
    assert e <= 1e-8
    tr.free()
