"""GPU parity: occk_far_K (HIP, through the C ABI) against the FP64 oracle.

Gate (normwise, FP64 path): max|K_gpu - K_oracle| <= 1e-8 * max|K_oracle|.
Cases span several GEMM and translation tiles, ragged j batches, i/j
sub-ranges, every MFMA row-tile count of the translation kernel (L = 0..8),
1-D, 2-D and 3-D trees, accumulation, and the no-far-field degenerate case.
"""
import numpy as np
import pytest

import workloads
from oracle.fmm import Setup, far_K as oracle_far_K

from conftest import rel, with_params

pytestmark = pytest.mark.gpu

TOL = 1e-8


@pytest.fixture(scope="module")
def torch_cuda():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    return torch


def _gpu(torch, wl, C, params=None, i_range=None, j_range=None, jblock=0, K0=None, accumulate=False):
    from paper_1708_05353_amd import occk
    tr = occk.Tree(wl.system, params or wl.params)
    Cd = torch.from_numpy(C).cuda()
    n = C.shape[1]
    K = torch.zeros((wl.system.nbasis, n), dtype=torch.float64, device="cuda") if K0 is None else \
        torch.from_numpy(K0.copy()).cuda()
    occk.far_K(tr, Cd, K, i_range=i_range, j_range=j_range, jblock=jblock, accumulate=accumulate)
    torch.cuda.synchronize()
    out = K.cpu().numpy()
    tr.free()
    return out


@pytest.mark.parametrize("L", [0, 1, 2, 4, 6, 8])
def test_tiny_chain_all_ranks(torch_cuda, tiny, L):
    wl, C, st = tiny
    p = with_params(wl, lmax=L)
    st = st if L == 2 else Setup(wl.system, p)
    ref = oracle_far_K(st, C)
    got = _gpu(torch_cuda, wl, C, params=p)
    assert rel(got, ref) <= TOL, rel(got, ref)


@pytest.fixture(scope="module")
def sheet3():
    wl = workloads.graphene_flake(n=2, lmax=3, nocc=12, depth=3)
    C = wl.orbitals()
    return wl, C, Setup(wl.system, wl.params)


def test_sheet_ranges_and_ragged_batches(torch_cuda, sheet3):
    wl, C, st = sheet3
    ref = oracle_far_K(st, C, i_range=(3, 11), j_range=(2, 12))
    got = _gpu(torch_cuda, wl, C, i_range=(3, 11), j_range=(2, 12), jblock=3)
    assert rel(got[:, 3:11], ref) <= TOL
    # columns outside [i0, i1) are untouched
    assert np.all(got[:, :3] == 0) and np.all(got[:, 11:] == 0)


def test_sheet_full_and_accumulate(torch_cuda, sheet3):
    wl, C, st = sheet3
    ref = oracle_far_K(st, C)
    K0 = np.random.default_rng(1).standard_normal((wl.system.nbasis, C.shape[1]))
    got = _gpu(torch_cuda, wl, C, K0=K0, accumulate=True)
    assert rel(got - K0, ref) <= TOL


def test_water_cluster_3d(torch_cuda):
    wl = workloads.water_cluster(20, 40, lmax=2)
    C = wl.orbitals()
    st = Setup(wl.system, wl.params)
    ref = oracle_far_K(st, C, j_range=(0, 17))
    got = _gpu(torch_cuda, wl, C, j_range=(0, 17), jblock=8)
    assert rel(got, ref) <= TOL


def test_no_far_field_gives_zero(torch_cuda):
    wl = workloads.tiny_chain()
    p = with_params(wl, depth=1)      # two leaves, both near: no interaction list
    K0 = np.ones((80, 20))
    got = _gpu(torch_cuda, wl, wl.orbitals(), params=p, K0=K0)
    assert np.all(got == 0)


def test_bitwise_reproducible(torch_cuda, sheet3):
    wl, C, st = sheet3
    a = _gpu(torch_cuda, wl, C, jblock=5)
    b = _gpu(torch_cuda, wl, C, jblock=5)
    assert np.array_equal(a, b)


def test_j_additivity_on_gpu(torch_cuda, sheet3):
    wl, C, st = sheet3
    full = _gpu(torch_cuda, wl, C)
    part = _gpu(torch_cuda, wl, C, j_range=(0, 5)) + _gpu(torch_cuda, wl, C, j_range=(5, 12))
    assert rel(part, full) <= 1e-13
