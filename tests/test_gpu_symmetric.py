"""Symmetric schedule of occk_far_K (i and j over the same orbitals).

Omega^B and the translated local expansions are symmetric in (i, j), so a
j batch starting at j0 carries only the columns i >= j0, and K takes a
second, mirrored L2P contraction per batch.  These cases check it against
the FP64 oracle and against the all-columns schedule (used whenever the i
and j ranges differ) on batch sizes that put the first carried column in
the middle of 64-column GEMM tiles and 256-column translation tiles, with
a ragged last batch, a single batch, one column per batch, and the MFMA
translation kernel (L = 4) as well as the vector one (L = 2).
"""
import numpy as np
import pytest

import workloads
from oracle.fmm import Setup, far_K as oracle_far_K

from conftest import rel

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def torch_cuda():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    return torch


@pytest.fixture(scope="module")
def water75():
    wl = workloads.water_cluster(15, 43, lmax=2)
    C = wl.orbitals()
    return wl, C, oracle_far_K(Setup(wl.system, wl.params), C)


def _run(torch, tr, C, n, **kw):
    from paper_1708_05353_amd import occk
    K = torch.zeros((C.shape[0], n), dtype=torch.float64, device="cuda")
    occk.far_K(tr, C, K, **kw)
    torch.cuda.synchronize()
    return K.cpu().numpy()


@pytest.mark.parametrize("jblock", [1, 7, 33, 70, 200])
def test_symmetric_batches_match_oracle(torch_cuda, water75, jblock):
    from paper_1708_05353_amd import occk
    wl, C, ref = water75
    n = C.shape[1]
    assert n == 75
    tr = occk.Tree(wl.system, wl.params)
    print(f"[sym] water75 L2 jblock {jblock}", flush=True)
    got = _run(torch_cuda, tr, torch_cuda.from_numpy(C).cuda(), n, jblock=jblock)
    tr.free()
    assert rel(got, ref) <= 1e-8


def test_symmetric_equals_all_columns(torch_cuda, water75):
    """Symmetric schedule vs two all-columns calls over j halves (the i
    range differs from each j range, so those use the full column set)."""
    from paper_1708_05353_amd import occk
    wl, C, _ = water75
    n = C.shape[1]
    tr = occk.Tree(wl.system, wl.params)
    Cd = torch_cuda.from_numpy(C).cuda()
    sym = _run(torch_cuda, tr, Cd, n, jblock=16)
    K = torch_cuda.zeros((C.shape[0], n), dtype=torch_cuda.float64, device="cuda")
    occk.far_K(tr, Cd, K, j_range=(0, 40), jblock=16)
    occk.far_K(tr, Cd, K, j_range=(40, n), jblock=16, accumulate=True)
    torch_cuda.cuda.synchronize()
    tr.free()
    assert rel(sym, K.cpu().numpy()) <= 1e-13


@pytest.mark.parametrize("prec,tol", [(0, 1e-8), (1, 1e-6), (3, 1e-6)], ids=["fp64", "fp32", "bf16x6"])
def test_symmetric_mfma_translations(torch_cuda, prec, tol):
    """L = 4 (Q = 25): the MFMA translation kernel on carried columns."""
    from paper_1708_05353_amd import occk
    wl = workloads.water_cluster(12, 42, lmax=4)
    C = wl.orbitals()
    ref = oracle_far_K(Setup(wl.system, wl.params), C)
    tr = occk.Tree(wl.system, wl.params)
    print(f"[sym] water60 L4 prec {prec}", flush=True)
    got = _run(torch_cuda, tr, torch_cuda.from_numpy(C).cuda(), C.shape[1], jblock=13, precision=prec)
    tr.free()
    assert rel(got, ref) <= tol


def test_symmetric_K_ij_is_symmetric(torch_cuda, water75):
    """C^T K is symmetric (the square-truncated far-field kernel is)."""
    from paper_1708_05353_amd import occk
    wl, C, _ = water75
    tr = occk.Tree(wl.system, wl.params)
    got = _run(torch_cuda, tr, torch_cuda.from_numpy(C).cuda(), C.shape[1], jblock=20)
    tr.free()
    Kij = C.T @ got
    assert np.abs(Kij - Kij.T).max() <= 1e-10 * np.abs(Kij).max()


@pytest.mark.parametrize("prec,tol", [(0, 1e-8), (1, 1e-6), (3, 1e-6), (2, 5e-5)],
                         ids=["fp64", "fp32", "bf16x6", "bf16x3"])
def test_symmetric_whole_leaf_mirrored_tiles(torch_cuda, prec, tol):
    """Alkane chain whose leaves hold at most 144 functions (mean 131): the
    direct and mirrored L2P run in 144 x 64 and 64 x 144 tiles, one per leaf,
    with ragged leaves, in every precision."""
    wl = workloads.alkane_chain(n_carbon=100, depth=6)
    C = wl.orbitals()
    ref = oracle_far_K(Setup(wl.system, wl.params), C)
    from paper_1708_05353_amd import occk
    tr = occk.Tree(wl.system, wl.params)
    assert tr.info.max_nb <= 144
    print(f"[sym] alkane C100 L2 prec {prec}", flush=True)
    got = _run(torch_cuda, tr, torch_cuda.from_numpy(C).cuda(), C.shape[1], jblock=64, precision=prec)
    tr.free()
    assert rel(got, ref) <= tol


@pytest.mark.parametrize("prec", ["fp64", "fp32"])
def test_two_streams_equal_one_stream(torch_cuda, prec):
    """On a chain-like tree (both walks) the default schedule runs Omega and
    the L2P on a second stream of the library, two j batches in flight, and
    the translations on the caller's stream.  Every output element takes
    the same kernels in the same order as in the one-stream schedule, so K
    is equal bit for bit; and it matches the oracle.  Ragged last batch and
    an odd number of batches (both leaf regions in use, the last batch in
    the first)."""
    from paper_1708_05353_amd import occk
    torch = torch_cuda
    wl = workloads.alkane_chain(n_carbon=40, depth=5)
    C = wl.orbitals()
    n = C.shape[1]
    tr = occk.Tree(wl.system, wl.params)
    Cd = torch.from_numpy(C).cuda()
    code = {"fp64": occk.PREC_FP64, "fp32": occk.PREC_FP32}[prec]
    for jb in (16, 48, 64):
        nb = -(-n // jb)
        K2 = _run(torch, tr, Cd, n, jblock=jb, precision=code)
        K1 = _run(torch, tr, Cd, n, jblock=jb, precision=code, one_stream=True)
        print(f"[sym] two streams, {prec}, jblock {jb} ({nb} batches)", flush=True)
        assert nb > 1
        assert np.array_equal(K2, K1)
    ref = oracle_far_K(Setup(wl.system, wl.params), C)
    assert rel(K2, ref) <= (1e-8 if prec == "fp64" else 1e-6)
    tr.free()


def test_automatic_batch_width_follows_the_schedule(torch_cuda):
    """Automatic j batches: at most 128 wide where the FP64 call runs the
    two-stream schedule (chain-like tree, symmetric, fixed rank), at most 256
    in one stream and in the mixed modes; the results agree with the oracle
    either way."""
    from paper_1708_05353_amd import occk
    torch = torch_cuda
    wl = workloads.alkane_chain(n_carbon=40, depth=5)
    C = wl.orbitals()
    n = C.shape[1]
    assert n > 128
    tr = occk.Tree(wl.system, wl.params)
    Cd = torch.from_numpy(C).cuda()
    ref = oracle_far_K(Setup(wl.system, wl.params), C)
    print(f"[sym] automatic j batch width, n = {n}", flush=True)
    K2 = _run(torch, tr, Cd, n, jblock=0, precision=occk.PREC_FP64)
    assert tr.workspace_jblock() == 128
    assert rel(K2, ref) <= 1e-8
    K1 = _run(torch, tr, Cd, n, jblock=0, precision=occk.PREC_FP64, one_stream=True)
    assert tr.workspace_jblock() == min(n, 256)
    assert rel(K1, ref) <= 1e-8
    Kf = _run(torch, tr, Cd, n, jblock=0, precision=occk.PREC_FP32)
    assert tr.workspace_jblock() == min(n, 256)
    assert rel(Kf, ref) <= 1e-6
    tr.free()
