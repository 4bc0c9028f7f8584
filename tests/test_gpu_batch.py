"""Many systems in one persistent launch (occk_batch_*).

* FP64 batched K of every system matches the oracle to 1e-8 (normwise).
* Each precision's batched K matches occk_far_K of the same precision:
  FP64 to 1e-12; mixed modes to the sum of their bounds against the oracle
  (the standalone call uses the symmetric schedule).
* Several j batches per system (explicit jblock) match the oracle.
* The autotuner returns a valid configuration and keeps results correct.
* A standalone call on one of the trees (which replaces its workspace)
  before a batched run is handled: the plan rebuilds its tables.
"""
import numpy as np
import pytest

import workloads
from oracle.fmm import Setup, far_K as oracle_far_K

from conftest import rel

pytestmark = pytest.mark.gpu

SIZES = [(6, 40), (9, 41), (12, 42), (15, 43), (7, 44)]   # (molecules, seed), uneven


@pytest.fixture(scope="module")
def systems():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_1708_05353_amd import occk
    out = []
    for n, seed in SIZES:
        wl = workloads.water_cluster(n, seed, depth=3)
        C = wl.orbitals()
        tr = occk.Tree(wl.system, wl.params)
        if tr.info.lmin < 0:
            continue
        out.append((wl, C, tr))
    assert len(out) >= 3
    return out


def _io(systems):
    import torch
    Cs = [torch.from_numpy(C).cuda() for wl, C, tr in systems]
    Ks = [torch.full((wl.system.nbasis, C.shape[1]), 7.0, dtype=torch.float64, device="cuda")
          for wl, C, tr in systems]
    return Cs, Ks


def test_batched_fp64_matches_oracle(systems):
    import torch
    from paper_1708_05353_amd import occk
    Cs, Ks = _io(systems)
    b = occk.Batch([tr for _, _, tr in systems], [C.shape[1] for _, C, _ in systems], occk.PREC_FP64)
    print("[batch] fp64 run", flush=True)
    b.run(Cs, Ks)
    torch.cuda.synchronize()
    print("[batch] fp64 done", flush=True)
    for (wl, C, tr), K in zip(systems, Ks):
        ref = oracle_far_K(Setup(wl.system, wl.params), C)
        assert rel(K.cpu().numpy(), ref) <= 1e-8
    b.free()


@pytest.mark.parametrize("prec", [0, 1, 3, 2], ids=["fp64", "fp32", "bf16x6", "bf16x3"])
def test_batched_equals_standalone(systems, prec):
    import torch
    from paper_1708_05353_amd import occk
    Cs, Ks = _io(systems)
    b = occk.Batch([tr for _, _, tr in systems], [C.shape[1] for _, C, _ in systems], prec)
    b.run(Cs, Ks)
    torch.cuda.synchronize()
    got = [K.cpu().numpy() for K in Ks]
    b.free()
    for (wl, C, tr), Cd, g in zip(systems, Cs, got):
        K1 = torch.zeros_like(Cd)
        occk.far_K(tr, Cd, K1, precision=prec, jblock=4)
        torch.cuda.synchronize()
        # FP64: the same arithmetic in another order.  Mixed modes: the
        # standalone call uses the symmetric schedule (column (j, i) stands
        # for (i, j)), the batched one all columns, so the two agree only to
        # the sum of their stated bounds against the FP64 oracle.
        tol = 1e-12 if prec == 0 else 2 * {1: 1e-6, 2: 5e-5, 3: 1e-6}[prec]
        assert rel(g, K1.cpu().numpy()) <= tol, prec


@pytest.mark.parametrize("prec,jblock,tol", [(0, 16, 1e-8), (1, 7, 1e-6), (0, 64, 1e-8)],
                         ids=["fp64-jb16", "fp32-jb7", "fp64-jb64"])
def test_batched_j_batches_match_oracle(systems, prec, jblock, tol):
    """Several j batches per system (symmetric schedule inside the
    persistent launch): first carried column inside 64-column GEMM tiles,
    ragged last batches, systems with one batch beside systems with many."""
    import torch
    from paper_1708_05353_amd import occk
    Cs, Ks = _io(systems)
    b = occk.Batch([tr for _, _, tr in systems], [C.shape[1] for _, C, _ in systems], prec, jblock=jblock)
    print(f"[batch] prec {prec} jblock {jblock}", flush=True)
    b.run(Cs, Ks)
    torch.cuda.synchronize()
    for (wl, C, tr), K in zip(systems, Ks):
        ref = oracle_far_K(Setup(wl.system, wl.params), C)
        assert rel(K.cpu().numpy(), ref) <= tol
    b.free()


def test_autotune_then_run(systems):
    import torch
    from paper_1708_05353_amd import occk
    Cs, Ks = _io(systems)
    b = occk.Batch([tr for _, _, tr in systems], [C.shape[1] for _, C, _ in systems], occk.PREC_FP32)
    choice = b.tune(Cs, Ks)
    assert 1 <= choice[0] <= 8 and choice[1] in (1, 2) and choice[2] in (1, 4)
    cfg = b.config()
    assert (cfg["blocks_per_cu"], cfg["gemm_group"], cfg["trans_group"]) == choice
    for K in Ks:
        K.fill_(3.0)
    b.run(Cs, Ks)
    torch.cuda.synchronize()
    wl, C, tr = systems[0]
    ref = oracle_far_K(Setup(wl.system, wl.params), C)
    assert rel(Ks[0].cpu().numpy(), ref) <= 1e-6
    b.free()


def test_plan_survives_standalone_call(systems):
    import torch
    from paper_1708_05353_amd import occk
    Cs, Ks = _io(systems)
    b = occk.Batch([tr for _, _, tr in systems], [C.shape[1] for _, C, _ in systems], occk.PREC_FP32)
    wl, C, tr = systems[1]
    K1 = torch.zeros_like(Cs[1])
    occk.far_K(tr, Cs[1], K1, precision=occk.PREC_FP32, jblock=3)   # replaces that tree's workspace
    b.run(Cs, Ks)
    torch.cuda.synchronize()
    ref = oracle_far_K(Setup(wl.system, wl.params), C)
    assert rel(Ks[1].cpu().numpy(), ref) <= 1e-6
    assert rel(K1.cpu().numpy(), ref) <= 1e-6
    b.free()


@pytest.mark.parametrize("L,prec", [(4, 0), (4, 3), (6, 1), (6, 2), (8, 0), (8, 3)],
                         ids=["L4-fp64", "L4-bf16x6", "L6-fp32", "L6-bf16x3", "L8-fp64", "L8-bf16x6"])
def test_batched_high_rank_equals_standalone(L, prec):
    """lmax 4..8 (2..6 MFMA row tiles): the persistent kernels are free of
    register spills (the split-BF16 GEMM tiles hold fragments, not FP32
    copies, and FP64/FP32 keep the compiler's allocation above one row
    tile), so batched plans are accepted at every rank the exchange kernels
    take.  Two uneven water clusters, several j batches; each system's K
    matches the standalone occk_far_K of the same precision, which the other
    tests pin on the oracle (FP64 to 1e-12, mixed modes to twice their
    bound)."""
    import torch
    from paper_1708_05353_amd import occk
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    sysl = [workloads.water_cluster(n, s, lmax=L, depth=3) for n, s in [(6, 40), (9, 41)]]
    trees = [occk.Tree(wl.system, wl.params) for wl in sysl]
    Cs = [torch.from_numpy(wl.orbitals()).cuda() for wl in sysl]
    Ks = [torch.zeros((wl.system.nbasis, C.shape[1]), dtype=torch.float64, device="cuda") for wl, C in zip(sysl, Cs)]
    b = occk.Batch(trees, [C.shape[1] for C in Cs], prec, jblock=16)
    print(f"[batch] L{L} prec {prec}", flush=True)
    b.run(Cs, Ks)
    torch.cuda.synchronize()
    b.free()
    tol = 1e-12 if prec == 0 else 2 * {1: 1e-6, 2: 5e-5, 3: 1e-6}[prec]
    for tr, C, K in zip(trees, Cs, Ks):
        K1 = torch.zeros_like(K)
        occk.far_K(tr, C, K1, precision=prec, jblock=16)
        torch.cuda.synchronize()
        assert rel(K.cpu().numpy(), K1.cpu().numpy()) <= tol
    if L == 4 and prec == 0:   # and the oracle itself at the smallest of these ranks
        wl = sysl[0]
        ref = oracle_far_K(Setup(wl.system, wl.params), Cs[0].cpu().numpy())
        assert rel(Ks[0].cpu().numpy(), ref) <= 1e-8
    for t in trees:
        t.free()


@pytest.mark.parametrize("prec,tol", [(0, 1e-8), (1, 1e-6), (3, 1e-6), (2, 5e-5)],
                         ids=["fp64", "fp32", "bf16x6", "bf16x3"])
def test_batched_L3_mfma_translations(prec, tol):
    """lmax = 3 (Q = 16): the persistent kernel's MFMA translation tiles with
    the operator staged in its shared memory; three uneven systems, two j
    batches for the larger ones."""
    import torch
    from paper_1708_05353_amd import occk
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    sysl = [workloads.water_cluster(n, s, lmax=3, depth=3) for n, s in [(6, 40), (9, 41), (12, 42)]]
    trees = [occk.Tree(wl.system, wl.params) for wl in sysl]
    Cs = [torch.from_numpy(wl.orbitals()).cuda() for wl in sysl]
    Ks = [torch.zeros((wl.system.nbasis, C.shape[1]), dtype=torch.float64, device="cuda") for wl, C in zip(sysl, Cs)]
    b = occk.Batch(trees, [C.shape[1] for C in Cs], prec, jblock=32)
    print(f"[batch] L3 prec {prec}", flush=True)
    b.run(Cs, Ks)
    torch.cuda.synchronize()
    for wl, C, K in zip(sysl, Cs, Ks):
        ref = oracle_far_K(Setup(wl.system, wl.params), C.cpu().numpy())
        assert rel(K.cpu().numpy(), ref) <= tol
    b.free()
    for t in trees:
        t.free()


def test_walks_equal_level_passes_bitwise():
    """Alkane chain (binary tree, short interaction lists): occk_far_K runs
    the translations as subtree walks and the L2P in whole-leaf tiles, the
    persistent batch kernel as level-by-level passes and 48-wide tiles.  Every
    output takes its terms in the same order, so the two agree bit for bit."""
    import torch
    from paper_1708_05353_amd import occk
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    wl = workloads.alkane_chain(n_carbon=100, depth=6)
    tr = occk.Tree(wl.system, wl.params)
    C = torch.from_numpy(wl.orbitals()).cuda()
    n = C.shape[1]
    print("[batch] alkane C100 walks vs level passes", flush=True)
    K1 = torch.zeros((wl.system.nbasis, n), dtype=torch.float64, device="cuda")
    occk.far_K(tr, C, K1, jblock=64)
    K2 = torch.zeros_like(K1)
    b = occk.Batch([tr], [n], occk.PREC_FP64, jblock=64)
    b.run([C], [K2])
    torch.cuda.synchronize()
    b.free()
    tr.free()
    assert np.array_equal(K1.cpu().numpy(), K2.cpu().numpy())


def test_one_call_batched_equals_the_plan(systems):
    """occk_far_K_batched (plan made, run and freed in one call) gives the
    plan's result bit for bit."""
    import torch
    from paper_1708_05353_amd import occk
    trees = [tr for _, _, tr in systems]
    Cs, Ks = _io(systems)
    b = occk.Batch(trees, [C.shape[1] for _, C, _ in systems], occk.PREC_FP32)
    b.run(Cs, Ks)
    torch.cuda.synchronize()
    b.free()
    _, K1 = _io(systems)
    occk.far_K_batched(trees, Cs, K1, precision=occk.PREC_FP32)
    torch.cuda.synchronize()
    for a, c in zip(Ks, K1):
        assert torch.equal(a, c)
