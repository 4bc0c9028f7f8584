"""Mixed-precision paths against the FP64 oracle on small inputs.

FP32: every contraction on FP32 MFMA with FP32 operands and accumulation.
BF16X6: the half transform, Omega and L2P contractions as three-way split-BF16
products (six MFMAs) with FP32 accumulation; translations on FP32 MFMA.
BF16X3: two-way split, three products: about 2^-16 per product, so it does
not meet 1e-6; its stated bound is 5e-5.
Operators are generated in FP64 and K partials accumulate in FP64 in all.
Gate: max|dK| / max|K| <= 1e-6 (FP32, BF16X6), <= 5e-5 (BF16X3).
"""
import numpy as np
import pytest

import workloads
from oracle.fmm import Setup, far_K as oracle_far_K

from conftest import rel, with_params

pytestmark = pytest.mark.gpu

TOL = {1: 1e-6, 2: 5e-5, 3: 1e-6}
PRECS = [1, 2, 3]
IDS = ["fp32", "bf16x3", "bf16x6"]


def _gpu(wl, C, prec, params=None, **kw):
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_1708_05353_amd import occk
    tr = occk.Tree(wl.system, params or wl.params)
    K = torch.zeros((wl.system.nbasis, C.shape[1]), dtype=torch.float64, device="cuda")
    occk.far_K(tr, torch.from_numpy(C).cuda(), K, precision=prec, **kw)
    torch.cuda.synchronize()
    out = K.cpu().numpy()
    tr.free()
    return out


@pytest.mark.parametrize("prec", PRECS, ids=IDS)
@pytest.mark.parametrize("L", [2, 5, 8])
def test_tiny_chain(tiny, prec, L):
    wl, C, st = tiny
    p = with_params(wl, lmax=L)
    st = st if L == 2 else Setup(wl.system, p)
    ref = oracle_far_K(st, C)
    e = rel(_gpu(wl, C, prec, params=p), ref)
    print(f"tiny chain L={L} prec={prec}: {e:.3e}")
    assert e <= TOL[prec]


@pytest.mark.parametrize("prec", PRECS, ids=IDS)
def test_sheet_ranges(prec):
    wl = workloads.graphene_flake(n=2, lmax=3, nocc=12, depth=3)
    C = wl.orbitals()
    st = Setup(wl.system, wl.params)
    ref = oracle_far_K(st, C, i_range=(2, 10), j_range=(1, 12))
    got = _gpu(wl, C, prec, i_range=(2, 10), j_range=(1, 12), jblock=4)
    e = rel(got[:, 2:10], ref)
    print(f"sheet prec={prec}: {e:.3e}")
    assert e <= TOL[prec]


@pytest.mark.parametrize("prec", PRECS, ids=IDS)
def test_mixed_reproducible(prec):
    wl = workloads.water_cluster(20, 41)
    C = wl.orbitals()
    a = _gpu(wl, C, prec, jblock=16)
    b = _gpu(wl, C, prec, jblock=16)
    assert np.array_equal(a, b)
