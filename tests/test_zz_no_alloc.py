"""occk_far_K_noalloc (workspace in the library's fixed scratch region)
against occk_far_K on the same inputs: two calls in a row, the second on a
smaller system, each compared with the allocating entry point (FP64 gate of
1e-12 normwise: the same kernels run, only the workspace placement differs)
and with the oracle (1e-8).  Also: ESTATE before the tree's device copy
exists, ENOMEM for a workspace beyond the region, and the allocating entry
point's workspace left untouched."""
import numpy as np
import pytest

import workloads
from oracle.fmm import Setup, far_K as oracle_far_K

from conftest import rel

pytestmark = pytest.mark.gpu


def _case(wl):
    import torch
    from paper_1708_05353_amd import occk
    C = wl.orbitals()
    tr = occk.Tree(wl.system, wl.params)
    Cd = torch.from_numpy(C).cuda()
    n = C.shape[1]
    Kr = torch.zeros((wl.system.nbasis, n), dtype=torch.float64, device="cuda")
    return C, tr, Cd, Kr


def test_noalloc_matches_far_K_twice():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_1708_05353_amd import occk
    big = workloads.water_cluster(20, 40)
    small = workloads.tiny_chain()
    results = []
    for wl in (big, small):                       # second call: smaller input
        C, tr, Cd, Kref = _case(wl)
        Kn = torch.full_like(Kref, 3.0)
        with pytest.raises(occk.OcckError) as e:   # no device copy of the tree yet
            occk.far_K_noalloc(tr, Cd, Kn)
        assert e.value.code == occk.ESTATE
        occk.far_K(tr, Cd, Kref)
        torch.cuda.synchronize()
        jb_before = tr.workspace_jblock()
        print(f"[noalloc] {wl.system.name}: nbasis {wl.system.nbasis} nocc {C.shape[1]}", flush=True)
        occk.far_K_noalloc(tr, Cd, Kn)
        torch.cuda.synchronize()
        a, b = Kn.cpu().numpy(), Kref.cpu().numpy()
        assert rel(a, b) <= 1e-12, rel(a, b)
        ref = oracle_far_K(Setup(wl.system, wl.params), C)
        assert rel(a, ref) <= 1e-8
        assert tr.workspace_jblock() == jb_before     # the handle's own workspace is untouched
        # a sub-range and accumulate, like occk_far_K
        n = C.shape[1]
        Ks = Kn.clone()
        occk.far_K_noalloc(tr, Cd, Ks, i_range=(1, n - 2), j_range=(2, n - 1), accumulate=True)
        Kr2 = Kref.clone()
        occk.far_K(tr, Cd, Kr2, i_range=(1, n - 2), j_range=(2, n - 1), accumulate=True)
        torch.cuda.synchronize()
        assert rel(Ks.cpu().numpy(), Kr2.cpu().numpy()) <= 1e-12
        # the allocating entry point still works on its own workspace
        Kr3 = torch.zeros_like(Kref)
        occk.far_K(tr, Cd, Kr3)
        torch.cuda.synchronize()
        assert np.array_equal(Kr3.cpu().numpy(), b)
        results.append(rel(a, ref))
        tr.free()
    print("[noalloc] errors vs oracle", results, flush=True)


def test_noalloc_rejects_workspace_beyond_the_region():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_1708_05353_amd import occk
    wl = workloads.water_cluster(100, 55)
    C, tr, Cd, Kref = _case(wl)
    occk.far_K(tr, Cd, Kref, i_range=(0, 4), j_range=(0, 4))
    torch.cuda.synchronize()
    Kn = torch.zeros_like(Kref)
    with pytest.raises(occk.OcckError) as e:       # 256 j columns in one batch: gigabytes of box data
        occk.far_K_noalloc(tr, Cd, Kn, jblock=256)
    assert e.value.code == occk.ENOMEM and "scratch" in str(e.value)
    occk.far_K_noalloc(tr, Cd, Kn, i_range=(0, 4), j_range=(0, 4))   # a small slice fits
    torch.cuda.synchronize()
    assert rel(Kn[:, :4].cpu().numpy(), Kref[:, :4].cpu().numpy()) <= 1e-12
    tr.free()
