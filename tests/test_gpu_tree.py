"""The whole tree of a column group in LDS (Eqs. 11-13, 17a-c), on request.

With occk_far_opts.lds_tree set, a chain (a tree split along x whose levels
are unbroken rows of boxes, L = 2) runs every translation of a j batch as
one kernel launch per reflection class of the real components, holding the
tree of a group of columns in LDS.  Each box takes its terms in the order
of the level-by-level passes with FP64 operators and accumulators, so in
FP64 the result equals the walks' bit for bit, and both match the oracle.
The FP32 path keeps its box data in FP32 (the walks' accumulators are FP32
too, so the two differ by rounding only).  Other trees keep the walks and
level passes.
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


def _run(torch, tr, Cd, n, **kw):
    from paper_1708_05353_amd import occk
    K = torch.zeros((Cd.shape[0], n), dtype=torch.float64, device="cuda")
    tr.profile(True)
    tr.profile_read()
    occk.far_K(tr, Cd, K, **kw)
    torch.cuda.synchronize()
    prof = tr.profile_read()
    tr.profile(False)
    return K.cpu().numpy(), prof


@pytest.mark.parametrize("prec", ["fp64", "fp32"])
def test_chain_tree_equals_walks_and_oracle(torch_cuda, prec):
    """Chain along x (four classes): one launch per class and batch, no
    upward launches; FP64 bitwise equal to the walks; both schedules within
    the precision's bound of the oracle.  Ragged last batch, two streams
    (both leaf regions in use) and one stream."""
    from paper_1708_05353_amd import occk
    torch = torch_cuda
    wl = workloads.alkane_chain(n_carbon=40, depth=5)
    C = wl.orbitals()
    n = C.shape[1]
    tr = occk.Tree(wl.system, wl.params)
    Cd = torch.from_numpy(C).cuda()
    code = {"fp64": occk.PREC_FP64, "fp32": occk.PREC_FP32}[prec]
    ref = oracle_far_K(Setup(wl.system, wl.params), C)
    tol = 1e-8 if prec == "fp64" else 1e-6
    for jb in (16, 48):
        nbatch = -(-n // jb)
        for one in (True, False):
            print(f"[tree] chain {prec} jblock {jb} one_stream {one}", flush=True)
            Kt, pt = _run(torch, tr, Cd, n, jblock=jb, precision=code, one_stream=one, lds_tree=True)
            Kw, pw = _run(torch, tr, Cd, n, jblock=jb, precision=code, one_stream=one)
            assert pt["tree"][1] == 4 * nbatch and pt["up"][1] == 0 and pt["down"][1] == 4 * nbatch
            assert pt["up_walk"][1] == pt["down_walk"][1] == 0
            assert pw["tree"][1] == 0 and pw["up_walk"][1] == nbatch
            if prec == "fp64":
                assert np.array_equal(Kt, Kw)
            else:
                assert rel(Kt, Kw) <= 1e-6
            assert rel(Kt, ref) <= tol
    tr.free()


def test_tree_kernel_only_on_chains(torch_cuda):
    """A sheet (reflection classes of the xy plane), a 3-D cluster and a chain
    at L = 4: lds_tree leaves the walks and level passes in place."""
    from paper_1708_05353_amd import occk
    torch = torch_cuda
    for name, wl in (("sheet L2", workloads.graphene_flake(n=2, lmax=2, nocc=12, depth=3)),
                     ("water L2", workloads.water_cluster(15, 43, lmax=2)),
                     ("chain L4", workloads.alkane_chain(n_carbon=20, lmax=4, depth=4))):
        C = wl.orbitals()
        tr = occk.Tree(wl.system, wl.params)
        print(f"[tree] {name}: tree kernel off", flush=True)
        Kt, p = _run(torch, tr, torch.from_numpy(C).cuda(), C.shape[1], lds_tree=True)
        Kw, _ = _run(torch, tr, torch.from_numpy(C).cuda(), C.shape[1])
        tr.free()
        assert p["tree"][1] == 0 and p["down"][1] > 0
        assert np.array_equal(Kt, Kw)
