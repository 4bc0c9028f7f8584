"""Which schedule runs the translations: subtree walks on chain-like trees
(binary splits, short interaction lists), level-by-level passes elsewhere.
The library's launch counts per call must match bench.walk_roots, which
prices and classifies the profiles with the same rule."""
import pytest

import bench
import workloads

pytestmark = pytest.mark.gpu


def _launches(wl, jblock):
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_1708_05353_amd import occk
    tr = occk.Tree(wl.system, wl.params)
    info = tr.info
    C = torch.from_numpy(wl.orbitals()).cuda()
    K = torch.zeros((wl.system.nbasis, C.shape[1]), dtype=torch.float64, device="cuda")
    tr.profile(True)
    tr.profile_read()
    occk.far_K(tr, C, K, jblock=jblock)
    torch.cuda.synchronize()
    prof = tr.profile_read()
    tr.profile(False)
    tr.free()
    nbatch = -(-C.shape[1] // jblock)
    # single-kernel scopes nested in their classes: one walk per batch when
    # walks run, one direct L2P per batch, and their times within the class
    walks = prof["up_walk"][1] > 0
    assert prof["up_walk"][1] == prof["down_walk"][1] == (nbatch if walks else 0)
    assert prof["l2p_direct"][1] == nbatch and prof["ht"][1] == 1
    for sub, cls in (("up_walk", "up"), ("down_walk", "down"), ("l2p_direct", "l2p"), ("l2p_mirror", "l2p"),
                     ("ht", "half")):
        assert prof[sub][0] <= prof[cls][0] * 1.0001 + 1e-3, (sub, prof[sub], prof[cls])
    return info, prof["up"][1] // nbatch, prof["down"][1] // nbatch, prof["up"][1] % nbatch


@pytest.mark.parametrize("name", ["alkane_C100", "water75", "graphene"])
def test_schedule_matches_bench_rule(name):
    wl = {"alkane_C100": lambda: workloads.alkane_chain(n_carbon=100, depth=6),
          "water75": lambda: workloads.water_cluster(15, 43, lmax=2),
          "graphene": lambda: workloads.graphene_flake(lmax=2)}[name]()
    print(f"[walks] {name}", flush=True)
    info, up, down, rest = _launches(wl, 64)
    assert rest == 0
    lr_up, lr_dn = bench.walk_roots(info)
    D, lmin = info.depth, info.lmin
    if name == "alkane_C100":
        assert lr_up is not None and lr_dn is not None
    else:
        assert lr_up is None and lr_dn is None
    if lr_up is None:
        assert (up, down) == (D - lmin, D - lmin + 1)
    else:
        assert (up, down) == (1 + lr_up - lmin, lr_dn - lmin + 1)


def _real_class(q, sym):
    """Class of real component q (l^2 + 0: (l,0); odd offsets Re, even Im):
    sym 1 (x-axis displacements) by Im-ness and l+m parity, sym 2 (xy plane)
    by l+m parity."""
    l = int(q ** 0.5)
    while (l + 1) * (l + 1) <= q:
        l += 1
    while l * l > q:
        l -= 1
    k = q - l * l
    m, im = (k + 1) // 2, int(k != 0 and k % 2 == 0)
    return 2 * im + ((l + m) & 1) if sym == 1 else ((l + m) & 1)


@pytest.mark.parametrize("name,sym,L", [("chain", 1, 2), ("chain", 1, 4), ("sheet", 2, 2), ("sheet", 2, 4)])
def test_generated_operators_have_the_structural_zeros(name, sym, L):
    """The library skips the operator entries that the displacements' axis
    symmetry makes zero (x axis on chains, xy plane on sheets): every such
    entry of the generated FP64 operators (fragment order, T[r][c] at
    ((r/16) KS + c/4) 64 + r%16 + 16 (c%4)) is exactly zero."""
    import numpy as np
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_1708_05353_amd import occk
    if name == "chain":
        wl = workloads.alkane_chain(n_carbon=40, lmax=L, depth=5)
    else:
        wl = workloads.graphene_flake(n=2, lmax=L, nocc=12, depth=3)
    tr = occk.Tree(wl.system, wl.params)
    C = torch.from_numpy(wl.orbitals()).cuda()
    K = torch.zeros((wl.system.nbasis, C.shape[1]), dtype=torch.float64, device="cuda")
    occk.far_K(tr, C, K)
    torch.cuda.synchronize()
    ops = tr.debug_buffer(0)
    tr.free()
    Q = (L + 1) ** 2
    MT, KS = (Q + 15) // 16, (Q + 3) // 4
    ops = ops.reshape(-1, MT * KS * 64)
    r, c = np.meshgrid(np.arange(Q), np.arange(Q), indexing="ij")
    pos = ((r // 16) * KS + c // 4) * 64 + r % 16 + 16 * (c % 4)
    T = ops[:, pos]                                   # (nops, Q, Q)
    cls = np.array([_real_class(q, sym) for q in range(Q)])
    dead = cls[:, None] != cls[None, :]
    assert np.all(T[:, dead] == 0.0)
    assert np.count_nonzero(T[:, ~dead]) > 0.5 * T[:, ~dead].size
    print(f"[opsym] {name} L={L}: {ops.shape[0]} operators, {int((~dead).sum())} of {Q * Q} entries live", flush=True)
