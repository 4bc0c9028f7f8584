"""Pins for the oracle's tree (Theory section: hierarchy and interaction list)."""
import numpy as np
import pytest

import workloads
from oracle.basis import Functions, function_pairs
from oracle.tree import Tree


def test_tiny_chain_counts(tiny):
    wl, C, st = tiny
    t = st.tree
    assert t.lo[0] == pytest.approx(-1.015)
    assert t.h(3) == pytest.approx(5.1125)
    assert len(t.boxes[3]) == 8
    # leaf-level near pairs: 3,4,5,5,5,5,4,3
    near = sum(1 for a in t.boxes[3] for b in t.boxes[3] if t.near(a, b))
    assert near == 34
    per_level = [sum(len(x) for x in t.il[l]) for l in range(4)]
    assert per_level == [0, 0, 2, 22]
    assert t.lmin == 2
    # atoms per leaf 3,2,3,2,3,2,3,2 (s-s same-atom pairs sit on the atom)
    xs = wl.system.xyz[:, 0]
    counts = np.bincount(np.floor((xs - t.lo[0]) / t.h(3)).astype(int), minlength=8)
    assert counts.tolist() == [3, 2, 3, 2, 3, 2, 3, 2]


def _partition_check(t):
    nl = len(t.boxes[t.depth])
    far = 0
    for b1 in range(nl):
        for b2 in range(nl):
            hits = 0
            for lev in range(1, t.depth + 1):
                a, b = t.ancestor(lev, b1), t.ancestor(lev, b2)
                if b in t.il[lev][a]:
                    hits += 1
            near = t.near(t.boxes[t.depth][b1], t.boxes[t.depth][b2])
            assert hits == (0 if near else 1)
            far += hits
    return far


@pytest.mark.parametrize("maker", ["sheet", "water"])
def test_partition_invariant(maker):
    """Every ordered leaf pair is near at the leaf level or lies in exactly one
    interaction list at exactly one level."""
    if maker == "sheet":
        wl = workloads.graphene_flake(n=3, nocc=20, depth=4)
    else:
        wl = workloads.water_cluster(20, 40)
    fn = Functions(wl.system)
    r, s, P = function_pairs(wl.system, fn, wl.params.pair_log_thresh)
    p = wl.params
    t = Tree(P, p.split_mask, p.depth, p.ws)
    assert _partition_check(t) > 0
    # the interaction list relation is symmetric
    for lev in range(t.depth + 1):
        for b, lst in enumerate(t.il[lev]):
            for b2 in lst:
                assert b in t.il[lev][b2]


def test_boundary_tie_rejected():
    c = np.array([[0.0, 0, 0], [10.0, 0, 0]])
    # lo = -0.35*(0.05*10+1) = -0.525, W = 11.5, h(depth 1) = 5.75 -> boundary at 5.225
    c2 = np.vstack([c, [[5.225, 0, 0]]])
    with pytest.raises(ValueError):
        Tree(c2, 1, 1, 0)


# ---------------------------------------------------------------------------
# the extent rule (near/far by the extents of the charge distributions)

def _extent_tree(wl, ws=0.0, tau=1e-8):
    from scipy.special import erfcinv
    fn = Functions(wl.system)
    r, s, P = function_pairs(wl.system, fn, wl.params.pair_log_thresh)
    ext = erfcinv(tau) / np.sqrt(fn.exp[r] + fn.exp[s])
    p = wl.params
    return Tree(P, p.split_mask, p.depth, ws, extents=ext), P, ext


@pytest.mark.parametrize("maker,ws", [("sheet", 0.0), ("sheet", -0.1), ("water", 0.0), ("chain", 0.5)])
def test_extent_rule_partition_and_symmetry(maker, ws):
    """Every ordered leaf pair is in the leaf-level near list or in exactly one
    interaction list at one level; both relations are symmetric."""
    wl = {"sheet": lambda: workloads.graphene_flake(n=3, nocc=20, depth=4),
          "water": lambda: workloads.water_cluster(20, 40),
          "chain": lambda: workloads.alkane_chain(n_carbon=40, depth=5)}[maker]()
    t, P, ext = _extent_tree(wl, ws)
    nl = len(t.boxes[t.depth])
    far = 0
    for b1 in range(nl):
        for b2 in range(nl):
            hits = sum(1 for lev in range(1, t.depth + 1)
                       if t.ancestor(lev, b2) in t.il[lev][t.ancestor(lev, b1)])
            near = b2 in t.near_list[t.depth][b1]
            assert hits == (0 if near else 1), (b1, b2)
            far += hits
    assert far > 0
    for lev in range(t.depth + 1):
        for b, lst in enumerate(t.il[lev]):
            for b2 in lst:
                assert b in t.il[lev][b2]


@pytest.mark.parametrize("maker", ["tiny", "water"])
def test_extent_rule_separates_every_far_distribution_pair(maker):
    """The point of the extents: for boxes A, B in each other's interaction
    list (ws >= 0), every distribution k in A and k' in B has
    |P_k - P_k'| > e_k + e_k', so its s-type penetration erfc stays below tau
    (brute force over all distribution pairs)."""
    wl = {"tiny": workloads.tiny_chain, "water": lambda: workloads.water_cluster(8, 41, depth=2)}[maker]()
    t, P, ext = _extent_tree(wl, 0.0)
    D = t.depth
    checked = 0
    for lev in range(1, D + 1):
        sh = D - lev
        box_of = np.array([t.index[lev][tuple(int(v) >> sh for v in c)] for c in t.pair_leaf_coord])
        members = [np.nonzero(box_of == b)[0] for b in range(len(t.boxes[lev]))]
        for a, lst in enumerate(t.il[lev]):
            for b in lst:
                ka, kb = members[a], members[b]
                d = np.linalg.norm(P[ka][:, None, :] - P[kb][None, :, :], axis=-1)
                assert np.all(d > ext[ka][:, None] + ext[kb][None, :])
                checked += d.size
    assert checked > 0


def test_extent_rule_bounds_the_penetration(tiny):
    """s-type chain with the extent rule at tau = 1e-8: the exact (Boys F0) far
    field and its point-charge limit differ by far less than with the box
    rule, whose far pairs include overlapping diffuse distributions."""
    from conftest import rel, with_params
    from oracle.exact import far_K_exact_s
    from oracle.fmm import Setup
    wl, C, st = tiny
    ste = Setup(wl.system, with_params(wl, near_rule=1, ext_ws=0.0, ext_tau=1e-8))
    assert ste.tree.lmin is not None
    pen_ext = rel(far_K_exact_s(ste, C, "pc"), far_K_exact_s(ste, C, "exact"))
    pen_box = rel(far_K_exact_s(st, C, "pc"), far_K_exact_s(st, C, "exact"))
    assert pen_ext < 1e-7 and pen_box > 100 * pen_ext
