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
