"""Host logic of bench.py that turns profiles into per-kernel figures: the
kernel of every dispatch of one call (all-column half transform, tree walks
and level passes, direct and mirrored L2P), the algorithmic bytes of the
walks against the level-by-level passes, and the per-kernel cost model
against the per-class one."""
from types import SimpleNamespace

import pytest

import bench


def _info(depth, lmin, ncomp=9, nb=None, il=4):
    nb = nb or [2 ** l for l in range(depth + 1)]
    ilp = [il * nb[l] if l >= lmin else 0 for l in range(depth + 1)]
    return SimpleNamespace(depth=depth, lmin=lmin, ncomp=ncomp, boxes_per_level=nb, m2m_nnz=36,
                           sum_nb=1000, sum_nb2=100000, nleaf=nb[depth], npairs=5000, n_edges=sum(nb[lmin + 1:]),
                           n_il=il * sum(nb[lmin:]), il_per_level=ilp, nbasis=800)


def _call(depth, lmin, nbatch):
    lr_up, lr_dn = bench.walk_roots(_info(depth, lmin))
    seq = ["occk::opgen_kernel", "occk::half_kernel<0>"]      # the all-column half transform first
    for _ in range(nbatch):
        seq += ["occk::half_kernel<0>", "occk::omega_kernel<0>", "occk::up_walk_kernel<double, 9, 6>"]
        seq += ["occk::translate_vec_kernel<double, 9, 1>"] * (lr_up - lmin)
        seq += ["occk::translate_vec_kernel<double, 9, 1>"] * (lr_dn - lmin)
        seq += ["occk::down_walk_kernel<double, 9, 2>", "occk::l2p_wide_kernel<0>", "occk::l2pt_wide_kernel<0>"]
    seq += ["occk::reduce_kernel"]
    return {i + 1: k for i, k in enumerate(seq)}


@pytest.mark.parametrize("depth,lmin", [(8, 2), (4, 2), (3, 2)])
def test_classes_of_walks_and_level_passes(depth, lmin):
    info = _info(depth, lmin)
    lr_up, lr_dn = bench.walk_roots(info)
    names = {0: "occk::opgen_kernel", **_call(depth, lmin, 3)}   # an earlier call's dispatch is ignored
    cls = bench._classify_last_call(names, info)
    got = [cls[i] for i in sorted(cls)]
    per_batch = (["half", "omega", "up_walk"] + ["up_pass"] * (lr_up - lmin) + ["down_pass"] * (lr_dn - lmin)
                 + ["down_walk", "l2p_direct", "l2p_mirror"])
    assert got == ["opgen", "ht"] + per_batch * 3 + ["reduce"]


def test_walk_launch_count_mismatch_is_an_error():
    info = _info(8, 2)
    names = _call(8, 2, 2)
    first_translate = min(i for i, k in names.items() if "translate" in k)
    del names[first_translate]
    with pytest.raises(SystemExit):
        bench._classify_last_call(names, info)


def test_walk_roots_and_bytes():
    info = _info(8, 2)
    assert bench.walk_roots(info) == (2, 7)
    assert bench.walk_roots(_info(8, 2, ncomp=16)) == (None, None)
    assert bench.walk_roots(_info(8, 2, il=40)) == (None, None)          # long interaction lists
    assert bench.walk_roots(_info(4, 2, nb=[1, 4, 16, 64, 256])) == (None, None)   # 4 children per box
    walk = bench.class_costs(info, 100, 32, "fp64")
    nb = info.boxes_per_level
    # upward: leaves read once, every other box written once
    cols = sum(32 * (100 - k * 32) for k in range(4))
    assert walk["up"][1] == (nb[8] + sum(nb[2:8])) * 9 * cols * 8
    # downward: levels 2..6 level by level, then the walk reads sources and
    # its roots' parents and writes the leaves
    lv = sum(2 * nb[l] + (nb[l - 1] if l > 2 else 0) for l in range(2, 7))
    assert walk["down"][1] == (lv + nb[7] + nb[8] + nb[6] + nb[8]) * 9 * cols * 8


def test_classes_of_level_passes_only():
    info = _info(4, 2, il=40)
    seq = ["occk::opgen_kernel", "occk::half_kernel<0>"]
    for _ in range(2):
        seq += ["occk::half_kernel<0>", "occk::omega_kernel<0>"]
        seq += ["occk::translate_vec_kernel<double, 9, 1>"] * 5   # 2 upward, 3 downward levels
        seq += ["occk::l2p_kernel<0>", "occk::l2pt_kernel<0>"]
    cls = bench._classify_last_call({i + 1: k for i, k in enumerate(seq)}, info)
    per_batch = ["half", "omega", "up_pass", "up_pass", "down_pass", "down_pass", "down_pass", "l2p_direct",
                 "l2p_mirror"]
    assert [cls[i] for i in sorted(cls)] == ["opgen", "ht"] + per_batch * 2


@pytest.mark.parametrize("il", [4, 40])
def test_kernel_costs_add_up_to_the_class_costs(il):
    """Walk + level-pass and direct + mirrored figures add up to the class
    figures; the translation flops to the method's F_M2M, F_M2L + F_L2L; the
    two L2P kernels to F_L2P = 2 Q n^2 sum_B n_B."""
    info = _info(8, 2, il=il)
    n, jb = 100, 32
    k = bench.kernel_costs(info, n, jb, "fp64")
    c = bench.class_costs(info, n, jb, "fp64")
    add = lambda a, b, i: k[a][i] + k[b][i]
    assert add("up_walk", "up_pass", 0) == c["up"][0]
    assert add("down_walk", "down_pass", 0) == c["down"][0]
    assert add("l2p_direct", "l2p_mirror", 0) == c["l2p"][0] == 2 * 9 * n * n * info.sum_nb
    for a, b, cl in (("up_walk", "up_pass", "up"), ("down_walk", "down_pass", "down"),
                     ("l2p_direct", "l2p_mirror", "l2p"), ("ht", "half", "half")):
        assert add(a, b, 1) == c[cl][1], cl
    assert k["omega"] == c["omega"]
    assert k["ht"][0] == k["half"][0] == c["half"][0]


def test_best_mixed_mode():
    """The headline mixed mode is the fastest within the 1e-6 budget."""
    import bench
    m = {"fp32": {"ms_per_step": 55.0, "rel_err_vs_fp64": 1.9e-7, "bound": 1e-6},
         "bf16x6": {"ms_per_step": 52.0, "rel_err_vs_fp64": 1.6e-7, "bound": 1e-6},
         "bf16x3": {"ms_per_step": 47.0, "rel_err_vs_fp64": 7.8e-6, "bound": 5e-5}}
    assert bench.best_mixed_mode(m) == "bf16x6"            # BF16x3 is faster but outside the budget
    m["bf16x6"]["rel_err_vs_fp64"] = 2e-6                   # over its bound: not chosen
    assert bench.best_mixed_mode(m) == "fp32"
    m["fp32"]["rel_err_vs_fp64"] = 3e-6
    assert bench.best_mixed_mode(m) == "fp32"               # none qualifies: FP32 is reported
