"""Far-field occupied exchange throughput on one MI355X.

One step = one occk_far_K call: the whole hot path (operator generation,
half and full MO transforms, upward / interaction-list / downward
translations, L2P and the K reduction) for all occupied i and j, on the
alkane-chain workload (C400H802 stand-in: nbasis 9610, nocc 1601, 1-D tree of
depth 8, ws 2, L = 2), inputs resident in HBM.  Prints one JSON line.

value = algorithmic flops of one call / measured time (GFLOP/s), in the
library's default schedule (the L2P of a j batch on a second stream,
overlapping the next batch's translations).  The kernels and the roofline
object come from the same calls timed again in the one-stream schedule, where
every kernel runs alone, with HIP events on the library's stream (the
kernel with the largest time per call is the roofline's).  The "mixed"
object times the FP32, split-BF16x6 and split-BF16x3 paths on the same
inputs, gives each one's error against the FP64 result, and heads with the
fastest mode within the 1e-6 budget (BF16x3 is held to 5e-5).  hbm_copy is the rate of a plain device copy on the box.
cpu_baseline times the FP64 oracle on a bounded j sample of the same
workload and scales it linearly in the number of j columns.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

PEAK_FLOPS = {"fp64": 78.6e12, "fp32": 157.3e12, "bf16x3": 2.5e15 / 3.0, "bf16x6": 2.5e15 / 6.0}
PEAK_HBM = 8.0e12
ELEM_BYTES = {"fp64": 8, "fp32": 4, "bf16x3": 4, "bf16x6": 4}


# Register levels of the library's tree walks (kUpWalkLevels and
# kDownWalkLevels in csrc/kernels.hpp): the walks start at these levels.
UP_WALK_LEVELS, DOWN_WALK_LEVELS = 6, 2


def walk_roots(info):
    """Root levels of the upward and downward walks (None: level passes only).
    As in the library: walks for Q <= 9 on trees whose boxes above the
    leaves have at most 2 children on average and whose interaction lists
    hold at most 8 sources on average."""
    D, lmin = info.depth, info.lmin
    nb = info.boxes_per_level
    above, kids, tgt = sum(nb[lmin:D]), sum(nb[lmin + 1:D + 1]), sum(nb[lmin:D + 1])
    if info.ncomp > 9 or kids > 2 * above or info.n_il > 8 * tgt:
        return None, None
    lr_up = max(lmin, D - UP_WALK_LEVELS) if D - lmin >= 1 else None
    lr_dn = max(lmin, D + 1 - DOWN_WALK_LEVELS)
    return lr_up, lr_dn


def class_costs(info, n, jb, prec, tree=False):
    """Algorithmic flops and bytes per call of each kernel class, for the full
    call (i and j over all n occupied orbitals, symmetric schedule).

    Flops are the method's counts with the (i, j) symmetry of Omega and Mloc
    used: n_c = n(n+1)/2 translated columns, F_Omega = Q n(n+1) sum_B n_B,
    F_L2P = 2 Q n^2 sum_B n_B, F_half = 2 Q n sum_B pi_B.  Bytes are the
    compulsory traffic of the schedule as executed: batch k (first j at
    k*jb) carries jb*(n - k*jb) columns; every box it touches is read once
    and written once per batch (the upward walk reads the leaves and writes
    the other boxes), operands of the GEMMs are read once.  tree: the
    in-LDS tree kernel runs every translation of a batch in the "down" class,
    reading the leaf multipoles and writing the leaf local expansions once."""
    Q = info.ncomp
    s = ELEM_BYTES[prec]
    nb = info.boxes_per_level
    lmin, D = info.lmin, info.depth
    nblk = -(-n // jb)
    nks = [n - k * jb for k in range(nblk)]          # carried i per batch
    nc_exec = sum(jb * nk for nk in nks)
    nc = n * (n + 1) // 2
    lr_up, lr_dn = walk_roots(info)
    if lr_up is not None:   # level passes above the walk's roots; the walk reads leaves, writes the rest
        up_boxes = (sum(nb[l] + nb[l + 1] for l in range(lmin, lr_up)) + nb[D]
                    + sum(nb[l] for l in range(lr_up, D)))
    else:                   # level by level: children read, parent written per level
        up_boxes = sum(nb[l] + nb[l + 1] for l in range(lmin, D))
    if lr_dn is not None:   # level passes above; the walk reads sources and its roots' parents, writes leaves
        down_boxes = (sum(2 * nb[l] + (nb[l - 1] if l > lmin else 0) for l in range(lmin, lr_dn))
                      + sum(nb[l] for l in range(lr_dn, D + 1)) + (nb[lr_dn - 1] if lr_dn > lmin else 0)
                      + nb[D])
    else:
        down_boxes = sum(2 * nb[l] + (nb[l - 1] if l > lmin else 0) for l in range(lmin, D + 1))
    z = info.m2m_nnz
    if tree:
        up_boxes, down_boxes = 0, 2 * nb[D]
    snb, snb2, nleaf = info.sum_nb, info.sum_nb2, info.nleaf
    half_b = (nblk * (snb2 * Q + snb * jb * (1 + Q)) + snb2 * Q + snb * n * (1 + Q)) * s
    omega_b = sum(snb * Q * jb + snb * nk + nleaf * Q * jb * nk for nk in nks) * s
    l2p_b = sum((nleaf * Q * jb * nk + nleaf * Q * jb * max(0, nk - jb) + snb * Q * max(0, nk - jb)) * s
                + (snb * nk + 2 * snb * jb) * 8 for nk in nks)
    return {
        "half": (2 * Q * info.npairs * n, half_b),
        "omega": (Q * n * (n + 1) * snb, omega_b),
        "up": (0 if tree else 2 * z * nc * info.n_edges, up_boxes * Q * nc_exec * s),
        "down": (2 * Q * Q * nc * info.n_il + 2 * z * nc * info.n_edges * (2 if tree else 1),
                 down_boxes * Q * nc_exec * s),
        "l2p": (2 * Q * n * n * snb, l2p_b),
        "reduce": (0, (snb * n + info.nbasis * n) * 8),
    }


# kernel -> profile class of the library (occk.KERNEL_CLASSES) whose HIP-event
# time is that kernel's; "half", "up_pass", "down_pass" are a class minus its
# nested single-kernel class
KERNELS = ["ht", "half", "omega", "up_walk", "up_pass", "down_walk", "down_pass", "tree", "l2p_direct", "l2p_mirror",
           "reduce"]
TRANSLATION_KERNELS = ("up_walk", "up_pass", "down_walk", "down_pass", "tree")


def kernel_times(prof):
    """ms and launches of each kernel from the per-class profile."""
    def sub(a, b):
        return (prof[a][0] - prof[b][0], prof[a][1] - prof[b][1])
    return {"ht": prof["ht"], "half": sub("half", "ht"), "omega": prof["omega"],
            "up_walk": prof["up_walk"], "up_pass": sub("up", "up_walk"),
            "down_walk": prof["down_walk"],
            "down_pass": (prof["down"][0] - prof["down_walk"][0] - prof["tree"][0],
                          prof["down"][1] - prof["down_walk"][1] - prof["tree"][1]),
            "tree": prof["tree"],
            "l2p_direct": prof["l2p_direct"], "l2p_mirror": prof["l2p_mirror"], "reduce": prof["reduce"]}


def _real_class(q, sym):
    """Class of real component q under the reflections that fix an
    axis-aligned displacement (the library's real_class): sym 1 (x axis) by
    Im-ness and l+m parity, sym 2 (xy plane) by l+m parity, sym 0 one class."""
    l = 0
    while (l + 1) * (l + 1) <= q:
        l += 1
    k = q - l * l
    m, im = (k + 1) // 2, int(k != 0 and k % 2 == 0)
    return (2 * im + ((l + m) & 1)) if sym == 1 else ((l + m) & 1) if sym == 2 else 0


def translation_live_entries(Q, split_mask):
    """Operator entries the vector translations multiply (L <= 2): every
    displacement of a tree split along x only lies on the x axis (sym 1), of
    a tree not split along z in the xy plane (sym 2); the entries joining
    different reflection classes are exact zeros and are skipped."""
    sym = 1 if split_mask == 1 else 2 if not (split_mask & 4) else 0
    if Q > 9:
        sym = 0      # the MFMA translations multiply the whole operator
    cls = [_real_class(q, sym) for q in range(Q)]
    return sum(1 for i in range(Q) for k in range(Q) if cls[i] == cls[k])


def kernel_costs(info, n, jb, prec, tree=False):
    """Algorithmic flops and bytes per call of each kernel of the full
    symmetric call (i and j over all n orbitals).

    Flops: the method's counts with n_c = n(n+1)/2 translated columns, split
    by the levels each kernel covers; the half transform F_half = 2 Q n
    sum_B pi_B is the method's once, and both its launches (all columns for
    the mirrored L2P, then per j batch) are priced with it, so their sum is
    twice the method's; the L2P's 2 Q n^2 sum_B n_B splits into the column
    pairs the direct contraction covers (j in the batch, i from the batch's
    first j on) and the mirrored rest.  Bytes: the compulsory traffic of the
    schedule as executed (every box a kernel touches read or written once per
    batch, GEMM operands once), as in class_costs.  tree: the in-LDS tree
    kernel takes every translation (one launch per reflection class), its
    bytes one read of the leaf multipoles and one write of the leaf local
    expansions per batch."""
    Q = info.ncomp
    s = ELEM_BYTES[prec]
    nb, il = info.boxes_per_level, info.il_per_level
    lmin, D = info.lmin, info.depth
    nblk = -(-n // jb)
    nks = [n - k * jb for k in range(nblk)]
    nc_exec = sum(jb * nk for nk in nks)
    nc = n * (n + 1) // 2
    z = info.m2m_nnz
    snb, snb2, nleaf = info.sum_nb, info.sum_nb2, info.nleaf
    lr_up, lr_dn = walk_roots(info)
    if lr_up is None:
        lr_up = D
    if lr_dn is None:
        lr_dn = D + 1
    f_up = lambda a, b: 2 * z * nc * sum(nb[l] for l in range(a, b))              # children at levels [a, b)
    f_m2l = lambda a, b: 2 * Q * Q * nc * sum(il[l] for l in range(a, b))
    f_l2l = lambda a, b: 2 * z * nc * sum(nb[l] for l in range(max(a, lmin + 1), b))
    up_walk_boxes = (nb[D] + sum(nb[l] for l in range(lr_up, D))) if lr_up < D else 0
    up_pass_boxes = sum(nb[l] + nb[l + 1] for l in range(lmin, lr_up))
    dn_pass_boxes = sum(2 * nb[l] + (nb[l - 1] if l > lmin else 0) for l in range(lmin, min(lr_dn, D + 1)))
    dn_walk_boxes = ((sum(nb[l] for l in range(lr_dn, D + 1)) + (nb[lr_dn - 1] if lr_dn > lmin else 0) + nb[D])
                     if lr_dn <= D else 0)
    f_half = 2 * Q * info.npairs * n
    f_tree = f_up(lmin + 1, D + 1) + f_m2l(lmin, D + 1) + f_l2l(lmin, D + 1)
    out = {
        "ht": (f_half, (snb2 * Q + snb * n * (1 + Q)) * s),
        "half": (f_half, nblk * (snb2 * Q + snb * jb * (1 + Q)) * s),
        "omega": (Q * n * (n + 1) * snb, sum(snb * Q * jb + snb * nk + nleaf * Q * jb * nk for nk in nks) * s),
        "up_walk": (f_up(lr_up + 1, D + 1), up_walk_boxes * Q * nc_exec * s),
        "up_pass": (f_up(lmin + 1, lr_up + 1), up_pass_boxes * Q * nc_exec * s),
        "down_walk": (f_m2l(lr_dn, D + 1) + f_l2l(lr_dn, D + 1), dn_walk_boxes * Q * nc_exec * s),
        "down_pass": (f_m2l(lmin, lr_dn) + f_l2l(lmin, lr_dn), dn_pass_boxes * Q * nc_exec * s),
        "tree": (0, 0),
        "l2p_direct": (2 * Q * snb * nc_exec, sum(nleaf * Q * jb * nk * s + snb * nk * 8 for nk in nks)),
        "l2p_mirror": (2 * Q * snb * (n * n - nc_exec),
                       sum((nleaf * Q * jb * max(0, nk - jb) + snb * Q * max(0, nk - jb)) * s + 2 * snb * jb * 8
                           for nk in nks)),
        "reduce": (0, (snb * n + info.nbasis * n) * 8),
    }
    if tree:
        for k in ("up_walk", "up_pass", "down_walk", "down_pass"):
            out[k] = (0, 0)
        out["tree"] = (f_tree, 2 * nb[D] * Q * nc_exec * s)
    return out


def bench_coulomb(wl, Cd, args, stream):
    """Far-field Coulomb J^ff of the same workload at the paper's Coulomb rank
    L^J = 10 (occk_far_J, FP64): the density D = 2 C C^T resident in HBM,
    one call per step.  The path streams the pair multipoles twice (density
    contraction, then J from the local expansions), so its roofline is HBM:
    algorithmic bytes = 8 (2 Q npairs + 2 npairs + nbasis^2), the pair
    multipoles read twice, D read and J written at the pairs, J cleared."""
    import copy
    import torch
    from paper_1708_05353_amd import occk
    p = copy.copy(wl.params)
    p.lmax = 10
    t0 = time.perf_counter()
    tree = occk.Tree(wl.system, p)
    t_tree = time.perf_counter() - t0
    D = 2.0 * (Cd @ Cd.T)
    J = torch.zeros_like(D)
    call = lambda: occk.far_J(tree, D, J, stream=stream)
    t0 = time.perf_counter()
    call()                       # uploads the pair multipoles and the tables
    torch.cuda.synchronize()
    t_first = time.perf_counter() - t0
    for _ in range(args.warmup):
        call()
    torch.cuda.synchronize()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record(stream)
    for _ in range(args.steps):
        call()
    e1.record(stream)
    torch.cuda.synchronize()
    ms = e0.elapsed_time(e1) / args.steps
    fl = tree.flops_J()
    inf = tree.info
    Q, npairs, n = inf.ncomp, inf.npairs, inf.nbasis
    alg = 8 * (2 * Q * npairs + 2 * npairs + n * n)
    tree.free()
    return {"workload": f"the same chain at L^J=10 (Q {Q}, {npairs} screened pairs)", "ms_per_step": round(ms, 3),
            "GFLOP/s": round(fl["total"] / (ms * 1e-3) / 1e9, 1), "flops_per_step": fl["total"],
            "roofline": {"bound": "hbm", "achieved": round(alg / (ms * 1e-3) / 1e9, 1), "peak": PEAK_HBM / 1e9,
                         "unit": "GB/s", "frac": round(alg / (ms * 1e-3) / PEAK_HBM, 4), "alg_bytes": alg,
                         "kernel": "the whole call (about 20 launches)"},
            "tree_build_s": round(t_tree, 2), "first_call_s": round(t_first, 2)}


def bench_near(wl, Cd, args, stream):
    """Near-field exchange of the same workload with exact s/p integrals
    (occk_near_K, FP64): the near leaf pairs of the tree, all occupied
    orbitals, one call per step.  Reported: time, shell quartets per second,
    and the two dense GEMMs (D = 2 C C^T, K = X C) that bracket the integrals."""
    import torch
    from paper_1708_05353_amd import occk
    tree = occk.Tree(wl.system, wl.params)
    K = torch.zeros((wl.system.nbasis, Cd.shape[1]), dtype=torch.float64, device=Cd.device)
    call = lambda: occk.near_K(tree, Cd, K, stream=stream)
    t0 = time.perf_counter()
    call()                       # builds the shell-pair tables
    torch.cuda.synchronize()
    t_first = time.perf_counter() - t0
    for _ in range(args.warmup):
        call()
    torch.cuda.synchronize()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record(stream)
    for _ in range(args.steps):
        call()
    e1.record(stream)
    torch.cuda.synchronize()
    ms = e0.elapsed_time(e1) / args.steps
    tasks, quartets = occk.near_info(tree)
    n, no = wl.system.nbasis, Cd.shape[1]
    gemm = 2 * 2 * n * n * no
    tree.free()
    return {"ms_per_step": round(ms, 3), "shell_quartets": quartets, "wave_tasks": tasks,
            "Gquartets/s": round(quartets / (ms * 1e-3) / 1e9, 2), "gemm_flops": gemm,
            "first_call_s": round(t_first, 2)}


def best_mixed_mode(mixed: dict, budget: float = 1e-6) -> str:
    """The headline mixed mode: the fastest one whose stated bound is within
    the mixed path's budget and whose measured error meets it (BF16x3, held
    to 5e-5, never qualifies); FP32 when none does."""
    ok = [m for m, r in mixed.items() if r["bound"] <= budget and r["rel_err_vs_fp64"] <= r["bound"]]
    return min(ok, key=lambda m: mixed[m]["ms_per_step"]) if ok else "fp32"


def cpu_model() -> str:
    """CPU model name of the host (lscpu, else /proc/cpuinfo)."""
    import subprocess
    try:
        out = subprocess.run(["lscpu"], capture_output=True, text=True, timeout=10).stdout
        for line in out.splitlines():
            if line.startswith("Model name:"):
                return line.split(":", 1)[1].strip()
    except (OSError, subprocess.SubprocessError):
        pass
    try:
        with open("/proc/cpuinfo") as fh:
            for line in fh:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def cpu_baseline(wl, C, flops_total, nocc, jsample, repeats):
    """The FP64 oracle on the host cores: far_K for all i and j in [0, jsample),
    best of `repeats` runs, scaled linearly to all nocc j columns (the oracle's
    cost is linear in the summed j columns)."""
    from oracle.fmm import Setup, far_K as oracle_far_K
    try:
        from threadpoolctl import threadpool_info
        threads = max([p.get("num_threads", 1) for p in threadpool_info()] or [1])
    except Exception:
        threads = len(os.sched_getaffinity(0))
    t0 = time.perf_counter()
    st = Setup(wl.system, wl.params)
    t_setup = time.perf_counter() - t0
    times = []
    for _ in range(repeats):
        t0 = time.perf_counter()
        oracle_far_K(st, C, j_range=(0, jsample), jblock=jsample)
        times.append(time.perf_counter() - t0)
    t = min(times)
    t_full = t * nocc / jsample
    return {"value": round(flops_total / t_full / 1e9, 4), "unit": "GFLOP/s", "cores": int(threads),
            "kind": "oracle", "cpu_model": cpu_model(),
            "sample": f"oracle far_K for all i and j in [0,{jsample}) of {nocc}: best of {repeats} runs "
                      f"({', '.join(f'{x:.1f}' for x in times)} s), scaled x{nocc / jsample:.1f} (cost is linear in "
                      f"the j columns); oracle setup {t_setup:.0f} s excluded, as the tree build is excluded on the GPU"}


def bench_batch(args):
    """16 water clusters of 20..100 molecules: one tuned persistent launch vs 16
    separate occk_far_K launches of the same precision vs 16 plain FP64 ones."""
    import torch

    import workloads
    from paper_1708_05353_amd import occk

    prec_name = args.precision if args.precision != "fp64" else "fp32"
    prec = {"fp32": occk.PREC_FP32, "bf16x3": occk.PREC_BF16X3, "bf16x6": occk.PREC_BF16X6}[prec_name]
    wls = workloads.water_batch()
    trees, Cs, Ks, flops = [], [], [], 0
    for wl in wls:
        C = wl.orbitals()
        tr = occk.Tree(wl.system, wl.params)
        trees.append(tr)
        Cs.append(torch.from_numpy(C).cuda())
        Ks.append(torch.zeros((wl.system.nbasis, C.shape[1]), dtype=torch.float64, device="cuda"))
        flops += tr.flops(C.shape[1], C.shape[1], symmetric=True)["total"]
    noccs = [C.shape[1] for C in Cs]
    plan = occk.Batch(trees, noccs, prec)
    choice = plan.tune(Cs, Ks)
    torch.cuda.synchronize()

    def timeit(fn, steps):
        for _ in range(args.warmup):
            fn()
        torch.cuda.synchronize()
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record()
        for _ in range(steps):
            fn()
        e1.record()
        torch.cuda.synchronize()
        return e0.elapsed_time(e1) / steps

    t_batch = timeit(lambda: plan.run(Cs, Ks), args.steps)
    K_batch = [K.clone() for K in Ks]
    plan.free()

    def separate(code):
        for tr, C, K in zip(trees, Cs, Ks):
            occk.far_K(tr, C, K, precision=code, jblock=0)
    t_sep = timeit(lambda: separate(prec), args.steps)
    dev = max(float((a - b).abs().max() / b.abs().max()) for a, b in zip(K_batch, Ks))
    t_f64 = timeit(lambda: separate(occk.PREC_FP64), args.steps)
    value = flops / (t_batch * 1e-3) / 1e9
    out = {
        "metric": "far-field K_ri GFLOP/s (16-system batch)",
        "value": round(value, 1), "unit": "GFLOP/s", "n_gpus": 1, "steps": args.steps, "warmup": args.warmup,
        "ms_per_step": round(t_batch, 3), "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": {"fp32": "f32", "bf16x3": "bf16x3", "bf16x6": "bf16x6"}[prec_name], "data": "synthetic",
        "config": {"workload": "16 water clusters (20..100 molecules, nbasis 480..2400), 3-D depth 3, ws 2, L=2, "
                               "all i and j of each",
                   "precision": prec_name, "autotuned": {"blocks_per_cu": choice[0], "gemm_tiles_per_task": choice[1],
                                                          "translation_tiles_per_task": choice[2]},
                   "flops_per_step": flops},
        "separate_launches_ms": round(t_sep, 3), "separate_fp64_ms": round(t_f64, 3),
        "speedup_vs_separate": round(t_sep / t_batch, 3), "speedup_vs_fp64": round(t_f64 / t_batch, 3),
        "batched_vs_separate_rel_diff": dev,
    }
    print(json.dumps(out), flush=True)


def bench_protein(args):
    """Learned ranks on the protein-shaped globule (644 sites, nbasis 6187,
    nocc 1261, 3-D depth 3, ws 2, L = 8), j sample [0, J) of all i: the plain
    fixed-rank FP64 path (the judge) against the learned-rank path, and the
    learned ranks with the split-BF16x6 contractions.

    The selector is trained on method-generated targets of two smaller
    training globules (seeds 1000, 1001) and its threshold calibrated on them
    (the loosest log10 tau whose error stays below 1e-6 / 3); training and
    calibration are timed separately and not part of either timed call."""
    import numpy as np
    import torch

    import workloads
    from paper_1708_05353_amd import occk

    jn = args.protein_j
    t0 = time.perf_counter()
    Xs, Ts, trains = [], [], []
    for seed in (1000, 1001):
        w = workloads.protein_blob(seed=seed, scale=0.2, nocc=None)
        tr = occk.Tree(w.system, w.params)
        C = torch.from_numpy(w.orbitals()).cuda()
        X, T = occk.Selector.collect(tr, C, (0, 16), max_samples=40000, seed=seed)
        Xs.append(X)
        Ts.append(T)
        trains.append((w, tr, C))
    sel = occk.Selector(seed=11)
    sel.train(np.vstack(Xs), np.vstack(Ts), epochs=25, batch=512, lr=2e-3, seed=2)

    def rel(a, b):
        return float((a - b).abs().max() / b.abs().max())

    def pair(tr, C, nb, jr):
        Kf = torch.zeros((nb, C.shape[1]), dtype=torch.float64, device="cuda")
        occk.far_K(tr, C, Kf, j_range=jr)
        Kl = torch.zeros_like(Kf)
        occk.far_K(tr, C, Kl, j_range=jr, selector=sel)
        torch.cuda.synchronize()
        return rel(Kl, Kf)

    chosen = -10.0
    for lt in (-3.0, -3.5, -4.0, -4.5, -5.0, -5.5, -6.0, -6.5, -7.0, -8.0):
        sel.set_rule(lt, 0.5)
        if max(pair(tr, C, w.system.nbasis, (0, 16)) for w, tr, C in trains) <= 1e-6 / 3:
            chosen = lt
            break
    sel.set_rule(chosen, 0.5)
    for _, tr, _ in trains:
        tr.free()
    t_train = time.perf_counter() - t0
    print(f"[bench] selector trained and calibrated in {t_train:.1f} s (log10 tau {chosen})", file=sys.stderr,
          flush=True)

    wl = workloads.protein_blob()
    tree = occk.Tree(wl.system, wl.params)
    n = wl.system.nocc
    Cd = torch.from_numpy(wl.orbitals()).cuda()
    Kf = torch.zeros((wl.system.nbasis, n), dtype=torch.float64, device="cuda")
    Kl = torch.zeros_like(Kf)
    fixed = lambda: occk.far_K(tree, Cd, Kf, j_range=(0, jn))
    learned = lambda: occk.far_K(tree, Cd, Kl, j_range=(0, jn), selector=sel)

    def timeit(fn):
        for _ in range(args.warmup):
            fn()
        torch.cuda.synchronize()
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record()
        for _ in range(args.steps):
            fn()
        e1.record()
        torch.cuda.synchronize()
        return e0.elapsed_time(e1) / args.steps

    fixed()
    torch.cuda.synchronize()
    t_fixed = timeit(fixed)
    tree.rank_stats()                       # reset the rank histogram
    t_learned = timeit(learned)
    hist = tree.rank_stats()
    work = float(sum(hist[p] * (p + 1) ** 4 for p in range(9)) / (hist.sum() * 9 ** 4))
    err = rel(Kl, Kf)
    # the learned ranks with the split-BF16x6 contractions (FP32
    # translations): the mixed and learned forms together, against the same
    # fixed-rank FP64 result
    Km = torch.zeros_like(Kf)
    both = lambda: occk.far_K(tree, Cd, Km, j_range=(0, jn), selector=sel, precision=occk.PREC_BF16X6)
    t_both = timeit(both)
    err_both = rel(Km, Kf)
    fl = tree.flops(n, jn)["total"]
    out = {
        "metric": "far-field K_ri GFLOP/s (protein L=8, fixed rank; learned-rank path beside it)",
        "value": round(fl / (t_fixed * 1e-3) / 1e9, 1), "unit": "GFLOP/s", "n_gpus": 1, "steps": args.steps,
        "warmup": args.warmup, "ms_per_step": round(t_fixed, 3), "higher_is_better": True, "scaling": "weak",
        "vs_baseline": None, "dtype": "f64", "data": "synthetic",
        "config": {"workload": f"protein-shaped globule (644 sites, nbasis 6187, nocc {n}), 3-D depth 3, ws 2, "
                               f"L=8; all i, j in [0,{jn})",
                   "flops_per_step": fl},
        "learned": {"ms_per_step": round(t_learned, 3), "speedup_vs_fixed": round(t_fixed / t_learned, 3),
                    "rel_err_vs_fixed_L8": err, "m2l_work_fraction": round(work, 4),
                    "rank_histogram": [int(x) for x in hist], "log10_tau": chosen,
                    "train_and_calibrate_s": round(t_train, 1)},
        "learned_bf16x6": {"ms_per_step": round(t_both, 3), "speedup_vs_fixed": round(t_fixed / t_both, 3),
                           "rel_err_vs_fixed_L8": err_both, "bound": 1e-6, "within_bound": err_both <= 1e-6},
    }
    print(json.dumps(out), flush=True)


def bench_graphene(args):
    """Graphene-shaped sheet C150H30 (nbasis 2250, nocc 480, quadtree depth 4,
    ws 2), rank sweep L = 2..8 in FP64, FP32, BF16x3 and BF16x6: time per
    call, GFLOP/s, the error of each mixed result against the FP64 result at
    the same L (precision), and the error of the FP64 result at L against
    FP64 at L = 8 (truncation)."""
    import torch

    import workloads
    from paper_1708_05353_amd import occk

    precs = [("fp64", occk.PREC_FP64), ("fp32", occk.PREC_FP32), ("bf16x3", occk.PREC_BF16X3),
             ("bf16x6", occk.PREC_BF16X6)]

    def timeit(fn):
        for _ in range(args.warmup):
            fn()
        torch.cuda.synchronize()
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record()
        for _ in range(args.steps):
            fn()
        e1.record()
        torch.cuda.synchronize()
        return e0.elapsed_time(e1) / args.steps

    def rel(a, b):
        return float((a - b).abs().max() / b.abs().max())

    rows, K8 = [], None
    for L in (8, 7, 6, 5, 4, 3, 2):
        wl = workloads.graphene_flake(lmax=L)
        tree = occk.Tree(wl.system, wl.params)
        n = wl.system.nocc
        Cd = torch.from_numpy(wl.orbitals()).cuda()
        fl = tree.flops(n, n, symmetric=True)["total"]
        row = {"lmax": L, "flops_per_call": fl}
        K64 = None
        for name, code in precs:
            K = torch.zeros((wl.system.nbasis, n), dtype=torch.float64, device="cuda")
            ms = timeit(lambda: occk.far_K(tree, Cd, K, precision=code))
            row[name] = {"ms": round(ms, 3), "GFLOP/s": round(fl / (ms * 1e-3) / 1e9, 1)}
            if name == "fp64":
                K64 = K.clone()
                if K8 is None:
                    K8 = K64
                row["fp64"]["rel_err_vs_L8"] = rel(K64, K8)
            else:
                row[name]["rel_err_vs_fp64"] = rel(K, K64)
                row[name]["speedup_vs_fp64"] = round(row["fp64"]["ms"] / ms, 3)
        tree.free()
        rows.append(row)
        print(f"[bench] L={L}: " + ", ".join(f"{k} {row[k]['ms']:.1f} ms" for k, _ in precs), file=sys.stderr,
              flush=True)
    top = rows[0]
    out = {"metric": "far-field K_ri GFLOP/s (graphene sheet, L=8 FP64; sweep L=2..8 x precision beside it)",
           "value": top["fp64"]["GFLOP/s"], "unit": "GFLOP/s", "n_gpus": 1, "steps": args.steps,
           "warmup": args.warmup, "ms_per_step": top["fp64"]["ms"], "higher_is_better": True, "scaling": "weak",
           "vs_baseline": None, "dtype": "f64", "data": "synthetic",
           "config": {"workload": "graphene-shaped sheet C150H30 (nbasis 2250, nocc 480), quadtree depth 4, ws 2; "
                                  "all i and j"},
           "sweep": sorted(rows, key=lambda r: r["lmax"])}
    print(json.dumps(out), flush=True)


def copy_probe(mb: int):
    """A plain device-to-device copy of a known size, for scaling hardware
    traffic counters (bytes the counters report per byte moved)."""
    import torch
    n = mb * (1 << 20) // 8
    src = torch.ones(n, dtype=torch.float64, device="cuda")
    dst = torch.empty_like(src)
    torch.cuda.synchronize()
    dst.copy_(src)
    torch.cuda.synchronize()
    print(json.dumps({"copy_probe_bytes_read": n * 8, "copy_probe_bytes_written": n * 8}), flush=True)


def copy_rate(mb: int = 2048, reps: int = 10) -> dict:
    """HBM bytes per second of a plain device-to-device copy (read + write),
    timed with HIP events: what the memory system delivers to a streaming
    kernel on this machine, beside the datasheet peak."""
    import torch
    n = mb * (1 << 20) // 8
    src = torch.ones(n, dtype=torch.float64, device="cuda")
    dst = torch.empty_like(src)
    dst.copy_(src)
    torch.cuda.synchronize()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record()
    for _ in range(reps):
        dst.copy_(src)
    e1.record()
    torch.cuda.synchronize()
    t = e0.elapsed_time(e1) * 1e-3 / reps
    del src, dst
    torch.cuda.empty_cache()
    return {"bytes": 2 * n * 8, "GB/s": round(2 * n * 8 / t / 1e9, 1), "frac_of_peak": round(2 * n * 8 / t / PEAK_HBM, 4)}


TRAFFIC_FILE = os.path.join(ROOT, "profiles", "alkane_L2_fp64_hbm_traffic.md")


# the sources of the far-field K call (its kernels, their launches, the tree
# and the ABI layer); the batch, selector, Coulomb and near-field sources
# build other entry points
FAR_K_SOURCES = ("abi.cpp", "device.hpp", "far_k.hip", "kernels.hpp", "occk_internal.hpp", "tree_build.cpp")


def kernel_source_digest() -> str:
    """sha256 over the sources of the far-field K call: counters taken with
    other sources do not describe the current kernels."""
    import hashlib
    h = hashlib.sha256()
    for name in FAR_K_SOURCES:
        h.update(name.encode())
        with open(os.path.join(ROOT, "paper_1708_05353_amd", "csrc", name), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()[:16]


def measured_traffic(cls: str):
    """HBM bytes per launch of a kernel class from the committed counter
    summary, or None when it is missing or was taken on other sources."""
    try:
        with open(TRAFFIC_FILE) as fh:
            for line in fh:
                if line.startswith("<!-- traffic "):
                    rec = json.loads(line[len("<!-- traffic "):].rsplit("-->", 1)[0])
                    if rec["digest"] != kernel_source_digest():
                        return None
                    return rec["per_launch_bytes"].get(cls)
    except (OSError, ValueError, KeyError):
        return None
    return None


def measured_call_traffic():
    """HBM bytes of one whole call from the committed counter summary, or None."""
    try:
        with open(TRAFFIC_FILE) as fh:
            for line in fh:
                if line.startswith("<!-- traffic "):
                    rec = json.loads(line[len("<!-- traffic "):].rsplit("-->", 1)[0])
                    if rec["digest"] != kernel_source_digest():
                        return None
                    return rec.get("call_bytes")
    except (OSError, ValueError, KeyError):
        return None
    return None


def _pmc_rows(d, counter):
    import csv
    import glob
    import re
    rows = {}
    for f in glob.glob(os.path.join(d, "**", "*counter_collection.csv"), recursive=True):
        with open(f) as fh:
            for r in csv.DictReader(fh):
                if r["Counter_Name"] != counter:
                    continue
                rows[int(r["Dispatch_Id"])] = (re.sub(r"\(.*", "", r["Kernel_Name"]), float(r["Counter_Value"]))
    return rows


def _classify_last_call(names, info):
    """Kernel (one of KERNELS, or "opgen") of every dispatch of the last
    occk_far_K call in a profile of 'bench.py --no-mixed' (dispatch id ->
    kernel name): each call starts with the operator generation and, in the
    symmetric schedule, the all-column half transform; the translations of a
    j batch are the upward level passes, then the downward ones, with the
    walks (when used) covering the levels below their roots."""
    n_up, n_down = info.depth - info.lmin, info.depth - info.lmin + 1
    ids = sorted(i for i in names if "occk::" in names[i])
    start = max(i for i in ids if "opgen" in names[i])      # the last call
    lr_up, lr_dn = walk_roots(info)
    walks = [i for i in ids if i >= start and "_walk" in names[i]]
    if walks:           # level passes only above the walks' root levels
        n_up, n_down = lr_up - info.lmin, lr_dn - info.lmin
        ntr_all = sum(1 for i in ids if i >= start and "translate" in names[i])
        if ntr_all != (len(walks) // 2) * (n_up + n_down):
            raise SystemExit("translation launches do not match the walk root levels")
    kind, ntr, seen_half = {}, 0, False
    for i in ids:
        if i < start:
            continue
        k = names[i]
        if "tree_lds_kernel" in k:
            kind[i] = "tree"
            continue
        if "up_walk" in k or "down_walk" in k:
            kind[i] = "up_walk" if "up_walk" in k else "down_walk"
            continue
        if "translate" in k:
            ntr += 1
            kind[i] = "up_pass" if (ntr - 1) % (n_up + n_down) < n_up else "down_pass"
            continue
        if "half_kernel" in k:
            kind[i] = "half" if seen_half else "ht"
            seen_half = True
            continue
        for key, c in (("opgen", "opgen"), ("to_float", "convert"), ("reduce", "reduce"), ("omega_kernel", "omega"), ("omega_ht_kernel", "omega"),
                       ("l2pt_kernel", "l2p_mirror"), ("l2pt_wide_kernel", "l2p_mirror"),
                       ("l2p_kernel", "l2p_direct"), ("l2p_wide_kernel", "l2p_direct"),
                       ("l2p_ht_kernel", "l2p_direct"), ("l2p_ht_wide_kernel", "l2p_direct")):
            if key in k:
                kind[i] = c
                break
        else:
            raise SystemExit(f"unexpected kernel in the sequence: {k}")
    return kind


def trace_summary(trace_dir):
    """Per-kernel launch times of the last occk_far_K call recorded by
    'rocprofv3 --kernel-trace' of 'bench.py --no-mixed' (the same kernels
    and launch averages as the bench line's "kernels"); prints markdown."""
    import csv
    import glob
    import re
    import workloads
    from paper_1708_05353_amd import occk
    names, dur = {}, {}
    for f in glob.glob(os.path.join(trace_dir, "**", "*kernel_trace.csv"), recursive=True):
        with open(f) as fh:
            for r in csv.DictReader(fh):
                i = int(r["Dispatch_Id"])
                names[i] = re.sub(r"\(.*", "", r["Kernel_Name"])
                dur[i] = (int(r["End_Timestamp"]) - int(r["Start_Timestamp"])) * 1e-9
    wl = workloads.alkane_chain()
    tr = occk.Tree(wl.system, wl.params)
    kind = _classify_last_call(names, tr.info)
    tot = {}
    for i, c in kind.items():
        n, t = tot.get(c, (0, 0.0))
        tot[c] = (n + 1, t + dur[i])
    print("Per kernel, last call of the run (the bench line's \"kernels\"; `python3 bench.py --trace-summary "
          f"{trace_dir}`):\n")
    print("| kernel | launches | ms | average launch, us |\n|---|---|---|---|")
    for c in KERNELS:
        if c in tot:
            n, t = tot[c]
            print(f"| {c} | {n} | {t * 1e3:.2f} | {t / n * 1e6:.1f} |")


def pmc_summary(fetch_dir, write_dir, copy_fetch_dir, copy_write_dir, copy_mib, cmds):
    """Per-class HBM traffic of the last occk_far_K call recorded by two
    rocprofv3 --pmc runs of 'bench.py --steps 1 --warmup 0' (FETCH_SIZE,
    WRITE_SIZE; KiB per dispatch), scaled by what the same counters read for
    a plain copy of copy_mib MiB; prints a markdown summary."""
    import workloads
    from paper_1708_05353_amd import occk
    cf = _pmc_rows(copy_fetch_dir, "FETCH_SIZE")
    cw = _pmc_rows(copy_write_dir, "WRITE_SIZE")
    nbytes = copy_mib * (1 << 20)
    fk = [v for k, v in cf.values() if "copyBuffer" in k]
    wk = [v for k, v in cw.values() if "copyBuffer" in k]
    fetch_scale = nbytes / (fk[0] * 1024)
    write_scale = nbytes / (wk[0] * 1024)
    F = _pmc_rows(fetch_dir, "FETCH_SIZE")
    W = _pmc_rows(write_dir, "WRITE_SIZE")
    wl = workloads.alkane_chain()
    tr = occk.Tree(wl.system, wl.params)
    info = tr.info
    kind = _classify_last_call({i: F[i][0] for i in F}, info)
    tot = {}
    for i, c in kind.items():
        n, fb, wb = tot.get(c, (0, 0.0, 0.0))
        tot[c] = (n + 1, fb + F[i][1] * 1024 * fetch_scale, wb + W.get(i, ("", 0.0))[1] * 1024 * write_scale)
    jb = 256
    costs = kernel_costs(info, wl.system.nocc, jb, "fp64", tree="tree" in tot)
    b_alg = 8 * (info.ncomp * info.npairs + 2 * info.nbasis * wl.system.nocc)
    print("# HBM traffic per kernel: alkane chain, L = 2, FP64 (one occk_far_K call)\n")
    print("Commands (repository root, one MI355X, `export TMPDIR=/tmp`):\n\n```")
    for c in cmds:
        print(c)
    print("```\n")
    print(f"Scale factors from the {copy_mib} MiB copy: FETCH_SIZE x{fetch_scale:.3f}, WRITE_SIZE x{write_scale:.3f} "
          "(bytes moved per byte the counter reports).  Schedule bytes: the compulsory traffic of the schedule "
          "as executed (`kernel_costs` in bench.py: every box a kernel touches read or written once per j batch, "
          "GEMM operands once).\n")
    print("| kernel | launches | HBM read GB | HBM write GB | HBM total GB | schedule GB | ratio | bytes per launch |")
    print("|---|---|---|---|---|---|---|---|")
    per_launch, call = {}, 0.0
    for c in KERNELS + ["opgen"]:
        if c not in tot:
            continue
        n, fb, wb = tot[c]
        call += fb + wb
        if c == "opgen":
            continue
        alg = costs[c][1]
        per_launch[c] = (fb + wb) / n
        print(f"| {c} | {n} | {fb / 1e9:.2f} | {wb / 1e9:.2f} | {(fb + wb) / 1e9:.2f} | {alg / 1e9:.2f} | "
              f"{(fb + wb) / alg:.2f} | {per_launch[c]:.4g} |")
    print()
    print(f"Whole call: {call / 1e9:.1f} GB of HBM traffic against the method's compulsory "
          f"B_alg = 8 (Q sum_B pi_B + 2 nbasis nocc) = {b_alg / 1e9:.3f} GB (ratio {call / b_alg:.0f}).\n")
    print("<!-- traffic " + json.dumps({"digest": kernel_source_digest(), "fetch_scale": round(fetch_scale, 4),
                                        "write_scale": round(write_scale, 4), "call_bytes": round(call),
                                        "per_launch_bytes": {k: round(v) for k, v in per_launch.items()}}) + " -->")


SQ_COUNTERS = ["SQ_WAVE_CYCLES", "SQ_BUSY_CU_CYCLES", "SQ_VALU_MFMA_BUSY_CYCLES", "SQ_WAIT_ANY", "SQ_WAIT_INST_ANY",
               "SQ_WAIT_INST_LDS", "SQ_LDS_BANK_CONFLICT", "SQ_LDS_IDX_ACTIVE", "SQ_INSTS_VALU_MFMA_MOPS_F64",
               "SQ_INSTS_VALU_MFMA_MOPS_BF16", "SQ_INSTS_LDS", "SQ_INSTS_VMEM_RD", "SQ_INSTS_VALU", "SQ_INSTS_SALU"]


def sq_summary(dirs, cmds, precision="fp64"):
    """Per-kernel MFMA, wait-state and LDS counters of the last occk_far_K
    call recorded by rocprofv3 --pmc runs of 'bench.py --steps 1 --warmup 0
    --one-stream' (summed over the call's dispatches of each kernel class);
    prints markdown."""
    import workloads
    from paper_1708_05353_amd import occk
    per = {}
    names = {}
    for d in dirs:
        for c in SQ_COUNTERS:
            rows = _pmc_rows(d, c)
            for i, (k, v) in rows.items():
                names[i] = k
                per.setdefault(c, {})[i] = v
    wl = workloads.alkane_chain()
    tr = occk.Tree(wl.system, wl.params)
    kind = _classify_last_call(names, tr.info)
    tot = {}
    for i, cls in kind.items():
        t = tot.setdefault(cls, {c: 0.0 for c in SQ_COUNTERS})
        for c in SQ_COUNTERS:
            t[c] += per.get(c, {}).get(i, 0.0)
    print(f"# MFMA, wait-state and LDS counters per kernel: alkane chain, L = 2, {precision.upper()} (one occk_far_K call, "
          "one stream)\n")
    print("Commands (repository root, one MI355X, `export TMPDIR=/tmp`; two passes of at most 8 SQ counters):\n\n```")
    for c in cmds:
        print(c)
    print("```\n")
    print("Sums over the last call's dispatches of each kernel.  MFMA busy = SQ_VALU_MFMA_BUSY_CYCLES / "
          "(4 SQ_BUSY_CU_CYCLES) (the MFMA counter summed over the 4 SIMDs of a CU); waits are fractions of "
          "SQ_WAVE_CYCLES; LDS conflict = SQ_LDS_BANK_CONFLICT / SQ_LDS_IDX_ACTIVE.\n")
    print("| kernel | MFMA busy | wait on dependencies (WAIT_INST_ANY) | wait any | LDS wait | LDS conflict | "
          "VALU instr | SALU instr | VMEM reads | LDS instr | F64 MFMA ops | BF16 MFMA ops |")
    print("|---|---|---|---|---|---|---|---|---|---|---|---|")
    for cls in KERNELS:
        if cls not in tot:
            continue
        t = tot[cls]
        wc = max(t["SQ_WAVE_CYCLES"], 1.0)
        busy = t["SQ_VALU_MFMA_BUSY_CYCLES"] / max(4 * t["SQ_BUSY_CU_CYCLES"], 1.0)
        conf = t["SQ_LDS_BANK_CONFLICT"] / max(t["SQ_LDS_IDX_ACTIVE"], 1.0)
        print(f"| {cls} | {busy:.2f} | {t['SQ_WAIT_INST_ANY'] / wc:.2f} | {t['SQ_WAIT_ANY'] / wc:.2f} | "
              f"{t['SQ_WAIT_INST_LDS'] / wc:.3f} | {conf:.3f} | {t['SQ_INSTS_VALU']:.3g} | {t['SQ_INSTS_SALU']:.3g} | "
              f"{t['SQ_INSTS_VMEM_RD']:.3g} | {t['SQ_INSTS_LDS']:.3g} | {t['SQ_INSTS_VALU_MFMA_MOPS_F64']:.3g} | "
              f"{t['SQ_INSTS_VALU_MFMA_MOPS_BF16']:.3g} |")


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--workload", default="alkane", choices=["alkane", "batch16", "protein-learned", "graphene-sweep"])
    ap.add_argument("--protein-j", type=int, default=32, help="j sample of the protein-learned workload")
    ap.add_argument("--copy-probe", type=int, default=0, help="MiB; run only a plain copy of that size")
    ap.add_argument("--pmc-summary", nargs=4, metavar=("FETCH_DIR", "WRITE_DIR", "COPY_FETCH_DIR", "COPY_WRITE_DIR"),
                    help="summarise rocprofv3 --pmc FETCH_SIZE / WRITE_SIZE runs (CPU only)")
    ap.add_argument("--pmc-copy-mib", type=int, default=1024)
    ap.add_argument("--sq-summary", nargs="+", metavar="PMC_DIR",
                    help="summarise rocprofv3 --pmc SQ counter runs (CPU only)")
    ap.add_argument("--trace-summary", metavar="TRACE_DIR",
                    help="print per-class launch times of a rocprofv3 --kernel-trace run of this bench (--no-mixed)")
    ap.add_argument("--pmc-commands", nargs="*", default=[])
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--lmax", type=int, default=2)
    ap.add_argument("--precision", default="fp64", choices=["fp64", "fp32", "bf16x3", "bf16x6"])
    ap.add_argument("--jblock", type=int, default=0)
    ap.add_argument("--one-stream", action="store_true",
                    help="time the one-stream schedule (every kernel alone; for kernel traces and counters)")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-mixed", action="store_true", help="skip the FP32 mixed-path comparison")
    ap.add_argument("--no-coulomb", action="store_true", help="skip the far-field Coulomb J leg")
    ap.add_argument("--no-near", action="store_true", help="skip the near-field exchange leg")
    ap.add_argument("--cpu-sample-j", type=int, default=64)
    ap.add_argument("--cpu-repeats", type=int, default=3)
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py: this build runs on one GPU only (got --gpus {args.gpus}); the multi-GPU "
              "split over the output index i is described in DESIGN.md but not built.", file=sys.stderr)
        sys.exit(2)

    if args.copy_probe:
        copy_probe(args.copy_probe)
        return
    if args.pmc_summary:
        pmc_summary(*args.pmc_summary, args.pmc_copy_mib, args.pmc_commands)
        return
    if args.trace_summary:
        trace_summary(args.trace_summary)
        return
    if args.sq_summary:
        sq_summary(args.sq_summary, args.pmc_commands, args.precision)
        return
    if args.workload == "batch16":
        bench_batch(args)
        return
    if args.workload == "protein-learned":
        bench_protein(args)
        return
    if args.workload == "graphene-sweep":
        bench_graphene(args)
        return

    import torch

    import workloads
    from paper_1708_05353_amd import occk

    prec = {"fp64": occk.PREC_FP64, "fp32": occk.PREC_FP32, "bf16x3": occk.PREC_BF16X3,
            "bf16x6": occk.PREC_BF16X6}[args.precision]
    wl = workloads.alkane_chain(lmax=args.lmax)
    t0 = time.perf_counter()
    C = wl.orbitals()
    t_orb = time.perf_counter() - t0
    t0 = time.perf_counter()
    tree = occk.Tree(wl.system, wl.params)
    t_tree = time.perf_counter() - t0
    nocc = wl.system.nocc
    dev = torch.device("cuda:0")
    Cd = torch.from_numpy(C).to(dev)
    K = torch.zeros((wl.system.nbasis, nocc), dtype=torch.float64, device=dev)
    stream = torch.cuda.current_stream(dev)
    call = lambda one: occk.far_K(tree, Cd, K, precision=prec, jblock=args.jblock, stream=stream, one_stream=one)
    t0 = time.perf_counter()
    call(args.one_stream)       # uploads the tree and allocates the workspace
    torch.cuda.synchronize()
    t_first = time.perf_counter() - t0
    print(f"[bench] orbitals {t_orb:.1f}s tree {t_tree:.1f}s first call {t_first:.1f}s", file=sys.stderr, flush=True)
    for _ in range(args.warmup):
        call(args.one_stream)
    torch.cuda.synchronize()
    jb_call = tree.workspace_jblock()   # j batch width of the timed schedule
    ev0, ev1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    ev0.record(stream)
    for _ in range(args.steps):
        call(args.one_stream)
    ev1.record(stream)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    ms = ev0.elapsed_time(ev1) / args.steps
    # Kernel timings: the same calls in the one-stream schedule, where every
    # kernel runs alone (in the default schedule the L2P of a batch overlaps
    # the next batch's translations, and a kernel's events then span both).
    # The one-stream schedule picks its own j batch width (256 where the
    # FP64 two-stream schedule takes 128): one untimed call sets up its
    # workspace, and the kernel cost model takes that width.
    call(True)
    torch.cuda.synchronize()
    jb = tree.workspace_jblock()
    tree.profile(True)
    tree.profile_read()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record(stream)
    for _ in range(args.steps):
        call(True)
    e1.record(stream)
    torch.cuda.synchronize()
    prof = tree.profile_read()
    tree.profile(False)
    ms_one = e0.elapsed_time(e1) / args.steps
    fl = tree.flops(nocc, nocc, symmetric=True)
    value = fl["total"] / (ms * 1e-3) / 1e9
    print(f"[bench] {ms:.2f} ms/step, {value:.0f} GFLOP/s ({ms_one:.2f} ms/step in one stream)", file=sys.stderr,
          flush=True)

    lds_tree = prof["tree"][1] > 0
    costs = class_costs(tree.info, nocc, jb, args.precision, tree=lds_tree)
    breakdown = {}
    for cls, (flops, nbytes) in costs.items():
        t_ms, nl = prof[cls]
        if t_ms <= 0:
            continue
        per_call_ms = t_ms / args.steps
        breakdown[cls] = {"ms_per_step": round(per_call_ms, 3), "launches_per_step": nl // args.steps,
                          "TFLOP/s": round(flops / (per_call_ms * 1e-3) / 1e12, 2),
                          "GB/s": round(nbytes / (per_call_ms * 1e-3) / 1e9, 1)}
    # single kernels: time from the nested HIP-event scopes, algorithmic flops
    # and bytes per kernel, fraction of the MFMA (or vector) and HBM peaks
    kcost = kernel_costs(tree.info, nocc, jb, args.precision, tree=lds_tree)
    ktime = kernel_times(prof)
    pk = PEAK_FLOPS[args.precision]
    Q = tree.info.ncomp
    live = translation_live_entries(Q, wl.params.split_mask)
    kernels = {}
    for k in KERNELS:
        t_ms, nl = ktime[k]
        if t_ms <= 0 or nl <= 0:
            continue
        flops, nbytes = kcost[k]
        t = t_ms / args.steps * 1e-3
        kernels[k] = {"ms_per_step": round(t * 1e3, 3), "launches_per_step": nl // args.steps,
                      "alg_flops": flops, "alg_bytes": nbytes,
                      "TFLOP/s": round(flops / t / 1e12, 2), "frac_flops_peak": round(flops / t / pk, 4),
                      "GB/s": round(nbytes / t / 1e9, 1), "frac_hbm_peak": round(nbytes / t / PEAK_HBM, 4)}
        if k in TRANSLATION_KERNELS and live < Q * Q:
            # the vector translations skip the operators' structural zeros:
            # the products they execute (the M2M/L2L part of alg_flops counts
            # the operator's nonzeros, the M2L part the dense Q^2)
            kernels[k]["exec_flops_fraction"] = round(live / (Q * Q), 4)
    # the roofline object: the kernel with the largest time per call.  A
    # contraction (GEMM, or an MFMA translation) is priced by the method's
    # dense arithmetic against the MFMA peak of its dtype.  A vector
    # translation that skips structural zeros does a fraction of those
    # products and is bound by the memory traffic of its schedule (every box
    # it touches read or written once per j batch): it is priced by those
    # bytes against the HBM peak.  The other measure is reported beside it.
    dom = max(kernels, key=lambda k: kernels[k]["ms_per_step"])
    kd = kernels[dom]
    flops, nbytes = kd["alg_flops"], kd["alg_bytes"]
    t_dom = kd["ms_per_step"] * 1e-3
    nl_dom = kd["launches_per_step"]
    vector = dom in TRANSLATION_KERNELS and Q <= 9
    if vector and live < Q * Q:
        ach = nbytes / t_dom
        roof = {"bound": "hbm", "achieved": round(ach / 1e9, 1), "peak": PEAK_HBM / 1e9, "unit": "GB/s",
                "frac": round(ach / PEAK_HBM, 4), "traffic": None, "kernel": dom,
                "dense_flops": {"TFLOP/s": round(flops / t_dom / 1e12, 2), "peak": round(pk / 1e12, 1),
                                "exec_fraction": round(live / (Q * Q), 4)}}
    else:
        ach = flops / t_dom / 1e12
        roof = {"bound": "alu" if vector else "mfma", "achieved": round(ach, 2), "peak": round(pk / 1e12, 1),
                "unit": "TFLOP/s", "frac": round(ach * 1e12 / pk, 4), "traffic": None, "kernel": dom,
                "schedule_hbm": {"bytes_per_launch": round(nbytes / max(1, nl_dom)),
                                 "GB/s": round(nbytes / t_dom / 1e9, 1), "frac": round(nbytes / t_dom / PEAK_HBM, 4)}}
    roof["alg_bytes_per_launch"] = round(nbytes / max(1, nl_dom))
    roof["alg_flops_per_launch"] = round(flops / max(1, nl_dom))
    roof["avg_launch_us"] = round(t_dom / max(1, nl_dom) * 1e6, 1)
    if args.precision == "fp64" and args.lmax == 2 and args.jblock in (0, 256):
        roof["traffic"] = measured_traffic(dom)   # HBM bytes per launch from the counter summary, if current
    # the whole call's HBM bytes against the method's compulsory bytes
    inf = tree.info
    b_alg = 8 * (inf.ncomp * inf.npairs + 2 * inf.nbasis * nocc)
    meas = measured_call_traffic() if (args.precision == "fp64" and args.lmax == 2 and args.jblock in (0, 256)) \
        else None
    hbm_call = {"alg_bytes": b_alg, "measured_bytes": meas,
                "measured_over_alg": round(meas / b_alg, 1) if meas else None,
                "note": "alg_bytes = 8 (Q sum_B pi_B + 2 nbasis nocc): AO multipoles once, C read, K written"}
    out = {
        "metric": "far-field K_ri GFLOP/s",
        "value": round(value, 1),
        "unit": "GFLOP/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(ms, 3),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": {"fp64": "f64", "fp32": "f32", "bf16x3": "bf16x3", "bf16x6": "bf16x6"}[args.precision],
        "data": "synthetic",
        "config": {"workload": f"alkane chain (C400H802 stand-in): nbasis 9610, nocc 1601, L={args.lmax}, "
                               f"1-D tree depth 8, ws 2; all i and j",
                   "precision": args.precision, "jblock": jb_call, "jblock_one_stream": jb, "flops_per_step": fl["total"],
                   "flops_per_step_all_columns": tree.flops(nocc, nocc)["total"],
                   "pct_peak": round(100 * value * 1e9 / PEAK_FLOPS[args.precision], 2),
                   "tree_build_s": round(t_tree, 2), "wall_s_timed": round(wall, 3),
                   "schedule": "one stream" if args.one_stream else "two streams (L2P of a j batch overlapping the "
                                                                     "next batch's translations)",
                   "ms_per_step_one_stream": round(ms_one, 3)},
        "roofline": roof,
        "kernels": kernels,
        "breakdown": breakdown,
        "hbm_call": hbm_call,
    }
    out["hbm_copy"] = copy_rate()   # the streaming rate the box delivers (read + write), for the HBM rooflines
    if args.precision == "fp64" and not args.no_mixed:
        # the mixed path on the same inputs: FP32 contractions and translations
        # (FP32, or split-BF16 products on the MFMA with FP32 accumulation),
        # FP64 operators and K accumulation; error against this FP64 result
        K64 = K.clone()
        Km = torch.zeros_like(K)
        modes = [("fp32", occk.PREC_FP32, 1e-6), ("bf16x6", occk.PREC_BF16X6, 1e-6),
                 ("bf16x3", occk.PREC_BF16X3, 5e-5)]
        mixed = {}
        for mname, mcode, bound in modes:
            mcall = lambda: occk.far_K(tree, Cd, Km, precision=mcode, jblock=args.jblock, stream=stream,
                                       one_stream=args.one_stream)
            mcall()
            for _ in range(args.warmup):
                mcall()
            torch.cuda.synchronize()
            e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            e0.record(stream)
            for _ in range(args.steps):
                mcall()
            e1.record(stream)
            torch.cuda.synchronize()
            ms_m = e0.elapsed_time(e1) / args.steps
            err = float((Km - K64).abs().max() / K64.abs().max())
            mixed[mname] = {"ms_per_step": round(ms_m, 3), "value": round(fl["total"] / (ms_m * 1e-3) / 1e9, 1),
                            "speedup_vs_fp64": round(ms / ms_m, 3), "rel_err_vs_fp64": err, "bound": bound}
            print(f"[bench] mixed {mname} {ms_m:.2f} ms/step, x{ms / ms_m:.2f}, rel err {err:.2e}",
                  file=sys.stderr, flush=True)
        best = best_mixed_mode(mixed)
        out["mixed"] = dict(precision=best, **mixed[best], modes=mixed)
    if args.precision == "fp64" and not args.no_near:
        out["near_K"] = bench_near(wl, Cd, args, stream)
        print(f"[bench] near-field K {out['near_K']['ms_per_step']:.2f} ms/step", file=sys.stderr, flush=True)
    if args.precision == "fp64" and not args.no_coulomb:
        out["far_J"] = bench_coulomb(wl, Cd, args, stream)
        print(f"[bench] far-field J (L^J=10) {out['far_J']['ms_per_step']:.2f} ms/step", file=sys.stderr, flush=True)
    if not args.no_cpu_baseline:
        print("[bench] cpu baseline (oracle) ...", file=sys.stderr, flush=True)
        out["cpu_baseline"] = cpu_baseline(wl, C, fl["total"], nocc, args.cpu_sample_j, args.cpu_repeats)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
