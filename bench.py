"""Far-field occupied exchange throughput on one MI355X.

One step = one occk_far_K call: the whole hot path (operator generation,
half and full MO transforms, upward/interaction-list/downward translations,
L2P and the K reduction) on the alkane-chain workload (C400H802 stand-in:
nbasis 9610, nocc 1601, 1-D tree of depth 8, ws 2, L = 2), inputs resident in
HBM.  Prints one JSON line.
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

PEAK = {"fp64": 78.6e12, "fp32": 157.3e12, "bf16x3": 2.5e15 / 3.0}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--lmax", type=int, default=2)
    ap.add_argument("--precision", default="fp64", choices=["fp64", "fp32", "bf16x3"])
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--cpu-sample-j", type=int, default=2)
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py: this build runs on one GPU only (got --gpus {args.gpus}); "
              "the path would shard over the output index i (see DESIGN.md).", file=sys.stderr)
        sys.exit(2)

    import numpy as np
    import torch

    import workloads
    from paper_1708_05353_amd import occk

    prec = {"fp64": occk.PREC_FP64, "fp32": occk.PREC_FP32, "bf16x3": occk.PREC_BF16X3}[args.precision]
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
    t0 = time.perf_counter()
    occk.far_K(tree, Cd, K, precision=prec, stream=stream)     # uploads tree, allocates workspace
    torch.cuda.synchronize()
    t_first = time.perf_counter() - t0
    print(f"[bench] orbitals {t_orb:.1f}s tree {t_tree:.1f}s first call {t_first:.1f}s", file=sys.stderr,
          flush=True)
    for _ in range(args.warmup):
        occk.far_K(tree, Cd, K, precision=prec, stream=stream)
    torch.cuda.synchronize()
    ev0, ev1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    ev0.record(stream)
    for k in range(args.steps):
        occk.far_K(tree, Cd, K, precision=prec, stream=stream)
    ev1.record(stream)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    ms = ev0.elapsed_time(ev1) / args.steps
    fl = tree.flops(nocc, nocc)
    value = fl["total"] / (ms * 1e-3) / 1e9
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
        "dtype": {"fp64": "f64", "fp32": "f32", "bf16x3": "bf16x3"}[args.precision],
        "data": "synthetic",
        "config": {"workload": f"alkane chain C400H802 stand-in, nbasis 9610, nocc 1601, L={args.lmax}, "
                               f"1-D depth 8, ws 2",
                   "precision": args.precision, "flops_per_step": fl["total"],
                   "pct_peak": round(100 * value * 1e9 / PEAK[args.precision], 2),
                   "wall_s_timed": round(wall, 3)},
    }
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
