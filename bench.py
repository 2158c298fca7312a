#!/usr/bin/env python3
"""Benchmark of FRW capacitance extraction with MicroWalk transitions on one
MI355X.

Workload (one step): frw_extract on the crossing-wire structure (2x2x1 um
grounded window, four 100x100 nm wires on two layers, 20 nm eps 7.0 coatings,
background eps 3.9 / 2.7), master net 0, 16^3-cell transition cubes, 1e6 walks,
a fresh seed per step.  Prints one JSON line (see the keys below).

    python bench.py [--steps K] [--warmup W] [--gpus 1]
"""
import argparse
import hashlib
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "micro-steps/s + walks/s at 1% 3σ cap error; p50/p99 latency vs plain"
# Integer VALU issue peak of MI355X: 256 CUs x 4 SIMD16 x 16 lanes x 2.4 GHz.
PEAK_LANE_OPS = 256 * 64 * 2.4e9
# Algorithmic lane-op slots of one MicroWalk step (Alg. 3 loop body): a quarter
# of a Philox4x32-10 block (10 rounds x (2 quarter-rate 32x32->64 products =
# 8 slots + 2 three-input xors) / 4 = 25), five threshold compares, one index
# update and one boundary test.
MW_STEP_SLOTS = 32
WALKER_SRC = os.path.join(ROOT, "paper_2507_09730_amd", "csrc", "frw.hip")
TRAFFIC_FILE = os.path.join(ROOT, "profiles", "frw_walk_kernel_c2_traffic.txt")


def _sha(path):
    return hashlib.sha256(open(path, "rb").read()).hexdigest()


def _traffic():
    """HBM bytes per walker launch from the committed rocprofv3 --pmc summary,
    or None when the walker source changed since the counters were taken."""
    if not os.path.exists(TRAFFIC_FILE):
        return None
    vals = {}
    for line in open(TRAFFIC_FILE):
        if ":" in line and not line.startswith("#"):
            k, v = line.split(":", 1)
            vals[k.strip()] = v.strip()
    if vals.get("frw_hip_sha256") != _sha(WALKER_SRC):
        return None
    try:
        return float(vals["hbm_bytes_per_launch"])
    except (KeyError, ValueError):
        return None


def cpu_baseline(st, walks, seed):
    import oracle
    cores = len(os.sched_getaffinity(0)) if hasattr(os, "sched_getaffinity") else os.cpu_count()
    cores = max(1, min(cores, 64))
    oracle.build()
    t0 = time.perf_counter()
    r = oracle.frw_extract(st, 0, walks, seed=seed, threads=cores)
    dt = time.perf_counter() - t0
    return {"value": walks / dt, "unit": "walks/s", "cores": cores, "kind": "oracle",
            "sample": "%d walks of the same workload (binary64 C++ oracle, %d threads over walk "
                      "ranges), %.1f s; micro-steps/s %.4g" % (walks, cores, dt,
                                                                r["stats"]["micro_steps"] / dt)}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--walks", type=int, default=1000000)
    ap.add_argument("--n-cells", type=int, default=16)
    ap.add_argument("--cpu-walks", type=int, default=60000)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    args = ap.parse_args()
    if args.gpus != 1:
        print("bench.py runs on one GPU only: this build measures the single-GPU kernels "
              "(walk ranges would shard across GPUs with one fp64 all-reduce of the per-net "
              "sums; not built).", file=sys.stderr)
        sys.exit(2)

    import numpy as np
    import torch

    import paper_2507_09730_amd as mw
    import workloads as W

    mw.mw_init(0)
    st = W.c2_structure()
    h = mw.StructureHandle(st)
    for i in range(args.warmup):
        mw.frw_extract(h, 0, args.walks, seed=10000 + i, n_cells=args.n_cells)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    walks = steps = launches = 0
    walker_s = 0.0
    rel = []
    for k in range(args.steps):
        r = mw.frw_extract(h, 0, args.walks, seed=k, n_cells=args.n_cells)
        s = r["stats"]
        walks += s["walks"]
        steps += s["micro_steps"]
        launches += s["launches"]
        walker_s += s["walker_seconds"]
        rel.append(3 * r["se"][0] / r["row"][0])
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    value = walks / dt
    # roofline of the walker kernel (dominant kernel): algorithmic MicroWalk
    # slots per launch / measured launch duration
    achieved = steps * MW_STEP_SLOTS / walker_s / 1e12  # T lane-op slots/s
    peak = PEAK_LANE_OPS / 1e12
    traffic = _traffic()
    out = {
        "metric": METRIC, "value": value, "unit": "walks/s", "n_gpus": 1, "steps": args.steps,
        "warmup": args.warmup, "ms_per_step": dt / args.steps * 1e3, "higher_is_better": True,
        "scaling": "weak", "vs_baseline": None, "dtype": "u32", "data": "synthetic",
        "config": {"workload": "crossing wires 2x2x1 um, 4 nets, 20 nm eps-7 coatings, "
                               "eps 3.9/2.7 layers, master 0, %d^3-cell cubes, %d walks/step"
                               % (args.n_cells, args.walks),
                   "walks_per_step": args.walks, "n_cells": args.n_cells, "hybrid": 1},
        "micro_steps_per_s": steps / dt,
        "rel_3sigma_Cmm": float(np.mean(rel)),
        "walker_kernel_ms_per_step": walker_s / args.steps * 1e3,
        "walker_launches_per_step": launches / args.steps,
        "roofline": {"bound": "alu", "achieved": achieved, "peak": peak, "unit": "TOP/s",
                     "frac": achieved / peak, "traffic": traffic},
    }
    if not args.no_cpu_baseline:
        out["cpu_baseline"] = cpu_baseline(st, args.cpu_walks, seed=7)
    print(json.dumps(out))


if __name__ == "__main__":
    main()
