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

import numpy as np

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
                                                                r["stats"]["micro_steps"] / dt)}, r


def batched_vs_plain(mw, W, reps=5):
    """4096-cube batched MicroWalk workload: autotuned graph replay of one
    persistent launch vs one launch per cube, same walks and seed."""
    import torch
    cubes = W.c3_cubes()
    eps = [c for c, _ in cubes]
    walks = [w for _, w in cubes]
    packed = mw.pack_cubes(eps)
    best = mw.mw_autotune_batch(None, walks, packed=packed)
    plan = mw.BatchPlan(None, walks, packed=packed, tune=best)
    plan.run(1)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for k in range(reps):
        h, st = plan.run(100 + k)
    torch.cuda.synchronize()
    t_batch = (time.perf_counter() - t0) / reps
    steps = int(st.sum(dtype=torch.int64))
    total = int(sum(walks))
    eps_cat, ns, eoff = packed
    off = np.concatenate([[0], np.cumsum(walks)[:-1]]).astype(np.int64)
    hp = torch.empty(total, dtype=torch.int32, device="cuda")
    sp = torch.empty(total, dtype=torch.int32, device="cuda")
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for c in range(len(walks)):
        n = int(ns[c])
        e = eps_cat[int(eoff[c]):int(eoff[c]) + n ** 3].view(n, n, n)
        mw.mw_transition(e, walks[c], seed=100 + reps - 1, cube_index=c,
                         hits=hp[off[c]:off[c] + walks[c]], steps=sp[off[c]:off[c] + walks[c]])
    torch.cuda.synchronize()
    t_plain = time.perf_counter() - t0
    same = bool(torch.equal(hp, h) and torch.equal(sp, st))
    plan.close()
    return {"workload": "4096 cubes, n 8-32, 1-6 inclusions, %d walks, %d micro-steps" % (total, steps),
            "tune": best, "batched_ms": t_batch * 1e3, "plain_ms": t_plain * 1e3,
            "batched_micro_steps_per_s": steps / t_batch, "plain_micro_steps_per_s": steps / t_plain,
            "batched_walks_per_s": total / t_batch, "speedup": t_plain / t_batch,
            "bit_identical": same,
            "batched_alu_frac": steps * MW_STEP_SLOTS / t_batch / PEAK_LANE_OPS}


def microwalk_e(mw, W, st, walks, n_cells, steps=5, master=0):
    """A workload with MicroWalk-E transitions (expanded cubes of 4x the
    conductor-free size at n = 16, expansion option 5) beside the plain
    MicroWalk figure: time per extraction, hops and micro-steps per walk, and
    the master's self term shift against plain MicroWalk in combined SEs."""
    h = mw.StructureHandle(st)
    out = {}
    rows = {}
    for ex in (0, 5):
        mw.frw_extract(h, master, walks, seed=900, n_cells=n_cells, expand=ex)
        t0 = time.perf_counter()
        acc = []
        for k in range(steps):
            acc.append(mw.frw_extract(h, master, walks, seed=500 + k, n_cells=n_cells, expand=ex))
        dt = (time.perf_counter() - t0) / steps
        s = acc[-1]["stats"]
        rows[ex] = (np.mean([a["row"][master] for a in acc]),
                    np.sqrt(np.mean([a["se"][master] ** 2 for a in acc]) / steps))
        out["expand_%d" % ex] = {"ms_per_extraction": dt * 1e3, "walks_per_s": walks / dt,
                                 "hops_per_walk": s["hops"] / s["walks"],
                                 "micro_steps_per_walk": s["micro_steps"] / s["walks"],
                                 "C_mm": rows[ex][0]}
    h.close()
    out["C_mm_shift_rel"] = float(rows[5][0] / rows[0][0] - 1)
    out["C_mm_shift_z"] = float((rows[5][0] - rows[0][0]) / np.hypot(rows[5][1], rows[0][1]))
    out["speedup"] = out["expand_0"]["ms_per_extraction"] / out["expand_5"]["ms_per_extraction"]
    return out


def c4_to_target(mw, W, target=0.01, budget=100000000, reps=3):
    """The large interconnect (C4: 20x20x2 um, 192 wires) walked until the
    master's self capacitance reaches 3 SE / |C_mm| <= target (Alg. 1 with
    the stopping rule on the running estimate): walks, time and throughput
    of each run, with the error reached."""
    st = W.c4_structure()
    m = st.meta["master"]
    h = mw.StructureHandle(st)
    mw.frw_extract(h, m, 1000000, seed=800)  # table cache warm, as in a long-running process
    runs = []
    for k in range(reps):
        t0 = time.perf_counter()
        r = mw.frw_extract(h, m, budget, seed=810 + k, target_rel_3sigma=target)
        dt = time.perf_counter() - t0
        s = r["stats"]
        runs.append({"walks": s["walks"], "ms": dt * 1e3, "walks_per_s": s["walks"] / dt,
                     "micro_steps_per_s": s["micro_steps"] / dt,
                     "rel_3sigma_reached": float(3 * r["se"][m] / abs(r["row"][m])), "C_mm": float(r["row"][m])})
    h.close()
    return {"workload": "C4 interconnect, master %d, n = 16, stop at 3 SE / |C_mm| <= %g" % (m, target),
            "runs": runs, "median_walks_per_s": float(np.median([q["walks_per_s"] for q in runs]))}


def fig3a(mw, W, ns=(4, 8, 12, 16, 20, 24, 28, 32), count=500, walks=4096):
    """Fig. 3(a) study: E(tau) of MicroWalk over `count` cubes per lattice
    size with randomly placed blocks of exponentially distributed
    permittivity, each cube's E(tau) estimated by the mean step count of
    `walks` walks from one batched launch per size; min/mean/max per n and the
    log-log slope of the mean (O(N^2) expected)."""
    import torch
    rows = {}
    total_steps, total_s = 0, 0.0
    for n in ns:
        cubes = W.fig3a_cubes(n, count)
        packed = mw.pack_cubes(cubes)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        _, steps, off = mw.mw_transition_batch(None, [walks] * count, packed=packed, seed=3)
        torch.cuda.synchronize()
        dt = time.perf_counter() - t0
        per = steps[:count * walks].view(count, walks).double().mean(dim=1).cpu().numpy()
        rows[str(n)] = {"min": float(per.min()), "mean": float(per.mean()), "max": float(per.max()),
                        "mean_over_n2": float(per.mean() / n ** 2), "ms": dt * 1e3}
        total_steps += int(steps[:count * walks].sum(dtype=torch.int64))
        total_s += dt
    means = [rows[str(n)]["mean"] for n in ns]
    slope = float(np.polyfit(np.log(ns), np.log(means), 1)[0])
    return {"workload": "%d cubes per n, 1-6 blocks, eps ~ Exp(rate 0.1) clipped at 0.01, %d walks per cube"
                        % (count, walks),
            "per_n": rows, "loglog_slope": slope, "micro_steps_per_s": total_steps / total_s}


def serving(mw, W, n_req=300, loads=(0.5, 0.8, 1.2)):
    """Request stream built like the serving workload (windows of 4-200
    conductors, budgets 1e5-1e7 walks, Poisson arrivals at load x the serial
    plain service rate): served with continuous batching vs serial plain
    extraction (FIFO) on the same GPU, at each load."""
    reqs = W.c5_requests(n_req)
    service = []
    for st, m, b, seed in reqs:
        t0 = time.perf_counter()
        h = mw.StructureHandle(st)
        mw.frw_extract(h, m, b, seed=seed)
        h.close()
        service.append(time.perf_counter() - t0)
    service = np.array(service)
    mu = n_req / service.sum()
    walks = float(sum(r[2] for r in reqs))
    out = {"workload": "%d requests, 4-200 conductors, budgets 1e5-1e7 (%.3g walks), Poisson "
                       "arrivals at load x serial plain service rate (%.2f req/s)" % (n_req, walks, mu)}
    for load in loads:
        lam = load * mu
        rng = np.random.default_rng(55)
        arr = np.cumsum(rng.exponential(1.0 / lam, n_req))
        arr -= arr[0]
        t_free, lat_plain = 0.0, []
        for a, sv in zip(arr, service):
            start = max(a, t_free)
            t_free = start + sv
            lat_plain.append(t_free - a)
        srv = mw.Server(8 << 30)
        t0 = time.perf_counter()
        tickets = []
        for (st, m, b, seed), a in zip(reqs, arr):
            while time.perf_counter() - t0 < a:
                time.sleep(0.0002)
            tickets.append(srv.submit(st, m, b, seed))
        res = [srv.wait(t) for t in tickets]
        makespan = time.perf_counter() - t0
        stats = srv.stats()
        srv.close()
        lat = np.array([r["latency"] for r in res])
        out["load_%.1f" % load] = {
            "p50_ms": float(np.percentile(lat, 50) * 1e3), "p99_ms": float(np.percentile(lat, 99) * 1e3),
            "plain_p50_ms": float(np.percentile(lat_plain, 50) * 1e3),
            "plain_p99_ms": float(np.percentile(lat_plain, 99) * 1e3),
            "walks_per_s": walks / makespan, "plain_walks_per_s": walks / t_free,
            "max_concurrent": stats["max_concurrent"], "rounds": stats["rounds"]}
    return out


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--walks", type=int, default=1000000)
    ap.add_argument("--n-cells", type=int, default=16)
    ap.add_argument("--cpu-walks", type=int, default=900000)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-extras", action="store_true", help="skip the batched and serving comparisons")
    ap.add_argument("--serving-requests", type=int, default=300,
                    help="requests of the serving comparison (0 skips it)")
    ap.add_argument("--copy-probe-mib", type=int, default=0,
                    help="only copy a device buffer of this size 3 times (calibrates the rocprofv3 "
                         "FETCH_SIZE / WRITE_SIZE counters against a known byte count) and exit")
    args = ap.parse_args()
    if args.gpus != 1:
        print("bench.py runs on one GPU only: the library has single-GPU kernels only "
              "(walk ranges would shard across GPUs with one fp64 all-reduce of the per-net "
              "sums; not implemented).", file=sys.stderr)
        sys.exit(2)


    import torch

    if args.copy_probe_mib:
        n = args.copy_probe_mib << 18  # float32 elements
        a = torch.ones(n, device="cuda")
        b = torch.empty_like(a)
        torch.cuda.synchronize()
        for _ in range(3):
            b.copy_(a)
        torch.cuda.synchronize()
        print(json.dumps({"copy_probe_bytes_per_copy": n * 4, "copies": 3}))
        return

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
    rows, ses = [], []
    for k in range(args.steps):
        r = mw.frw_extract(h, 0, args.walks, seed=k, n_cells=args.n_cells)
        rows.append(r["row"])
        ses.append(r["se"])
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
    if not args.no_extras:
        out["batched"] = batched_vs_plain(mw, W)
        out["fig3a"] = fig3a(mw, W)
        out["microwalk_e"] = microwalk_e(mw, W, st, args.walks, args.n_cells)
        c4 = W.c4_structure()
        out["microwalk_e_c4"] = microwalk_e(mw, W, c4, args.walks, args.n_cells, master=c4.meta["master"])
        out["c4_to_1pct"] = c4_to_target(mw, W)
        if args.serving_requests > 0:
            out["serving"] = serving(mw, W, args.serving_requests)
    if not args.no_cpu_baseline:
        out["cpu_baseline"], r_or = cpu_baseline(st, args.cpu_walks, seed=7)
        # accuracy beside throughput: the timed extractions' mean row against
        # the oracle's row, entry by entry, in combined standard errors
        g_row = np.mean(rows, axis=0)
        g_se = np.sqrt(np.mean(np.square(ses), axis=0) / len(rows))
        den = np.hypot(g_se, r_or["se"])
        z = np.where(den > 0, np.abs(g_row - r_or["row"]) / np.where(den > 0, den, 1.0), 0.0)
        out["oracle_agreement"] = {"gpu_row": g_row.tolist(), "gpu_se": g_se.tolist(),
                                   "oracle_row": list(map(float, r_or["row"])),
                                   "oracle_se": list(map(float, r_or["se"])), "max_z": float(z.max())}
    print(json.dumps(out))


if __name__ == "__main__":
    main()
