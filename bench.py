#!/usr/bin/env python3
"""Benchmark of FRW capacitance extraction with MicroWalk transitions on one
MI355X.

Workload (one step): frw_extract on the large interconnect window (20x20x2 um,
three metal layers of 64 wires, layered eps 3.9 / 2.7 dielectric, 20 nm eps 7.0
coatings, eps 25 gap fills; 192 nets), the middle-layer wire nearest the window
centre as master, 16^3-cell transition cubes, walked until 3 SE / |C_mm| <= 1 %
(Alg. 1 with the stopping rule checked every convergence batch), a fresh seed
per step.  The structure and its transition-table cache are resident on the
device when the timed region starts.  Prints one JSON line (keys below); the
extras compare the crossing-wire workload, the single-cube and batched
MicroWalk workloads, the plain forms, MicroWalk-E and serving.

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
# 8 slots + 2 three-input xors) / 4 = 25) and about 15 for the direction
# (five threshold compares), the move and the boundary test: 40 slots.
MW_STEP_SLOTS = 40
WALKER_SRC = os.path.join(ROOT, "paper_2507_09730_amd", "csrc", "frw.hip")
TRAFFIC_FILE = os.path.join(ROOT, "profiles", "frw_walk_kernel_c4_traffic.txt")


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


def _progress(msg):
    """One line on stderr per finished section (the JSON result goes to stdout)."""
    print("[bench] %s" % msg, file=sys.stderr, flush=True)


def _cores():
    cores = len(os.sched_getaffinity(0)) if hasattr(os, "sched_getaffinity") else os.cpu_count()
    return max(1, min(cores, 64))


def cpu_baseline(st, master, walks_all, walks_one, seed):
    """The oracle on the same workload, a bounded sample of walks: all host
    cores (threads over walk ranges) and one thread."""
    import oracle
    cores = _cores()
    oracle.build()
    t0 = time.perf_counter()
    r = oracle.frw_extract(st, master, walks_all, seed=seed, threads=cores)
    dt = time.perf_counter() - t0
    t1 = time.perf_counter()
    r1 = oracle.frw_extract(st, master, walks_one, seed=seed + 1, threads=1)
    dt1 = time.perf_counter() - t1
    return {"value": walks_all / dt, "unit": "walks/s", "cores": cores, "kind": "oracle",
            "sample": "%d walks of the same workload and master, binary64 C++ oracle, %d threads over "
                      "walk ranges, %.1f s (%.4g micro-steps/s); one thread: %d walks in %.1f s"
                      % (walks_all, cores, dt, r["stats"]["micro_steps"] / dt, walks_one, dt1),
            "micro_steps_per_s": r["stats"]["micro_steps"] / dt,
            "one_thread_walks_per_s": walks_one / dt1,
            "one_thread_micro_steps_per_s": r1["stats"]["micro_steps"] / dt1}, r


def err_avg(row, ref):
    """The paper's average capacitance error (Sec. IV): sum |C - C_ref| over
    the row's capacitances / sum |C_ref| (the env column excluded)."""
    row, ref = np.asarray(row)[:-1], np.asarray(ref)[:-1]
    return float(np.abs(row - ref).sum() / np.abs(ref).sum())


def agreement(rows, ses, r_or):
    """Mean of the timed GPU rows against an oracle row, on the entries both
    resolve (|C| > 4 SE), in combined standard errors; and Err_avg of the
    mean row against the oracle's (both Monte Carlo estimates, so it holds
    the two samples' statistical error as well)."""
    g_row = np.mean(rows, axis=0)
    g_se = np.sqrt(np.mean(np.square(ses), axis=0) / len(rows))
    o_row, o_se = np.asarray(r_or["row"]), np.asarray(r_or["se"])
    both = (np.abs(g_row) > 4 * g_se) & (np.abs(o_row) > 4 * o_se)
    z = np.abs(g_row - o_row)[both] / np.hypot(g_se, o_se)[both]
    # E|X| of a zero-mean normal is sqrt(2 / pi) sigma: the Err_avg that the
    # two samples' standard errors alone would give
    noise = float(np.sqrt(2 / np.pi) * np.hypot(g_se, o_se)[:-1].sum() / np.abs(o_row[:-1]).sum())
    return {"entries_compared": int(both.sum()), "max_z": float(z.max()) if z.size else None,
            "mean_z2": float(np.mean(z ** 2)) if z.size else None, "err_avg": err_avg(g_row, o_row),
            "err_avg_noise": noise}


def c1_single_cube(mw, W, reps=20):
    """Single-cube MicroWalk (8^3 cells, eps 3.9 with an eps 7.0 block, 1e5
    walks from the centre): one mw_transition call per repetition."""
    import torch
    eps_h = W.c1_eps()
    eps = torch.as_tensor(eps_h).cuda()
    hits = torch.empty(100000, dtype=torch.int32, device="cuda")
    steps = torch.empty(100000, dtype=torch.int32, device="cuda")
    mw.mw_transition(eps, 100000, seed=0, hits=hits, steps=steps)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for k in range(reps):
        mw.mw_transition(eps, 100000, seed=k, hits=hits, steps=steps)
    torch.cuda.synchronize()
    dt = (time.perf_counter() - t0) / reps
    n_steps = int(steps.sum(dtype=torch.int64))
    return {"workload": "8^3-cell cube, eps 3.9 with an eps 7.0 block at cells [1,4)x[1,5)x[3,8), "
                        "1e5 walks from the centre (one mw_transition call)",
            "ms_per_call": dt * 1e3, "walks_per_s": 1e5 / dt, "micro_steps_per_s": n_steps / dt,
            "mean_steps": n_steps / 1e5}


def cpu_baseline_c1(W):
    """The oracle's MicroWalk on the single-cube workload (one thread)."""
    import oracle
    t0 = time.perf_counter()
    _, so = oracle.microwalk(W.c1_eps(), 0, 100000, seed=1)
    dt = time.perf_counter() - t0
    return {"walks_per_s": 1e5 / dt, "micro_steps_per_s": float(so.sum()) / dt, "threads": 1}


def c2_figures(mw, W, steps=20, walks=1000000, n_cells=16):
    """Crossing wires (4 nets), 1e6 walks per extraction: the persistent
    walker and the plain form (one walker launch per transition round)."""
    st = W.c2_structure()
    h = mw.StructureHandle(st)
    out, rows, ses = {}, [], []
    for plain, reps in ((0, steps), (1, 5)):
        mw.frw_extract(h, 0, walks, seed=9000, n_cells=n_cells, plain=plain)
        t0 = time.perf_counter()
        wsum = ssum = wk = launches = 0
        for k in range(reps):
            r = mw.frw_extract(h, 0, walks, seed=k, n_cells=n_cells, plain=plain)
            s = r["stats"]
            wsum += s["walks"]
            ssum += s["micro_steps"]
            wk += s["walker_seconds"]
            launches += s["launches"]
            if not plain:
                rows.append(r["row"])
                ses.append(r["se"])
        dt = time.perf_counter() - t0
        out["plain" if plain else "persistent"] = {
            "ms_per_extraction": dt / reps * 1e3, "walks_per_s": wsum / dt, "micro_steps_per_s": ssum / dt,
            "walker_ms_per_extraction": wk / reps * 1e3, "walker_launches_per_extraction": launches / reps,
            "roofline_frac": ssum * MW_STEP_SLOTS / wk / PEAK_LANE_OPS}
    h.close()
    out["workload"] = "crossing wires 2x2x1 um, 4 nets, master 0, %d^3-cell cubes, %d walks per extraction" % (
        n_cells, walks)
    out["rel_3sigma_Cmm"] = float(np.mean([3 * e[0] / r[0] for r, e in zip(rows, ses)]))
    out["persistent_speedup_over_plain"] = out["plain"]["ms_per_extraction"] / out["persistent"]["ms_per_extraction"]
    return out, rows, ses


def cell_lattice(mw, W, steps=10, walks=1000000, n_cells=15):
    """Crossing wires (4 nets), 1e6 walks per extraction on the cell-centred
    lattice of Sec. III-A (15^3-cell cubes, nodes at the voxel centres)."""
    st = W.c2_structure()
    h = mw.StructureHandle(st)
    kw = dict(n_cells=n_cells, lattice=mw.MW_LATTICE_CELL)
    mw.frw_extract(h, 0, walks, seed=9000, **kw)
    rows, ses = [], []
    wsum = ssum = wk = hops = 0
    t0 = time.perf_counter()
    for k in range(steps):
        r = mw.frw_extract(h, 0, walks, seed=k, **kw)
        s = r["stats"]
        wsum += s["walks"]
        ssum += s["micro_steps"]
        hops += s["hops"]
        wk += s["walker_seconds"]
        rows.append(r["row"])
        ses.append(r["se"])
    dt = time.perf_counter() - t0
    h.close()
    out = {"workload": "crossing wires 2x2x1 um, 4 nets, master 0, cell-centred lattice, %d^3-cell cubes, "
                       "%d walks per extraction" % (n_cells, walks),
           "ms_per_extraction": dt / steps * 1e3, "walks_per_s": wsum / dt, "micro_steps_per_s": ssum / dt,
           "walker_ms_per_extraction": wk / steps * 1e3, "hops_per_walk": hops / wsum,
           "micro_steps_per_walk": ssum / wsum,
           "C_mm": float(np.mean([r[0] for r in rows])),
           "rel_3sigma_Cmm": float(np.mean([3 * e[0] / r[0] for r, e in zip(rows, ses)]))}
    return out, rows, ses


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
    rows, full = {}, {}
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
        full[ex] = np.mean([a["row"] for a in acc], axis=0)
        out["expand_%d" % ex] = {"ms_per_extraction": dt * 1e3, "walks_per_s": walks / dt,
                                 "hops_per_walk": s["hops"] / s["walks"],
                                 "micro_steps_per_walk": s["micro_steps"] / s["walks"],
                                 "C_mm": rows[ex][0]}
    h.close()
    out["C_mm_shift_rel"] = float(rows[5][0] / rows[0][0] - 1)
    out["C_mm_shift_z"] = float((rows[5][0] - rows[0][0]) / np.hypot(rows[5][1], rows[0][1]))
    # the paper's Table III accuracy measure, plain MicroWalk as the reference
    out["err_avg_vs_plain"] = err_avg(full[5], full[0])
    out["speedup"] = out["expand_0"]["ms_per_extraction"] / out["expand_5"]["ms_per_extraction"]
    return out


def c4_plain_vs_persistent(mw, h, master, walks, reps=3):
    """The large interconnect at a fixed walk count (the headline's mean walks
    to 1 %): persistent walker launches against the plain form."""
    out = {}
    for plain in (0, 1):
        mw.frw_extract(h, master, walks, seed=700, plain=plain)
        t0 = time.perf_counter()
        wk = 0.0
        launches = 0
        for k in range(reps):
            r = mw.frw_extract(h, master, walks, seed=710 + k, plain=plain)
            wk += r["stats"]["walker_seconds"]
            launches += r["stats"]["launches"]
        dt = (time.perf_counter() - t0) / reps
        out["plain" if plain else "persistent"] = {"ms_per_extraction": dt * 1e3, "walks_per_s": walks / dt,
                                                   "walker_ms": wk / reps * 1e3,
                                                   "walker_launches": launches / reps}
    out["walks"] = walks
    out["persistent_speedup_over_plain"] = out["plain"]["ms_per_extraction"] / out["persistent"]["ms_per_extraction"]
    return out


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


def serving(mw, W, n_req=2000, loads=(0.5, 0.8, 1.2)):
    """Request stream built like the serving workload (windows of 4-200
    conductors, budgets 1e5-1e7 walks, Poisson arrivals at load x the serial
    plain service rate): served with continuous batching against serial plain
    extraction on the same GPU.  The serial plain latencies are a FIFO queue
    model over the measured per-request service times (structure upload and
    frw_extract, one request at a time): serial service does not depend on
    the arrival pattern, so the model gives the latency a serial server
    would have on the same arrival trace.  Both forms run after a warm-up
    pass, with the transition tables of the windows cached."""
    reqs = W.c5_requests(n_req)
    # warm-up: every request once through the server at full rate, so that
    # the serial and the served runs below both find the transition tables
    # of these windows in the cache (a long-running process)
    srv = mw.Server(8 << 30)
    t0 = time.perf_counter()
    for t in [srv.submit(st, m, b, seed) for st, m, b, seed in reqs]:
        srv.wait(t)
    srv.close()
    _progress("serving: warm-up pass over %d requests in %.1f s" % (n_req, time.perf_counter() - t0))
    service = []
    for st, m, b, seed in reqs:
        t0 = time.perf_counter()
        h = mw.StructureHandle(st)
        mw.frw_extract(h, m, b, seed=seed)
        h.close()
        service.append(time.perf_counter() - t0)
    service = np.array(service)
    _progress("serving: serial plain pass over %d requests in %.1f s" % (n_req, service.sum()))
    mu = n_req / service.sum()
    walks = float(sum(r[2] for r in reqs))
    out = {"workload": "%d requests, 4-200 conductors, budgets 1e5-1e7 (%.3g walks), Poisson "
                       "arrivals at load x serial plain service rate (%.2f req/s)" % (n_req, walks, mu),
           "plain_latency": "FIFO model over measured serial service times"}
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
        _progress("serving load %.1f: %d requests in %.1f s" % (load, n_req, makespan))
        out["load_%.1f" % load] = {
            "p50_ms": float(np.percentile(lat, 50) * 1e3), "p99_ms": float(np.percentile(lat, 99) * 1e3),
            "plain_p50_ms": float(np.percentile(lat_plain, 50) * 1e3),
            "plain_p99_ms": float(np.percentile(lat_plain, 99) * 1e3),
            "walks_per_s": walks / makespan, "plain_walks_per_s": walks / t_free,
            "max_concurrent": stats["max_concurrent"], "rounds": stats["rounds"]}
    return out


def headline(mw, W, steps, warmup, target):
    """The large interconnect walked to 3 SE / |C_mm| <= target, `steps`
    timed extractions after `warmup` untimed ones (the first builds the
    transition tables the structure needs)."""
    import torch
    st = W.c4_structure()
    m = st.meta["master"]
    h = mw.StructureHandle(st)
    budget = 100000000
    for i in range(warmup):
        mw.frw_extract(h, m, budget, seed=10000 + i, target_rel_3sigma=target)
    torch.cuda.synchronize()
    acc = {"walks": 0, "walks_launched": 0, "micro_steps": 0, "launches": 0, "walker_s": 0.0, "hops": 0,
           "rel": [], "rows": [], "ses": [], "halved": 0}
    t0 = time.perf_counter()
    for k in range(steps):
        r = mw.frw_extract(h, m, budget, seed=k, target_rel_3sigma=target)
        s = r["stats"]
        acc["walks"] += s["walks"]
        acc["walks_launched"] += s["walks_launched"]
        acc["micro_steps"] += s["micro_steps"]
        acc["launches"] += s["launches"]
        acc["walker_s"] += s["walker_seconds"]
        acc["hops"] += s["hops"]
        acc["halved"] += s["cube_halved"]
        acc["rel"].append(3 * r["se"][m] / abs(r["row"][m]))
        acc["rows"].append(r["row"])
        acc["ses"].append(r["se"])
    torch.cuda.synchronize()
    acc["dt"] = time.perf_counter() - t0
    return st, m, h, acc


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--target", type=float, default=0.01, help="3 SE / |C_mm| at which an extraction stops")
    ap.add_argument("--cpu-walks", type=int, default=40000, help="oracle sample, all host cores")
    ap.add_argument("--cpu-walks-one", type=int, default=1000, help="oracle sample, one thread")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-extras", action="store_true", help="skip the comparison workloads")
    ap.add_argument("--serving-requests", type=int, default=2000,
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
    st, m, h, acc = headline(mw, W, args.steps, args.warmup, args.target)
    dt = acc["dt"]
    # roofline of the walker kernel (dominant kernel): algorithmic MicroWalk
    # slots of the timed launches / their summed duration (HIP events on the
    # launch stream)
    achieved = acc["micro_steps"] * MW_STEP_SLOTS / acc["walker_s"] / 1e12  # T lane-op slots/s
    peak = PEAK_LANE_OPS / 1e12
    out = {
        "metric": METRIC, "value": acc["walks"] / dt, "unit": "walks/s", "n_gpus": 1, "steps": args.steps,
        "warmup": args.warmup, "ms_per_step": dt / args.steps * 1e3, "higher_is_better": True,
        "scaling": "weak", "vs_baseline": None, "dtype": "u32", "data": "synthetic",
        "config": {"workload": "large interconnect 20x20x2 um: 3 metal layers x 64 wires (192 nets), "
                               "eps 3.9/2.7 dielectric stack, 20 nm eps-7 coatings, eps-25 gap fills; "
                               "master net %d; 16^3-cell cubes; each step walks until 3 SE/|C_mm| <= %g"
                               % (m, args.target),
                   "target_rel_3sigma": args.target, "n_cells": 16, "hybrid": 1, "master": m},
        # every micro-step walked, including those of walks after the
        # stopping checkpoint (dropped from the row)
        "micro_steps_per_s": acc["micro_steps"] / dt,
        "walks_per_step": acc["walks"] / args.steps,
        "walks_launched_per_step": acc["walks_launched"] / args.steps,
        "ms_to_target": dt / args.steps * 1e3,
        "rel_3sigma_reached": float(np.mean(acc["rel"])),
        "hops_per_walk": acc["hops"] / acc["walks_launched"],
        "cube_halved": acc["halved"],
        "walker_kernel_ms_per_step": acc["walker_s"] / args.steps * 1e3,
        "walker_launches_per_step": acc["launches"] / args.steps,
        "roofline": {"bound": "alu", "kernel": "frw_walk_kernel", "achieved": achieved, "peak": peak,
                     "unit": "TOP/s", "frac": achieved / peak, "traffic": _traffic()},
    }
    extras_rows = {}
    _progress("headline: %d extractions to target in %.2f s" % (args.steps, dt))
    if not args.no_extras:
        out["c4_plain_vs_persistent"] = c4_plain_vs_persistent(mw, h, m, int(round(out["walks_per_step"] / 1e5)) * 100000)
        _progress("c4 plain vs persistent")
        out["c2"], extras_rows["c2_rows"], extras_rows["c2_ses"] = c2_figures(mw, W)
        _progress("c2")
        out["cell_lattice"], extras_rows["cell_rows"], extras_rows["cell_ses"] = cell_lattice(mw, W)
        # the two lattices' C2 rows (means of the timed extractions) in the
        # paper's accuracy measure, the vertex lattice as the reference
        out["cell_lattice"]["err_avg_vs_vertex"] = err_avg(np.mean(extras_rows["cell_rows"], axis=0),
                                                           np.mean(extras_rows["c2_rows"], axis=0))
        _progress("cell lattice")
        out["c1"] = c1_single_cube(mw, W)
        out["batched"] = batched_vs_plain(mw, W)
        _progress("c1, batched")
        out["fig3a"] = fig3a(mw, W)
        _progress("fig3a")
        out["microwalk_e"] = microwalk_e(mw, W, W.c2_structure(), 1000000, 16)
        out["microwalk_e_c4"] = microwalk_e(mw, W, st, 1000000, 16, master=m)
        _progress("microwalk-e")
        if args.serving_requests > 0:
            out["serving"] = serving(mw, W, args.serving_requests)
    h.close()
    if not args.no_cpu_baseline:
        out["cpu_baseline"], r_or = cpu_baseline(st, m, args.cpu_walks, args.cpu_walks_one, seed=7)
        # accuracy beside throughput: the timed extractions' mean row against
        # the oracle's row
        out["oracle_agreement"] = agreement(acc["rows"], acc["ses"], r_or)
        _progress("cpu baseline")
        if not args.no_extras:
            import oracle
            out["c1"]["oracle"] = cpu_baseline_c1(W)
            r2 = oracle.frw_extract(W.c2_structure(), 0, 200000, seed=7, threads=_cores())
            out["c2"]["oracle_agreement"] = agreement(extras_rows["c2_rows"], extras_rows["c2_ses"], r2)
            r3 = oracle.frw_extract(W.c2_structure(), 0, 100000, seed=7, threads=_cores(), n_cells=15, lattice=1)
            out["cell_lattice"]["oracle_agreement"] = agreement(extras_rows["cell_rows"], extras_rows["cell_ses"],
                                                                r3)
    print(json.dumps(out))


if __name__ == "__main__":
    main()
