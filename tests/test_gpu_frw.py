"""GPU FRW extraction (Alg. 1 with the hybrid strategy of Sec. III-C) through
the C ABI, against closed forms, Maxwell-matrix properties and the CPU oracle.

Capacitances are Monte Carlo estimates: rows are compared in combined
standard errors (3 sigma).  Walks are compared one by one as well: GPU and
oracle draw every random word from the same Philox streams (walk, hop, step,
purpose), so a walk follows the same path on both until an fp32 decision of
the GPU differs from the oracle's fp64 one (a point within rounding of a box
face or a lattice boundary); nearly every walk must end on the same net with
the same weight to fp32 rounding.  Per-walk scores are integer- and
seed-determined, so repeated or resumed runs must reproduce them exactly.
"""
import os

import numpy as np
import pytest

import workloads as W
from _stats import z_crit

pytestmark = pytest.mark.gpu


def _threads():
    try:
        return max(1, min(16, len(os.sched_getaffinity(0))))
    except AttributeError:
        return 4


@pytest.fixture(scope="module")
def mw():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_2507_09730_amd as lib
    lib.mw_init(0)
    return lib


def _z(a, b, sa, sb):
    return abs(a - b) / np.sqrt(sa ** 2 + sb ** 2)


def test_plates_uniform_small(mw):
    st = W.parallel_plates("uniform")
    r = mw.frw_extract(st, 0, 20000, seed=1)
    exact = W.parallel_plates_exact("uniform")
    print("plates uniform", r["row"], r["se"], r["stats"])
    assert abs(r["row"][0] - exact) < 3 * r["se"][0]
    assert r["row"][2] == 0.0
    assert r["stats"]["walks"] == 20000


@pytest.mark.parametrize("variant,hybrid", [("uniform", 1), ("uniform", 0), ("columns", 0),
                                            ("columns", 1), ("checkerboard", 1)])
def test_plates_closed_forms(mw, variant, hybrid):
    st = W.parallel_plates(variant)
    r = mw.frw_extract(st, 0, 400000, seed=2, hybrid=hybrid)
    exact = W.parallel_plates_exact(variant)
    print(variant, hybrid, r["row"], r["se"], (r["row"][0] - exact) / r["se"][0])
    assert abs(r["row"][0] - exact) < 3 * r["se"][0]
    assert abs(r["row"][1] + exact) < 3 * r["se"][1]


@pytest.fixture(scope="module")
def c2_gpu(mw):
    st = W.c2_structure()
    h = mw.StructureHandle(st)
    out = {m: mw.frw_extract(h, m, 1000000, seed=20 + m, scores=True) for m in (0, 1)}
    for m in (0, 1):
        print("gpu master", m, out[m]["row"], out[m]["se"], out[m]["stats"])
    return out


def test_c2_matches_oracle(c2_gpu, oracle_lib):
    st = W.c2_structure()
    r_or = oracle_lib.frw_extract(st, 0, 100000, seed=77, threads=_threads())
    r_gpu = c2_gpu[0]
    print("oracle", r_or["row"], r_or["se"], r_or["stats"])
    zs = [_z(r_gpu["row"][j], r_or["row"][j], r_gpu["se"][j], r_or["se"][j]) for j in range(5)]
    print("z", zs)
    assert max(zs) < 3.0


# walks whose weights agree to this relative error count as equal (the GPU
# weight is fp32: one walk's weight is a product and quotient of a few fp32
# terms, a few ulp of 6e-8 apart from the fp64 value)
W_REL = 1e-5


def _walk_agreement(g, o_net, o_w):
    g_net = g["net"].cpu().numpy() if hasattr(g["net"], "cpu") else np.asarray(g["net"])
    g_w = (g["w"].cpu().numpy() if hasattr(g["w"], "cpu") else np.asarray(g["w"])).astype(np.float64)
    same = g_net == o_net
    rel = np.abs(g_w - o_w) / np.maximum(np.abs(o_w), 1e-30)
    return float(same.mean()), float((same & (rel <= W_REL)).mean())


@pytest.mark.parametrize("name,expand,n_cells,floor", [
    ("plates", 0, 16, 0.999), ("stack", 0, 16, 0.999), ("c2", 0, 16, 0.999), ("c4", 0, 16, 0.995),
    ("c2", 5, 16, 0.99), ("c2", 0, 8, 0.999), ("c2", 0, 12, 0.999), ("c2", 0, 24, 0.999), ("c2", 0, 32, 0.999)])
def test_walks_match_oracle_one_by_one(mw, oracle_lib, name, expand, n_cells, floor):
    """Cube sizes above 16 cells run the walker's general MicroWalk step, the
    twelve-layer stack its background-layer walk over global memory."""
    st = {"plates": W.parallel_plates, "stack": lambda: W.parallel_plates("stack"), "c2": W.c2_structure,
          "c4": W.c4_structure}[name]()
    m = st.meta["master"] if name == "c4" else 0
    N = 20000 if n_cells <= 16 else 5000
    g = mw.frw_extract(st, m, N, seed=77, scores=True, expand=expand, n_cells=n_cells)
    o = oracle_lib.frw_extract(st, m, N, seed=77, threads=_threads(), scores=True, n_cells=n_cells,
                               expand=float(expand) if expand else 1.0, kernel_limits=True)
    same_net, same_walk = _walk_agreement(g, o["net"], o["w"])
    # the oracle reproduces the kernel's capacity rule here (kernel_limits);
    # cube_halved counts the transitions where that rule applied
    print(name, expand, n_cells, "same net", same_net, "same net and weight", same_walk,
          "halved cubes", g["stats"]["cube_halved"], "of", g["stats"]["hops"] + N)
    if name in ("plates", "stack") or (name == "c2" and not expand):
        assert g["stats"]["cube_halved"] == 0
    assert same_walk >= floor


def test_c2_full_size_sampled_walks_match_oracle(c2_gpu, oracle_lib):
    """The bench configuration (1e6 walks, 16^3-cell cubes, hybrid): eight
    runs of 250 walks spread over the extraction, recomputed by the oracle
    from their walk indices, equal the GPU's walks one by one."""
    st = W.c2_structure()
    g = c2_gpu[0]
    n_walks = len(g["net"])
    assert n_walks == 1000000
    agree = []
    for f in np.linspace(0, n_walks - 250, 8).astype(np.int64):
        o = oracle_lib.frw_extract(st, 0, 250, seed=20, first_walk=int(f), threads=_threads(), scores=True,
                                   kernel_limits=True)
        part = {"net": g["net"][f:f + 250], "w": g["w"][f:f + 250]}
        agree.append(_walk_agreement(part, o["net"], o["w"])[1])
    print("per-run agreement", agree)
    assert min(agree) >= 0.99 and np.mean(agree) >= 0.999


def test_c2_reciprocity_and_signs(c2_gpu):
    r0, r1 = c2_gpu[0], c2_gpu[1]
    assert _z(r0["row"][1], r1["row"][0], r0["se"][1], r1["se"][0]) < 3
    for m, r in c2_gpu.items():
        row, se = r["row"], r["se"]
        assert row[m] > 0
        assert all(row[j] <= 3 * se[j] for j in range(len(row)) if j != m)
        assert 3 * se[m] / row[m] < 0.015  # about 1.1% 3-sigma on C_mm at 1e6 walks


def test_c2_row_sums_to_zero(c2_gpu):
    for m, r in c2_gpu.items():
        w = r["w"].double().cpu().numpy()
        assert abs(w.mean()) < 3 * w.std() / np.sqrt(w.size)


def test_c2_reduction_matches_fp64_resum(c2_gpu):
    """fp32 compensated block sums + fp64 grand reduction vs an fp64 re-sum of
    the same per-walk fp32 scores: 1e-6 relative."""
    for m, r in c2_gpu.items():
        net = r["net"].cpu().numpy()
        w = r["w"].cpu().numpy().astype(np.float64)
        K = len(r["row"])
        resum = np.bincount(net, weights=w, minlength=K) / w.size
        floor = 1e-6 * abs(resum[m])
        assert np.all(np.abs(r["row"] - resum) <= 1e-6 * np.abs(resum) + floor * 1e-3), (r["row"], resum)
        sq = np.bincount(net, weights=w * w, minlength=K) / w.size
        se = np.sqrt(np.maximum(sq - resum ** 2, 0) / (w.size - 1))
        assert np.allclose(r["se"], se, rtol=1e-5, atol=1e-12)


def test_c4_reduction_matches_fp64_resum(mw):
    """The 193-column row of the large interconnect (most nets absent from a
    given 4096-walk slice of the reduction) against an fp64 re-sum of the
    same per-walk fp32 scores."""
    st = W.c4_structure()
    m = st.meta["master"]
    r = mw.frw_extract(st, m, 300000, seed=44, scores=True)
    net = r["net"].cpu().numpy()
    w = r["w"].cpu().numpy().astype(np.float64)
    K = len(r["row"])
    resum = np.bincount(net, weights=w, minlength=K) / w.size
    scale = np.abs(resum).max()
    assert np.all(np.abs(r["row"] - resum) <= 1e-6 * np.abs(resum) + 1e-9 * scale)
    sq = np.bincount(net, weights=w * w, minlength=K) / w.size
    se = np.sqrt(np.maximum(sq - resum ** 2, 0) / (w.size - 1))
    assert np.allclose(r["se"], se, rtol=1e-5, atol=1e-12)
    assert (r["row"][np.bincount(net, minlength=K) == 0] == 0).all()


def test_c2_hybrid_equals_all_microwalk(mw, c2_gpu):
    st = W.c2_structure()
    r_mw = mw.frw_extract(st, 0, 1000000, seed=321, hybrid=0)
    r_hy = c2_gpu[0]
    print("all-microwalk", r_mw["row"], r_mw["se"], r_mw["stats"])
    assert r_mw["stats"]["hop_class"][1] + r_mw["stats"]["hop_class"][0] > 0
    zs = [_z(r_hy["row"][j], r_mw["row"][j], r_hy["se"][j], r_mw["se"][j]) for j in range(5)]
    print("z", zs)
    assert max(zs) < z_crit(5)


def test_scores_independent_of_cache_state_and_resume(mw):
    """A cold table cache (walks park and resume) and a warm one give the
    same per-walk scores; so does a run split at walk 7000."""
    import torch
    st = W.c2_structure()
    h = mw.StructureHandle(st)
    a = mw.frw_extract(h, 0, 20000, seed=5, n_cells=12, scores=True)
    b = mw.frw_extract(h, 0, 20000, seed=5, n_cells=12, scores=True)
    assert a["stats"]["launches"] >= 1
    assert torch.equal(a["net"], b["net"]) and torch.equal(a["w"], b["w"])
    c1 = mw.frw_extract(h, 0, 7000, seed=5, n_cells=12, scores=True)
    c2 = mw.frw_extract(h, 0, 13000, seed=5, n_cells=12, first_walk=7000, scores=True)
    assert torch.equal(torch.cat([c1["net"], c2["net"]]), a["net"])
    assert torch.equal(torch.cat([c1["w"], c2["w"]]), a["w"])


def test_cleared_table_cache_keeps_scores(mw):
    """mw_table_cache_clear empties one lattice size's table cache (the
    20-cell one, which no other test uses): the next extraction rebuilds
    every table it needs, and its walks equal those of the warm run bit for
    bit."""
    import torch
    st = W.c2_structure()
    h = mw.StructureHandle(st)
    mw.mw_table_cache_clear(20)
    a = mw.frw_extract(h, 0, 30000, seed=8, n_cells=20, scores=True)
    b = mw.frw_extract(h, 0, 30000, seed=8, n_cells=20, scores=True)
    mw.mw_table_cache_clear(20)
    c = mw.frw_extract(h, 0, 30000, seed=8, n_cells=20, scores=True)
    print("misses cold", a["stats"]["cache_miss"], "warm", b["stats"]["cache_miss"], "cleared",
          c["stats"]["cache_miss"])
    assert a["stats"]["cache_miss"] > 0 and b["stats"]["cache_miss"] == 0
    # (the same keys again; a lane that compares a key row its compute
    # unit's cache still holds from before the row was written adds the key
    # a second time, so the counts may differ slightly)
    assert abs(c["stats"]["cache_miss"] - a["stats"]["cache_miss"]) <= 0.05 * a["stats"]["cache_miss"]
    for r in (b, c):
        assert torch.equal(a["net"], r["net"]) and torch.equal(a["w"], r["w"])
    with pytest.raises(mw.MWError):
        mw.mw_table_cache_clear(33)
    h.close()


@pytest.mark.parametrize("target", [0.0, 0.02])
def test_graph_replays_equal_eager(mw, monkeypatch, target):
    """A structure keeps frw_extract's buffers between calls, and the usual
    launch is captured in a HIP graph on first use and replayed afterwards:
    replay after replay, with eager work of other extractions between them,
    the rows equal those of eager launches (MWALK_FRW_GRAPHS=0) bit for
    bit."""
    st = W.c2_structure()
    h = mw.StructureHandle(st)
    kw = dict(target_rel_3sigma=target, batch_walks=65536) if target else {}
    for k in range(4):
        g = mw.frw_extract(h, 0, 400000, seed=70 + k, **kw)
        monkeypatch.setenv("MWALK_FRW_GRAPHS", "0")
        e = mw.frw_extract(h, 0, 400000, seed=70 + k, **kw)
        monkeypatch.delenv("MWALK_FRW_GRAPHS")
        mw.frw_extract(h, 1, 100000, seed=5)  # other work between the replays
        print(k, g["stats"]["walks"], g["stats"]["launches"], g["stats"]["walker_seconds"],
              e["stats"]["walker_seconds"])
        assert np.array_equal(g["row"], e["row"]) and np.array_equal(g["se"], e["se"])
        assert g["stats"]["walks"] == e["stats"]["walks"]
        if not target:
            # (with a target the launch sizes follow the last call's count)
            for key in ("walks_launched", "hops", "micro_steps", "launches"):
                assert g["stats"][key] == e["stats"][key], key
        assert g["stats"]["walker_seconds"] > 0
    h.close()


@pytest.mark.parametrize("expand", [0, 5])
def test_plain_form_equals_persistent(mw, expand):
    """The plain form (one walker launch per transition round, survivors
    queued for the next launch) gives every walk the same result as the
    persistent launch; it needs as many launches as the longest walk has
    transitions."""
    import torch
    st = W.c2_structure()
    h = mw.StructureHandle(st)
    a = mw.frw_extract(h, 0, 30000, seed=15, scores=True, expand=expand)
    b = mw.frw_extract(h, 0, 30000, seed=15, scores=True, expand=expand, plain=1)
    print("launches persistent", a["stats"]["launches"], "plain", b["stats"]["launches"])
    assert torch.equal(a["net"], b["net"]) and torch.equal(a["w"], b["w"])
    assert b["stats"]["launches"] > 4 * a["stats"]["launches"]
    assert a["stats"]["hops"] == b["stats"]["hops"]
    assert a["stats"]["micro_steps"] == b["stats"]["micro_steps"]


def test_full_table_cache_keeps_results(mw, oracle_lib, monkeypatch):
    """A table cache far too small for the workload (MWALK_TABLE_CAP=200 for
    the 10-cell lattice, which no other test uses) fills again and again:
    walks that meet the full cache park as on a miss, the host builds what
    was queued or empties the cache, and the walks still equal the oracle's
    one by one."""
    monkeypatch.setenv("MWALK_TABLE_CAP", "200")
    st = W.c2_structure()
    g = mw.frw_extract(st, 0, 10000, seed=6, n_cells=10, scores=True)
    monkeypatch.delenv("MWALK_TABLE_CAP")
    o = oracle_lib.frw_extract(st, 0, 10000, seed=6, n_cells=10, threads=_threads(), scores=True,
                               kernel_limits=True)
    same_net, same_walk = _walk_agreement(g, o["net"], o["w"])
    print("cache of 200 tables: misses", g["stats"]["cache_miss"], "launches", g["stats"]["launches"],
          "same walk", same_walk)
    assert g["stats"]["cache_miss"] > 200  # more builds than the cache holds: it was emptied
    assert same_walk >= 0.999


@pytest.mark.parametrize("n_cells,lattice", [(14, 0), (13, 1)])
def test_frw_autotune_keeps_results(mw, monkeypatch, tmp_path, n_cells, lattice):
    """The walker's launch geometry (resident waves per CU) is tuned on a
    lattice size no other test uses (14 cells, and 13 cells of the cell
    lattice), kept in the tune cache file and used by later extractions,
    whose walks stay bit-identical."""
    import json
    import torch
    cache = tmp_path / "tune.json"
    monkeypatch.setenv("MWALK_TUNE_CACHE", str(cache))
    st = W.c2_structure()
    h = mw.StructureHandle(st)
    kw = dict(n_cells=n_cells, lattice=lattice)
    a = mw.frw_extract(h, 0, 30000, seed=4, scores=True, **kw)
    w = mw.frw_autotune(h, 0, 300000, **kw)
    b = mw.frw_extract(h, 0, 30000, seed=4, scores=True, **kw)
    print("tuned waves per CU", w)
    assert 4 <= w <= 16
    assert torch.equal(a["net"], b["net"]) and torch.equal(a["w"], b["w"])
    entries = next(iter(json.load(open(cache)).values()))
    assert any(e["key"] == [-1, n_cells, 0] and e["tune"][1] == w for e in entries)


def test_convergence_target(mw):
    st = W.c2_structure()
    r = mw.frw_extract(st, 0, 50000000, seed=9, target_rel_3sigma=0.02, batch_walks=200000)
    ck = 262144  # 200000 rounded up to whole 65536-walk summation groups
    assert r["stats"]["walks"] < 50000000 and r["stats"]["walks"] % ck == 0
    assert r["stats"]["walks_launched"] >= r["stats"]["walks"]
    assert 3 * r["se"][0] / r["row"][0] <= 0.02


def _rel_at(net, w, n, master):
    """3 SE / |mean| of the master column over the first n walks (binary64)."""
    x = np.where(net[:n] == master, w[:n], 0.0)
    m = x.sum() / n
    var = max((x * x).sum() / n - m * m, 0.0) / (n - 1)
    return 3 * np.sqrt(var) / abs(m)


def test_target_stops_at_first_checkpoint(mw):
    """The stopping rule against the per-walk scores: the row holds the walks
    up to the first checkpoint (every 65536 walks) where 3 SE(C_mm)/|C_mm|
    meets the target, recomputed here in binary64 from the same scores (the
    GPU sums in fp32 per block, so a checkpoint within 1e-5 of the target
    may fall either way)."""
    st = W.c2_structure()
    ck, target = 65536, 0.02
    r = mw.frw_extract(st, 0, 3000000, seed=12, target_rel_3sigma=target, batch_walks=ck, scores=True)
    n = r["stats"]["walks"]
    assert n % ck == 0 and n < 3000000
    net = r["net"].cpu().numpy()
    w = r["w"].cpu().numpy().astype(np.float64)
    assert _rel_at(net, w, n, 0) <= target * (1 + 1e-5)
    for c in range(ck, n, ck):
        assert _rel_at(net, w, c, 0) > target * (1 - 1e-5), c


def test_target_rows_independent_of_launch_split(mw):
    """A target-mode row depends on the walks, not on how they were split
    into launches: a fresh structure handle (first launch of 2^20 walks,
    then a predicted one), the same handle again (one launch sized from the
    first call) and a fixed-budget call over the same number of walks give
    bit-identical rows."""
    st = W.c2_structure()
    h = mw.StructureHandle(st)
    kw = dict(seed=31, target_rel_3sigma=0.006, batch_walks=131072)
    a = mw.frw_extract(h, 0, 20000000, **kw)
    b = mw.frw_extract(h, 0, 20000000, **kw)
    n = a["stats"]["walks"]
    print("walks", n, a["stats"]["walks_launched"], a["stats"]["launches"], b["stats"]["walks_launched"],
          b["stats"]["launches"])
    assert n > (1 << 20) and n == b["stats"]["walks"]
    assert np.array_equal(a["row"], b["row"]) and np.array_equal(a["se"], b["se"])
    c = mw.frw_extract(h, 0, n, seed=31)
    assert np.array_equal(a["row"], c["row"]) and np.array_equal(a["se"], c["se"])
    h.close()


def test_errors(mw):
    st = W.c2_structure()
    with pytest.raises(mw.MWError) as e:
        mw.frw_extract(st, 7, 1000)
    assert e.value.status == mw.MW_EINVAL
    bad = W.c2_structure()
    bad.cond[1] = bad.cond[0] + np.float32(0.01)
    with pytest.raises(mw.MWError) as e:
        mw.StructureHandle(bad)
    assert e.value.status == mw.MW_EGEOM
    with pytest.raises(mw.MWError) as e:
        mw.frw_extract(st, 0, 1000, n_cells=15)
    assert e.value.status == mw.MW_EINVAL


def test_c4_matches_oracle(mw, oracle_lib):
    """Large interconnect window (192 nets, 7 background layers, coatings and
    high-k fills): the GPU row at 2e6 walks against an oracle sample of 30000
    walks (independent seeds), entry by entry in combined standard errors
    for the self term and every coupling the oracle resolves."""
    st = W.c4_structure()
    m = st.meta["master"]
    r_gpu = mw.frw_extract(st, m, 2000000, seed=41)
    r_or = oracle_lib.frw_extract(st, m, 30000, seed=42, threads=_threads())
    print("gpu stats", r_gpu["stats"])
    print("oracle stats", r_or["stats"])
    K = len(r_gpu["row"])
    assert K == st.n_nets + 1
    assert r_gpu["stats"]["walks"] == 2000000
    zs = np.array([_z(r_gpu["row"][j], r_or["row"][j], r_gpu["se"][j], r_or["se"][j])
                   if (r_gpu["se"][j] > 0 or r_or["se"][j] > 0) else 0.0 for j in range(K)])
    resolved = [j for j in range(K) if abs(r_or["row"][j]) > 4 * r_or["se"][j]]
    print("C_mm gpu %.6g +- %.3g, oracle %.6g +- %.3g; resolved couplings %d; max z %.2f"
          % (r_gpu["row"][m], r_gpu["se"][m], r_or["row"][m], r_or["se"][m], len(resolved),
             zs[resolved].max()))
    assert m in resolved and len(resolved) >= 5
    print("halved cubes", r_gpu["stats"]["cube_halved"], "of", r_gpu["stats"]["hops"] + 2000000)
    # the self term alone at 3 combined SE; the resolved entries together at
    # the Bonferroni threshold over their number
    assert zs[m] < 3.0
    assert zs[resolved].max() < z_crit(len(resolved))
    # the resolved entries as a whole: mean z^2 near 1
    assert np.mean(zs[resolved] ** 2) < 2.5
    # nets the GPU never reached are ones the oracle sample barely reached
    for j in range(K):
        if r_gpu["row"][j] == 0.0:
            assert abs(r_or["row"][j]) < z_crit(K) * r_or["se"][j] + 1e-30



def test_c4_headline_sampled_walks_match_oracle(mw, oracle_lib):
    """The headline configuration as the bench times it (the large window
    walked to 3 SE / |C_mm| <= 1 %, one launch of several checkpoints
    replayed from a HIP graph after warm-up calls): five runs of 200 walks
    spread over the kept walks, recomputed by the oracle from their walk
    indices, equal the GPU's walks one by one; the stopping checkpoint
    meets the target."""
    st = W.c4_structure()
    m = st.meta["master"]
    h = mw.StructureHandle(st)
    for k in range(2):
        mw.frw_extract(h, m, 100000000, seed=60 + k, target_rel_3sigma=0.01)
    g = mw.frw_extract(h, m, 100000000, seed=7, target_rel_3sigma=0.01, scores=True)
    n = int(g["stats"]["walks"])
    assert n % 65536 == 0 and 3 * g["se"][m] / g["row"][m] <= 0.01
    agree = []
    for f in np.linspace(0, n - 200, 5).astype(np.int64):
        o = oracle_lib.frw_extract(st, m, 200, seed=7, first_walk=int(f), threads=_threads(), scores=True,
                                   kernel_limits=True)
        part = {"net": g["net"][f:f + 200], "w": g["w"][f:f + 200]}
        agree.append(_walk_agreement(part, o["net"], o["w"])[1])
    print("walks", n, "per-run agreement", agree)
    assert min(agree) >= 0.98 and np.mean(agree) >= 0.99
    h.close()


def test_matrix_rows_equal_single_extractions(mw):
    """frw_extract_matrix: every row equals frw_extract of that master with
    key seed + i (same walks, fp32 summation order aside); the matrix obeys
    reciprocity within standard errors and the symmetrised block is the
    mean of the two estimates."""
    st = W.c2_structure()
    h = mw.StructureHandle(st)
    walks = 300000
    M = mw.frw_extract_matrix(h, walks, seed=40)
    assert M["stats"]["walks"] == 4 * walks
    cap, se, sym = M["cap"], M["se"], M["sym"]
    for i, m in enumerate(M["masters"]):
        alone = mw.frw_extract(h, m, walks, seed=40 + i)
        scale = np.abs(alone["row"]).max()
        assert np.all(np.abs(cap[i] - alone["row"]) <= 1e-6 * np.abs(alone["row"]) + 1e-9 * scale)
        assert np.allclose(se[i], alone["se"], rtol=1e-4, atol=1e-12)
    for a in range(4):
        assert sym[a, a] == cap[a, a]
        for b in range(4):
            if a != b:
                assert _z(cap[a, b], cap[b, a], se[a, b], se[b, a]) < z_crit(6)
                assert sym[a, b] == pytest.approx(0.5 * (cap[a, b] + cap[b, a]))
    # a subset of masters, converging on its own target
    M2 = mw.frw_extract_matrix(h, 20000000, seed=5, masters=[2, 0], target_rel_3sigma=0.03,
                               batch_walks=100000)
    assert M2["masters"] == [2, 0] and M2["sym"].shape == (2, 2)
    for i, m in enumerate(M2["masters"]):
        assert 3 * M2["se"][i, m] / M2["cap"][i, m] <= 0.03
    assert M2["stats"]["walks"] < 2 * 20000000
    with pytest.raises(mw.MWError) as e:
        mw.frw_extract_matrix(h, 1000, masters=[1, 1])
    assert e.value.status == mw.MW_EINVAL


def test_matrix_rows_match_oracle(mw, oracle_lib):
    """frw_extract_matrix on the crossing wires against the oracle: each GPU
    row against the oracle's row of the same master, and reciprocity across
    the two implementations (GPU C_ab against the oracle's C_ba), all
    entries together at the Bonferroni threshold."""
    st = W.c2_structure()
    M = mw.frw_extract_matrix(st, 1000000, seed=70)
    rows = {m: oracle_lib.frw_extract(st, m, 60000, seed=170 + m, threads=_threads()) for m in range(4)}
    zs, zr = [], []
    for i, m in enumerate(M["masters"]):
        o = rows[m]
        zs += [_z(M["cap"][i, j], o["row"][j], M["se"][i, j], o["se"][j]) for j in range(5)]
        for j in range(4):
            if j != m:
                zr.append(_z(M["cap"][i, j], rows[j]["row"][m], M["se"][i, j], rows[j]["se"][m]))
    zs, zr = np.array(zs), np.array(zr)
    print("rows: max z %.2f; reciprocity across implementations: max z %.2f" % (zs.max(), zr.max()))
    assert zs.max() < z_crit(zs.size)
    assert zr.max() < z_crit(zr.size)


# ---------------------------------------------------------------------------
# MicroWalk-E (expanded transition cubes holding conductors)
# ---------------------------------------------------------------------------
@pytest.mark.parametrize("variant", ["uniform", "columns"])
def test_microwalk_e_plates(mw, variant):
    st = W.parallel_plates(variant)
    exact = W.parallel_plates_exact(variant)
    r = mw.frw_extract(st, 0, 1000000, seed=12, hybrid=0, expand=5)
    print(variant, r["row"][0] / exact - 1, r["se"][0] / exact, r["stats"])
    assert r["stats"]["micro_steps"] > 0
    assert abs(r["row"][0] - exact) < 0.01 * exact + 3 * r["se"][0]


def test_microwalk_e_c2_matches_oracle(mw, oracle_lib):
    """GPU and oracle MicroWalk-E share the expanded-cube readings: the C2 rows
    agree in combined standard errors (the GPU cuts links with 16-bit
    fractions and fp32 geometry, so agreement is statistical)."""
    st = W.c2_structure()
    g = mw.frw_extract(st, 0, 2000000, seed=21, expand=5)
    o = oracle_lib.frw_extract(st, 0, 150000, seed=22, threads=_threads(), expand=5.0)
    p = mw.frw_extract(st, 0, 1000000, seed=23)
    print("gpu E", g["row"], g["se"], g["stats"])
    print("oracle E", o["row"], o["se"], o["stats"])
    print("gpu plain", p["row"], p["stats"])
    zs = [_z(g["row"][j], o["row"][j], g["se"][j], o["se"][j]) for j in range(5)]
    print("z", zs)
    assert max(zs) < z_crit(5)
    per = lambda r, k: r["stats"][k] / r["stats"]["walks"]
    assert per(g, "hops") * 2 < per(p, "hops")
    assert per(g, "micro_steps") * 4 < per(p, "micro_steps")


def test_microwalk_e_high_permittivity_beside_conductors(mw, oracle_lib):
    """MicroWalk-E with eps = 1e3 (the largest accepted) filling half of a
    parallel-plate gap: links cut near the plates carry up to 16 times a
    link code of 2.6e8, so the direction sums pass 2^32.  Walks equal the
    oracle's one by one, and the row meets the closed form."""
    st = W.parallel_plates("columns_highk")
    g = mw.frw_extract(st, 0, 20000, seed=77, scores=True, hybrid=0, expand=5)
    o = oracle_lib.frw_extract(st, 0, 20000, seed=77, threads=_threads(), scores=True, hybrid=0, expand=5.0,
                               kernel_limits=True)
    same_net, same_walk = _walk_agreement(g, o["net"], o["w"])
    print("highk MicroWalk-E same net", same_net, "same net and weight", same_walk)
    assert same_walk >= 0.99
    exact = W.parallel_plates_exact("columns_highk")
    r = mw.frw_extract(st, 0, 1000000, seed=13, hybrid=0, expand=5)
    print("highk", r["row"][0] / exact - 1, r["se"][0] / exact, r["stats"]["micro_steps"])
    assert abs(r["row"][0] - exact) < 0.01 * exact + 3 * r["se"][0]


# ---------------------------------------------------------------------------
# Importance sampling of the Gaussian-surface point
# ---------------------------------------------------------------------------
@pytest.mark.parametrize("name", ["highk", "c2"])
def test_gauss_importance_walks_match_oracle(mw, oracle_lib, name):
    """Both sides cut G into the same patches and weight them by the first-
    transition kernel at the patch centres (fp32 on the GPU, fp64 in the
    oracle), so walks agree one by one except where a draw falls within
    rounding of a patch boundary."""
    st = W.parallel_plates("columns_highk") if name == "highk" else W.c2_structure()
    g = mw.frw_extract(st, 0, 20000, seed=78, scores=True, gauss_is=1.0)
    o = oracle_lib.frw_extract(st, 0, 20000, seed=78, threads=_threads(), scores=True, gauss_is=1.0,
                               kernel_limits=True)
    same_net, same_walk = _walk_agreement(g, o["net"], o["w"])
    print(name, "importance sampling: same net", same_net, "same net and weight", same_walk)
    assert same_walk >= 0.995


def test_gauss_importance_closed_form_and_variance(mw):
    st = W.parallel_plates("columns_highk")
    exact = W.parallel_plates_exact("columns_highk")
    u = mw.frw_extract(st, 0, 1000000, seed=30)
    s = mw.frw_extract(st, 0, 1000000, seed=31, gauss_is=1.0)
    print("uniform %.5f +- %.5f; importance %.5f +- %.5f; exact %.5f"
          % (u["row"][0], u["se"][0], s["row"][0], s["se"][0], exact))
    assert abs(s["row"][0] - exact) < 3 * s["se"][0]
    assert abs(s["row"][1] + exact) < 3 * s["se"][1]
    assert s["se"][0] < 0.85 * u["se"][0]


def test_gauss_importance_keeps_c2_rows(mw, c2_gpu):
    s = mw.frw_extract(W.c2_structure(), 0, 1000000, seed=33, gauss_is=1.0)
    u = c2_gpu[0]
    zs = np.abs(s["row"] - u["row"]) / np.hypot(s["se"], u["se"])
    print("importance", s["row"], s["se"], "z", zs)
    assert zs.max() < z_crit(5)
    with pytest.raises(mw.MWError) as e:
        mw.frw_extract(W.c2_structure(), 0, 1000, gauss_is=0.01)
    assert e.value.status == mw.MW_EINVAL


def test_microwalk_e_options(mw):
    st = W.c2_structure()
    with pytest.raises(mw.MWError) as e:
        mw.frw_extract(st, 0, 1000, expand=8)  # 8x the conductor-free size at n = 16
    assert e.value.status == mw.MW_EINVAL
    import torch
    a = mw.frw_extract(st, 0, 20000, seed=3, scores=True)
    b = mw.frw_extract(st, 0, 20000, seed=3, scores=True, expand=1)
    assert torch.equal(a["net"], b["net"]) and torch.equal(a["w"], b["w"])


@pytest.mark.parametrize("walks,n_cells,lattice", [(2, 16, 0), (63, 16, 0), (4097, 16, 0), (65537, 16, 0),
                                                   (3001, 4, 0), (1500, 32, 0), (3001, 3, 1), (65537, 15, 1)])
def test_ragged_budgets_and_extreme_cube_sizes(mw, oracle_lib, walks, n_cells, lattice):
    """The smallest budget (2 walks), counts that end inside a wave, a
    4096-walk reduction block and a 65536-walk summation group, and the
    smallest and largest cubes of both lattices: walks equal the oracle's one
    by one and the row is the mean of the scores."""
    st = W.c2_structure()
    g = mw.frw_extract(st, 0, walks, seed=61, scores=True, n_cells=n_cells, lattice=lattice)
    o = oracle_lib.frw_extract(st, 0, walks, seed=61, threads=_threads(), scores=True, n_cells=n_cells,
                               lattice=lattice, kernel_limits=True)
    assert g["stats"]["walks"] == walks and len(g["net"]) == walks
    same_net, same_walk = _walk_agreement(g, o["net"], o["w"])
    print(walks, n_cells, lattice, "same net", same_net, "same net and weight", same_walk)
    assert same_walk >= (0.995 if walks > 1000 else 1.0 - 1.0 / walks)
    K = len(g["row"])
    w = g["w"].double().cpu().numpy()
    s = np.bincount(g["net"].cpu().numpy(), weights=w, minlength=K) / walks
    assert np.allclose(s, g["row"], rtol=1e-5, atol=1e-7 * np.abs(g["row"]).max())
    with pytest.raises(mw.MWError) as e:
        mw.frw_extract(st, 0, 1, n_cells=n_cells, lattice=lattice)
    assert e.value.status == mw.MW_EINVAL


def test_concurrent_extractions_equal_sequential(mw):
    """frw_extract from several host threads on one structure (the binding
    releases the GIL during the call): masters, lattice sizes, both lattices,
    a target and the plain form at once, twice over; every call returns the
    walks and row of the same call made alone, bit for bit."""
    import threading
    import torch
    st = W.c2_structure()
    h = mw.StructureHandle(st)
    jobs = [dict(master=0, seed=71), dict(master=1, seed=72), dict(master=0, seed=73, n_cells=12),
            dict(master=2, seed=74, target_rel_3sigma=0.05), dict(master=0, seed=75, n_cells=15, lattice=1),
            dict(master=3, seed=76, plain=1)]

    def run(j):
        j = dict(j)
        m = j.pop("master")
        return mw.frw_extract(h, m, 40000, scores=True, **j)

    alone = [run(j) for j in jobs]
    for rep in range(2):
        out, errs = [None] * len(jobs), []

        def worker(i):
            try:
                out[i] = run(jobs[i])
            except Exception as e:  # reported below
                errs.append(repr(e))

        th = [threading.Thread(target=worker, args=(i,)) for i in range(len(jobs))]
        for t in th:
            t.start()
        for t in th:
            t.join(timeout=120)
        assert not errs, errs
        assert all(t.is_alive() is False for t in th)
        for a, b in zip(alone, out):
            n = int(a["stats"]["walks"])
            assert int(b["stats"]["walks"]) == n
            assert torch.equal(a["net"][:n], b["net"][:n]) and torch.equal(a["w"][:n], b["w"][:n])
            assert np.array_equal(a["row"], b["row"]) and np.array_equal(a["se"], b["se"])
    h.close()
