"""GPU FRW on the cell-centred lattice of Sec. III-A (frw_options.lattice =
MW_LATTICE_CELL) through the C ABI, against the CPU oracle.

* Tables: hop and first-transition tables of stratified cubes built on the
  device (DST-II sine basis in the plane, transposed tridiagonal solves of the
  non-symmetric Eq. (6) chain) against the oracle's BiCGSTAB solve, every CDF
  entry within one 32-bit step.
* Walks: GPU and oracle draw every random word from the same Philox streams,
  so walks are compared one by one (plates, C2 with and without the hybrid
  strategy, three cube sizes).
* Rows: closed forms on plates; C2 rows against the oracle's in combined
  standard errors (Bonferroni over the entries compared together).
* The shared-round kernels (capacitance matrix, serving) on the cell lattice
  give the single extraction's walks and rows; the plain form and split runs
  give its walks bit for bit; importance sampling over G (patch weights from
  the cell-lattice first kernel) matches the oracle walk by walk.
"""
import os

import numpy as np
import pytest

import workloads as W
from _stats import z, z_crit

pytestmark = pytest.mark.gpu

W_REL = 1e-5  # fp32 weight against the oracle's binary64 one


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


def _expected_cdf(wts):
    wts = np.abs(np.asarray(wts, dtype=np.float64))
    cum = np.cumsum(wts) / wts.sum()
    return np.minimum(np.ceil(cum * 4294967296.0), 4294967295.0)


def _profiles(n):
    rng = np.random.Generator(np.random.PCG64(2000 + n))
    half = n // 2
    return {
        "uniform": [3.9] * n,
        "two_layers": [3.9] * half + [2.7] * (n - half),
        "film": [3.9] * (n // 4) + [25.0] * (n // 4) + [2.7] * (n - 2 * (n // 4)),
        "random": list(rng.choice([2.5, 3.9, 7.0, 25.0], size=n)),
    }


@pytest.mark.parametrize("n", [7, 15, 31])
@pytest.mark.parametrize("axis", [0, 2])
def test_cell_hop_tables_match_oracle(mw, oracle_lib, n, axis):
    for name, planes in _profiles(n).items():
        g = mw.mw_sgf_table(planes, axis, kind=0, lattice=mw.MW_LATTICE_CELL)
        P = oracle_lib.hop_table(planes, axis, lattice=1)
        assert g["cdf"].size == 6 * n * n
        diff = np.abs(g["cdf"].astype(np.float64) - _expected_cdf(P))
        print(n, axis, name, "max CDF step difference", diff.max())
        assert diff.max() <= 1.0, (name, int(np.argmax(diff)))
        assert g["cdf"][-1] == 0xffffffff


@pytest.mark.parametrize("n", [7, 15])
@pytest.mark.parametrize("axis,normal", [(2, 2), (2, 0), (0, 1), (1, 1)])
def test_cell_first_tables_match_oracle(mw, oracle_lib, n, axis, normal):
    for name, planes in _profiles(n).items():
        g = mw.mw_sgf_table(planes, axis, kind=1, normal_axis=normal, lattice=mw.MW_LATTICE_CELL)
        Pc, Pp, Pm, Gp, Gm = oracle_lib.first_table(planes, axis, normal, lattice=1)
        w = 0.5 * (Gp * (Pc - Pp) + Gm * (Pm - Pc))
        K = np.abs(w).sum()
        diff = np.abs(g["cdf"].astype(np.float64) - _expected_cdf(w))
        print(n, axis, normal, name, "max CDF step difference", diff.max(), "K h", g["kh"], K)
        assert diff.max() <= 1.0, (name, int(np.argmax(diff)))
        big = np.abs(w) > 1e-9 * K
        assert np.array_equal(g["sign"][big], (w > 0)[big])
        assert abs(g["kh"] - K) <= 1e-6 * K
        assert abs(w.sum()) < 1e-9 * K


def _agreement(g, o):
    g_net = g["net"].cpu().numpy()
    g_w = g["w"].cpu().numpy().astype(np.float64)
    same = g_net == o["net"]
    rel = np.abs(g_w - o["w"]) / np.maximum(np.abs(o["w"]), 1e-30)
    return float(same.mean()), float((same & (rel <= W_REL)).mean())


@pytest.mark.parametrize("name,hybrid,n_cells,floor", [
    ("plates", 1, 15, 0.999), ("checker", 1, 15, 0.999), ("stack", 1, 15, 0.999), ("c2", 1, 15, 0.999),
    ("c2", 0, 15, 0.999), ("c2", 1, 7, 0.999), ("c2", 1, 31, 0.999), ("c4", 1, 15, 0.99)])
def test_cell_walks_match_oracle_one_by_one(mw, oracle_lib, name, hybrid, n_cells, floor):
    """The twelve-layer stack reads its background layers from global memory
    (more layers than the LDS copy holds).  Its layer faces are shifted by
    12.3 nm here: in the plain stack the Gaussian surface and some cell
    centres of every first cube lie exactly on layer faces, where the fp32
    and binary64 half-open tests may choose different layers (either cube is
    valid; walk-by-walk comparisons need points off the faces).  The large
    interconnect window has cubes that the kernel's capacity rule halves,
    which the oracle follows here (kernel_limits)."""
    def stack():
        st = W.parallel_plates("stack")
        st.layer_z0[1:] += np.float32(0.0123)
        return st

    st = {"plates": lambda: W.parallel_plates("columns"), "checker": lambda: W.parallel_plates("checkerboard"),
          "stack": stack, "c2": W.c2_structure, "c4": W.c4_structure}[name]()
    m = st.meta["master"] if name == "c4" else 0
    N = 3000 if name == "c4" else (20000 if n_cells <= 15 else 4000)
    g = mw.frw_extract(st, m, N, seed=31, scores=True, hybrid=hybrid, n_cells=n_cells,
                       lattice=mw.MW_LATTICE_CELL)
    o = oracle_lib.frw_extract(st, m, N, seed=31, threads=_threads(), scores=True, hybrid=hybrid,
                               n_cells=n_cells, lattice=1, kernel_limits=True)
    same_net, same_walk = _agreement(g, o)
    print(name, hybrid, n_cells, "same net", same_net, "same net and weight", same_walk, g["stats"])
    if name != "c4":
        assert g["stats"]["cube_halved"] == 0
    if hybrid == 0:
        assert g["stats"]["micro_steps"] > 0
    assert same_walk >= floor


@pytest.mark.parametrize("variant", ["uniform", "columns", "checkerboard"])
def test_cell_plates_closed_forms(mw, variant):
    st = W.parallel_plates(variant)
    r = mw.frw_extract(st, 0, 400000, seed=5, n_cells=15, lattice=mw.MW_LATTICE_CELL)
    exact = W.parallel_plates_exact(variant)
    zc = z_crit(2)
    print(variant, r["row"], r["se"], (r["row"][0] - exact) / r["se"][0])
    assert abs(r["row"][0] - exact) < zc * r["se"][0]
    assert abs(r["row"][1] + exact) < zc * r["se"][1]


@pytest.fixture(scope="module")
def c2_cell_gpu(mw):
    st = W.c2_structure()
    return mw.frw_extract(st, 0, 1000000, seed=40, scores=True, n_cells=15, lattice=mw.MW_LATTICE_CELL)


def test_cell_c2_row_matches_oracle(mw, oracle_lib, c2_cell_gpu):
    st = W.c2_structure()
    o = oracle_lib.frw_extract(st, 0, 100000, seed=41, threads=_threads(), n_cells=15, lattice=1)
    g = c2_cell_gpu
    zs = z(g["row"], o["row"], g["se"], o["se"])
    print("gpu", g["row"], g["se"], g["stats"], "oracle", o["row"], o["se"], "z", zs)
    assert (zs < z_crit(len(zs))).all(), zs
    # row sums and signs of a Maxwell row
    assert g["row"][0] > 0 and all(g["row"][j] <= 3 * g["se"][j] for j in range(1, len(g["row"])))
    w = g["w"].double().cpu().numpy()
    assert abs(g["row"].sum() - w.mean()) < 1e-9 * np.abs(g["row"]).sum()


def test_cell_c2_sampled_walks_of_large_run_match_oracle(oracle_lib, c2_cell_gpu):
    st = W.c2_structure()
    g = c2_cell_gpu
    agree = []
    for f in np.linspace(0, len(g["net"]) - 200, 5).astype(np.int64):
        o = oracle_lib.frw_extract(st, 0, 200, seed=40, first_walk=int(f), threads=_threads(), scores=True,
                                   n_cells=15, lattice=1, kernel_limits=True)
        part = {"net": g["net"][f:f + 200], "w": g["w"][f:f + 200]}
        agree.append(_agreement(part, o)[1])
    print("per-run agreement", agree)
    assert min(agree) >= 0.99


def test_cell_matrix_and_server_equal_single_extraction(mw):
    """Shared-round walker and reductions on the cell lattice: a matrix row
    and a served request reproduce the single extraction's row."""
    st = W.c2_structure()
    h = mw.StructureHandle(st)
    one = [mw.frw_extract(h, m, 60000, seed=50 + m, n_cells=15, lattice=mw.MW_LATTICE_CELL) for m in (0, 1)]
    mat = mw.frw_extract_matrix(h, 60000, seed=50, masters=[0, 1], n_cells=15, lattice=mw.MW_LATTICE_CELL)
    for i in (0, 1):
        assert np.allclose(mat["cap"][i], one[i]["row"], rtol=1e-5, atol=1e-9)
    srv = mw.Server(2 << 30, n_cells=15, lattice=mw.MW_LATTICE_CELL)
    try:
        t = srv.submit(st, 0, 60000, seed=50)
        r = srv.wait(t)
    finally:
        srv.close()
    assert np.allclose(r["row"], one[0]["row"], rtol=1e-5, atol=1e-9)


def test_cell_lattice_options_are_checked(mw):
    st = W.parallel_plates("uniform")
    for kw in ({"n_cells": 16, "lattice": mw.MW_LATTICE_CELL}, {"n_cells": 15},
               {"n_cells": 15, "lattice": mw.MW_LATTICE_CELL, "expand": 5}, {"n_cells": 15, "lattice": 2}):
        with pytest.raises(mw.MWError) as e:
            mw.frw_extract(st, 0, 1000, **kw)
        assert e.value.status == mw.MW_EINVAL


@pytest.mark.parametrize("name", ["highk", "c2"])
def test_cell_gauss_importance_walks_match_oracle(mw, oracle_lib, name):
    """Importance sampling over G on the cell lattice: the patch weights come
    from the first-transition kernel evaluated by the cell-lattice first
    kernel (fp32) and by the oracle (fp64); walks agree one by one except
    where a draw falls within rounding of a patch boundary.  The first cube's
    centre cell is centred on the evaluated point, so a patch centre lying
    exactly on a dielectric face would put a cell centre on that face, where
    the fp32 and fp64 half-open tests may differ (either cube is valid); the
    patch edge 0.7 g keeps the centres off the faces of both structures (with
    1.0 g the middle patch of the high-k plates sits on the column's face)."""
    st = W.parallel_plates("columns_highk") if name == "highk" else W.c2_structure()
    g = mw.frw_extract(st, 0, 20000, seed=78, scores=True, gauss_is=0.7, n_cells=15, lattice=mw.MW_LATTICE_CELL)
    o = oracle_lib.frw_extract(st, 0, 20000, seed=78, threads=_threads(), scores=True, gauss_is=0.7,
                               n_cells=15, lattice=1, kernel_limits=True)
    same_net, same_walk = _agreement(g, o)
    print(name, "cell lattice, importance sampling: same net", same_net, "same net and weight", same_walk)
    assert same_walk >= 0.995


def test_cell_plain_form_and_resume_are_bit_identical(mw):
    """The plain form (one walker launch per transition round) and a run
    split at walk 12345 give the persistent run's walks bit for bit."""
    import torch
    st = W.c2_structure()
    h = mw.StructureHandle(st)
    kw = dict(n_cells=15, lattice=mw.MW_LATTICE_CELL, scores=True)
    a = mw.frw_extract(h, 0, 30000, seed=12, **kw)
    p = mw.frw_extract(h, 0, 30000, seed=12, plain=1, **kw)
    b1 = mw.frw_extract(h, 0, 12345, seed=12, **kw)
    b2 = mw.frw_extract(h, 0, 30000 - 12345, seed=12, first_walk=12345, **kw)
    assert p["stats"]["launches"] > a["stats"]["launches"]
    assert torch.equal(a["net"], p["net"]) and torch.equal(a["w"], p["w"])
    assert torch.equal(a["net"], torch.cat([b1["net"], b2["net"]]))
    assert torch.equal(a["w"], torch.cat([b1["w"], b2["w"]]))
    h.close()
