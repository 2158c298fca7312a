"""Oracle pins for FRW on the cell-centred lattice of Sec. III-A.

Every transition cube is N^3 voxels (N odd) with nodes at the voxel
centres: walks start in the centre cell, step with the Eq. (6) coefficients
and leave through the centre of a boundary panel.  Pins:

* the oracle's BiCGSTAB exit distributions (hop tables, the three rows of a
  first-transition table, off-centre sources) against a scipy sparse-LU solve
  of the same absorbing chain (Theorem 1);
* the first-transition face conductances against the series formula;
* parallel plates with uniform, column and checkerboard dielectrics, whose
  linear potential the cell lattice solves exactly: closed forms;
* Theorem 1 at the FRW level: hybrid (tables on stratified cubes) and
  all-MicroWalk runs estimate the same C2 row;
* the cell and vertex discretisations estimate the same C2 row.
"""
import numpy as np
import pytest

import workloads as W
from _stats import z, z_crit


def _layered(planes, axis, N):
    e = np.empty((N, N, N), dtype=np.float32)  # [k, j, i]
    for p in range(N):
        idx = [slice(None)] * 3
        idx[2 - axis] = p
        e[tuple(idx)] = planes[p]
    return e


@pytest.mark.parametrize("N", [3, 5, 7])
def test_sgf_cell_matches_sparse_lu(oracle_lib, N):
    from oracle import pins
    rng = np.random.default_rng(N)
    eps = (10 ** rng.uniform(-1, 2, (N, N, N))).astype(np.float32)
    links, _ = oracle_lib.cell_thresholds(eps)
    c = (N - 1) // 2
    for src in [(c, c, c), (c + 1, c, c), (0, N - 1, 1)]:
        P, et = oracle_lib.sgf_cell(eps, src)
        Q, et2 = pins.cell_exit_distribution(links, N, src)
        assert np.abs(P - Q).max() < 1e-13
        assert abs(et - et2) < 1e-10 * et2
        assert abs(P.sum() - 1.0) < 1e-12


@pytest.mark.parametrize("axis", [0, 1, 2])
def test_cell_hop_table_is_exit_distribution_of_layered_cube(oracle_lib, axis):
    from oracle import pins
    N = 7
    planes = np.array([3.9, 3.9, 7.0, 2.7, 2.7, 25.0, 3.9], dtype=np.float32)
    P = oracle_lib.hop_table(planes, axis, lattice=1)
    e = _layered(planes, axis, N)
    links, _ = oracle_lib.cell_thresholds(e)
    Q, _ = pins.cell_exit_distribution(links, N)
    assert P.shape == (6 * N * N,)
    assert np.abs(P - Q).max() < 1e-13


@pytest.mark.parametrize("axis,normal", [(2, 2), (2, 0), (0, 1)])
def test_cell_first_table(oracle_lib, axis, normal):
    from oracle import pins
    N = 7
    planes = np.array([2.7, 3.9, 3.9, 7.0, 3.9, 2.2, 2.2], dtype=np.float32)
    Pc, Pp, Pm, gp, gm = oracle_lib.first_table(planes, axis, normal, lattice=1)
    e = _layered(planes, axis, N)
    links, _ = oracle_lib.cell_thresholds(e)
    c = (N - 1) // 2
    for P, d in ((Pc, 0), (Pp, 1), (Pm, -1)):
        src = [c, c, c]
        src[normal] += d
        Q, _ = pins.cell_exit_distribution(links, N, tuple(src))
        assert np.abs(P - Q).max() < 1e-13
    # face conductances of the centre cell along the normal: the series
    # combination of the two half cells (equal permittivities: that value)
    ec = float(planes[c])
    ep = float(planes[c + 1]) if axis == normal else ec
    em = float(planes[c - 1]) if axis == normal else ec
    assert gp == pytest.approx(2 * ec * ep / (ec + ep), rel=1e-15)
    assert gm == pytest.approx(2 * ec * em / (ec + em), rel=1e-15)


@pytest.mark.parametrize("variant,hybrid", [("uniform", 1), ("uniform", 0), ("columns", 1), ("columns", 0),
                                            ("checkerboard", 1)])
def test_cell_lattice_parallel_plates_closed_form(oracle_lib, variant, hybrid):
    """Two entries (C_00, C_01) against the closed form at once."""
    st = W.parallel_plates(variant)
    exact = W.parallel_plates_exact(variant)
    r = oracle_lib.frw_extract(st, 0, 40000, seed=3, threads=8, hybrid=hybrid, n_cells=15, lattice=1)
    zc = z_crit(2)
    assert abs(r["row"][0] - exact) < zc * r["se"][0], (r["row"], r["se"], exact)
    assert abs(r["row"][1] + exact) < zc * r["se"][1]
    assert r["row"][2] == 0.0
    if hybrid == 0:
        assert r["stats"]["micro_steps"] > 0


def test_cell_lattice_needs_odd_cubes(oracle_lib):
    st = W.parallel_plates("uniform")
    with pytest.raises(RuntimeError):
        oracle_lib.frw_extract(st, 0, 100, n_cells=16, lattice=1)
    with pytest.raises(RuntimeError):
        oracle_lib.frw_extract(st, 0, 100, n_cells=15, lattice=1, expand=5.0)


@pytest.fixture(scope="module")
def c2_cell(oracle_lib):
    st = W.c2_structure()
    return oracle_lib.frw_extract(st, 0, 60000, seed=21, threads=8, hybrid=1, n_cells=15, lattice=1, scores=True)


def test_cell_lattice_c2_hybrid_equals_all_microwalk(oracle_lib, c2_cell):
    """Theorem 1 at the FRW level on the cell lattice (five entries)."""
    st = W.c2_structure()
    mw = oracle_lib.frw_extract(st, 0, 60000, seed=22, threads=8, hybrid=0, n_cells=15, lattice=1)
    assert c2_cell["stats"]["cls_stratified"] + c2_cell["stats"]["cls_uniform"] > 0
    assert c2_cell["stats"]["cache_miss"] > 0 and mw["stats"]["micro_steps"] > c2_cell["stats"]["micro_steps"]
    zs = z(c2_cell["row"], mw["row"], c2_cell["se"], mw["se"])
    assert (zs < z_crit(len(zs))).all(), zs


def test_cell_and_vertex_lattices_agree_on_c2(oracle_lib, c2_cell):
    st = W.c2_structure()
    v = oracle_lib.frw_extract(st, 0, 60000, seed=23, threads=8, hybrid=1, n_cells=16)
    zs = z(c2_cell["row"], v["row"], c2_cell["se"], v["se"])
    assert (zs < z_crit(len(zs))).all(), zs
    # Maxwell signs and the score identity hold on the cell lattice too
    row, se = c2_cell["row"], c2_cell["se"]
    assert row[0] > 0 and all(row[j] <= 3 * se[j] for j in range(1, len(row)))
    s = np.bincount(c2_cell["net"], weights=c2_cell["w"], minlength=len(row)) / c2_cell["w"].size
    assert np.allclose(s, row, rtol=1e-12, atol=1e-15)


def test_cell_lattice_series_plates_soft(oracle_lib):
    """Series stack on the cell lattice: interfaces between cell centres are
    resolved exactly by the series (Eq. 6) link, but the voxelisation snaps
    the interface to cell faces, a bias that shrinks with the lattice step
    (reported as z-scores; the vertex-lattice counterpart is in
    test_oracle_frw.py)."""
    st = W.parallel_plates("series")
    exact = W.parallel_plates_exact("series")
    r = oracle_lib.frw_extract(st, 0, 40000, seed=4, threads=8, n_cells=15, lattice=1)
    zs = (r["row"][0] - exact) / r["se"][0]
    assert abs(zs) < 4.0, zs
