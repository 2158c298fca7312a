"""GPU FRW extraction with nets made of several boxes (Alg. 1 with a master
net whose conductor is a union of boxes), through the C ABI.

The library builds the master's Gaussian surface itself; its growth g and
area must equal the oracle's (which the voxel-boundary pins fix).  The
capacitances are Monte Carlo estimates compared in combined standard errors
with a closed form and with the oracle; cutting a non-master conductor into
abutting boxes must leave every walk, and so the row, bit-identical.
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


@pytest.mark.parametrize("name", ["sandwich", "sandwich-split", "c2-multibox", "random-3", "random-4"])
def test_gauss_surface_matches_oracle(mw, oracle_lib, name):
    st = {"sandwich": lambda: W.sandwich_plates(False),
          "sandwich-split": lambda: W.sandwich_plates(True),
          "c2-multibox": lambda: W.c2_multibox_structure(False),
          "random-3": lambda: W.random_multibox_net(3),
          "random-4": lambda: W.random_multibox_net(4)}[name]()
    g, area, faces = oracle_lib.gauss(st, 0)
    r = mw.frw_extract(st, 0, 20000, seed=3)
    s = r["stats"]
    print(name, "g", s["gauss_g"], g, "area", s["gauss_area"], area, "rects", s["gauss_faces"], len(faces))
    assert s["gauss_g"] == pytest.approx(g, rel=1e-6)
    assert s["gauss_area"] == pytest.approx(area, rel=1e-6)
    assert 1 <= s["gauss_faces"] <= len(faces)


@pytest.mark.parametrize("split,hybrid", [(False, 1), (True, 1), (True, 0)])
def test_sandwich_plates_closed_form(mw, split, hybrid):
    st = W.sandwich_plates(split)
    exact = W.sandwich_plates_exact()
    r = mw.frw_extract(st, 0, 1000000, seed=5, hybrid=hybrid)
    print("sandwich", split, hybrid, r["row"], r["se"], (r["row"][0] - exact) / r["se"][0])
    assert abs(r["row"][0] - exact) < 3 * r["se"][0] + 2e-4 * exact
    assert abs(r["row"][1] + exact) < 3 * r["se"][1] + 2e-4 * exact
    assert r["row"][2] == 0.0


def test_c2_multibox_matches_oracle(mw, oracle_lib):
    st = W.c2_multibox_structure(False)
    r_gpu = mw.frw_extract(st, 0, 2000000, seed=31)
    r_or = oracle_lib.frw_extract(st, 0, 30000, seed=32, threads=_threads())
    K = len(r_gpu["row"])
    assert K == st.n_nets + 1
    zs = np.array([_z(r_gpu["row"][j], r_or["row"][j], r_gpu["se"][j], r_or["se"][j])
                   if (r_gpu["se"][j] > 0 or r_or["se"][j] > 0) else 0.0 for j in range(K)])
    print("gpu", r_gpu["row"], r_gpu["se"])
    print("oracle", r_or["row"], r_or["se"])
    print("z", zs)
    assert zs.max() < z_crit(K)
    # Maxwell signs: positive self term, negative couplings
    assert r_gpu["row"][0] > 0 and (r_gpu["row"][1:] <= 0).all()


def test_split_non_master_net_is_bit_identical(mw):
    a = mw.frw_extract(W.c2_multibox_structure(False), 0, 500000, seed=9)
    b = mw.frw_extract(W.c2_multibox_structure(True), 0, 500000, seed=9)
    assert list(a["row"]) == list(b["row"])
    assert list(a["se"]) == list(b["se"])
    assert a["stats"]["micro_steps"] == b["stats"]["micro_steps"]


def test_multibox_microwalk_e_runs(mw):
    """MicroWalk-E with a multi-box master: conductor boxes inside expanded
    cubes absorb as their net; the row keeps Maxwell's signs and sums to
    about zero with the grounded window."""
    st = W.c2_multibox_structure(False)
    r = mw.frw_extract(st, 0, 500000, seed=12, expand=5)
    row, se = np.array(r["row"]), np.array(r["se"])
    print("mw-e multibox", row, se, r["stats"]["hops"] / r["stats"]["walks"])
    assert row[0] > 0 and (row[1:] <= 0).all()
    assert abs(row.sum()) < 4 * np.sqrt((se ** 2).sum()) + 0.02 * row[0]


def test_c2_multibox_cell_lattice_matches_oracle(mw, oracle_lib):
    """A multi-box master on the cell-centred lattice (15-cell cubes):
    Gaussian surface of the union, first transitions and walks on that
    lattice, rows against the oracle's."""
    st = W.c2_multibox_structure(False)
    r_gpu = mw.frw_extract(st, 0, 1000000, seed=33, n_cells=15, lattice=mw.MW_LATTICE_CELL)
    r_or = oracle_lib.frw_extract(st, 0, 30000, seed=34, threads=_threads(), n_cells=15, lattice=1)
    K = len(r_gpu["row"])
    zs = np.array([_z(r_gpu["row"][j], r_or["row"][j], r_gpu["se"][j], r_or["se"][j])
                   if (r_gpu["se"][j] > 0 or r_or["se"][j] > 0) else 0.0 for j in range(K)])
    print("cell lattice gpu", r_gpu["row"], r_gpu["se"], "oracle", r_or["row"], r_or["se"], "z", zs)
    assert zs.max() < z_crit(K)
    assert r_gpu["row"][0] > 0 and (r_gpu["row"][1:] <= 0).all()
