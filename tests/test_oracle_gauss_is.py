"""Importance sampling of the Gaussian-surface point (the first transition of
Alg. 1 is importance sampling with its weight) in the oracle.

Reading: G is cut into patches of edge at most g; a walk picks a patch with
probability proportional to q = area x K(patch centre), K the first-transition
kernel sum at the patch centre, then a uniform point in it, and its weight is
multiplied by Q area / q (Q = sum of q) instead of |G|.  The estimator stays
unbiased for any positive q.  Pins: the parallel-plate closed forms, the same
rows as uniform sampling on the crossing wires, and a smaller standard error
where K varies over G (a half-filled eps 1e3 gap).
"""
import os
import sys

import numpy as np
import pytest

import workloads as W

sys.path.insert(0, os.path.dirname(os.path.abspath(__file__)))
from _stats import z_crit  # noqa: E402


@pytest.mark.parametrize("variant", ["uniform", "columns", "columns_highk"])
def test_importance_sampling_meets_plate_closed_forms(oracle_lib, variant):
    st = W.parallel_plates(variant)
    exact = W.parallel_plates_exact(variant)
    r = oracle_lib.frw_extract(st, 0, 40000, seed=3, threads=8, gauss_is=1.0)
    print(variant, r["row"][0], r["se"][0], exact)
    assert abs(r["row"][0] - exact) < 3 * r["se"][0]
    assert abs(r["row"][1] + exact) < 3 * r["se"][1]


def test_importance_sampling_lowers_variance_where_kernel_varies(oracle_lib):
    st = W.parallel_plates("columns_highk")
    u = oracle_lib.frw_extract(st, 0, 40000, seed=4, threads=8)
    s = oracle_lib.frw_extract(st, 0, 40000, seed=4, threads=8, gauss_is=1.0)
    print("SE uniform %.5f, importance %.5f" % (u["se"][0], s["se"][0]))
    assert s["se"][0] < 0.85 * u["se"][0]


def test_importance_sampling_keeps_the_c2_row(oracle_lib):
    st = W.c2_structure()
    u = oracle_lib.frw_extract(st, 0, 60000, seed=5, threads=8)
    s = oracle_lib.frw_extract(st, 0, 60000, seed=6, threads=8, gauss_is=1.0)
    z = np.abs(u["row"] - s["row"]) / np.hypot(u["se"], s["se"])
    print("uniform", u["row"], u["se"])
    print("importance", s["row"], s["se"])
    assert z.max() < z_crit(5)
    # the row still sums to zero with the enclosure column
    assert abs(s["row"].sum()) < 3 * np.sqrt((s["se"] ** 2).sum())
