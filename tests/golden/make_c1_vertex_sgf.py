"""Writes c1_vertex_sgf.txt: exact exit statistics of the single-cube
workload on the vertex lattice (Eqs. 8 and 11 via Theorem 1), from a sparse
LU solve of the absorbing chain in oracle/pins.py (not the oracle's CG solver,
which the file is used to check).

    python tests/golden/make_c1_vertex_sgf.py
"""
import os
import sys

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
sys.path.insert(0, ROOT)

import workloads  # noqa: E402
from oracle import pins  # noqa: E402

OUT = os.path.join(os.path.dirname(os.path.abspath(__file__)), "c1_vertex_sgf.txt")


def stats(eps):
    n = eps.shape[0]
    codes = np.rint(eps.astype(np.float64) * 65536.0)  # cell codes rint(eps 2^16)
    P, etau = pins.vertex_exit_distribution(pins.vertex_links_from_codes(codes), n)
    return P, etau


def main():
    P, etau = stats(workloads.c1_eps())
    faces = P.reshape(6, -1).sum(axis=1)
    Pu, etu = stats(np.full((8, 8, 8), 3.9, dtype=np.float32))
    M = 7
    lines = [
        "# Exact exit statistics of the single-cube workload (8^3 cells, eps 3.9 with",
        "# an eps 7.0 block at cells x in [1,4), y in [1,5), z in [3,8)) on the vertex",
        "# lattice reading of Sec. III-A (Eq. 6 as face conductance), Eqs. (8) and (11).",
        "# Written by make_c1_vertex_sgf.py (sparse LU of the absorbing chain,",
        "# oracle/pins.py); not printed in the paper.  Tolerance 1e-4 (relative).",
        "etau %.7g" % etau,
        "face_total " + " ".join("%.7g" % f for f in faces),
        "node_min %.7g" % P.min(),
        "node_max %.7g" % P.max(),
        "# uniform eps, n = 8: each face 1/6; +z face-centre node; E(tau)",
        "uniform8_face_centre_pz %.7g" % Pu[5 * M * M + 3 * M + 3],
        "uniform8_etau %.7g" % etu,
    ]
    with open(OUT, "w") as f:
        f.write("\n".join(lines) + "\n")
    print("\n".join(lines))


if __name__ == "__main__":
    main()
