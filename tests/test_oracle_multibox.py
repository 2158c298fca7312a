"""Oracle pins for nets made of several boxes (Alg. 1 with a master net whose
conductor is a union of boxes).

The Gaussian surface is pinned against a brute-force voxel boundary: with box
coordinates and the growth g on a common grid, the boundary of the union of
grown boxes is exactly the set of voxel faces between an inside and an outside
voxel, so the oracle's rectangles must cover that set once and nothing else.
The capacitance pin is a closed form (two parallel-plate gaps in parallel),
and splitting a conductor into abutting boxes must change nothing.
"""
import numpy as np
import pytest

import workloads as W


def _voxel_boundary(grown, win_hi, h):
    """Boundary faces of the union of grown boxes on the voxel grid of pitch h
    over the window [0, win_hi): {(axis, side): bool (planes, n_ta, n_tb)},
    faces on the window's own faces excluded."""
    shape = tuple(int(round(w / h)) for w in win_hi)
    inside = np.zeros(shape, dtype=bool)
    for b in grown:
        lo = [max(0, int(round(b[a] / h))) for a in range(3)]
        hi = [min(shape[a], int(round(b[3 + a] / h))) for a in range(3)]
        if all(lo[a] < hi[a] for a in range(3)):
            inside[lo[0]:hi[0], lo[1]:hi[1], lo[2]:hi[2]] = True
    out = {}
    for a in range(3):
        x = np.moveaxis(inside, a, 0)
        faces = {s: np.zeros((x.shape[0] + 1,) + x.shape[1:], dtype=bool) for s in (0, 1)}
        faces[1][1:-1] = x[:-1] & ~x[1:]    # outward normal +a at plane k+1
        faces[0][1:-1] = ~x[:-1] & x[1:]    # outward normal -a at plane k+1
        out[(a, 1)], out[(a, 0)] = faces[1], faces[0]
    return out


def _rasterise(faces, win_hi, h):
    shape = tuple(int(round(w / h)) for w in win_hi)
    cnt = {}
    for a in range(3):
        t = [q for q in range(3) if q != a]
        for s in (0, 1):
            cnt[(a, s)] = np.zeros((shape[a] + 1, shape[t[0]], shape[t[1]]), dtype=np.int32)
    for f in faces:
        a, s = int(f[0]), int(f[1])
        t = [q for q in range(3) if q != a]
        p = int(round(f[2] / h))
        assert abs(p * h - f[2]) < 1e-5, "rectangle off the voxel grid"
        u0, u1 = int(round(f[3 + t[0]] / h)), int(round(f[6 + t[0]] / h))
        v0, v1 = int(round(f[3 + t[1]] / h)), int(round(f[6 + t[1]] / h))
        assert u0 < u1 and v0 < v1
        cnt[(a, s)][p, u0:u1, v0:v1] += 1
    return cnt


def _check_surface(oracle_lib, st, master, h, g_expected):
    g, area, faces = oracle_lib.gauss(st, master)
    assert g == pytest.approx(g_expected, abs=1e-6)
    sel = st.cond_net == master
    grown = [np.concatenate([b[:3] - g_expected, b[3:] + g_expected]) for b in st.cond[sel].astype(np.float64)]
    win_hi = st.win_hi.astype(np.float64)
    assert (st.win_lo == 0).all()
    ref = _voxel_boundary(grown, win_hi, h)
    got = _rasterise(faces, win_hi, h)
    n_ref = 0
    for key in ref:
        # every boundary voxel face covered exactly once, nothing else
        assert (got[key] == ref[key].astype(np.int32)).all(), key
        n_ref += int(ref[key].sum())
    assert area == pytest.approx(n_ref * h * h, rel=1e-5)
    assert np.sum(faces[:, 9]) == pytest.approx(area, rel=1e-12)
    return faces


def test_gauss_surface_sandwich_plates(oracle_lib):
    for split in (False, True):
        st = W.sandwich_plates(split)
        faces = _check_surface(oracle_lib, st, 0, 0.025, 0.175)
        # two faces of area 1 facing the middle plate: +z at 0.275, -z at 0.725
        up = faces[(faces[:, 0] == 2) & (faces[:, 1] == 1)]
        dn = faces[(faces[:, 0] == 2) & (faces[:, 1] == 0)]
        assert np.allclose(up[:, 2], 0.275) and np.allclose(dn[:, 2], 0.725)
        assert up[:, 9].sum() == pytest.approx(1.0) and dn[:, 9].sum() == pytest.approx(1.0)
        _check_surface(oracle_lib, st, 1, 0.025, 0.175)


def test_gauss_surface_c2_multibox(oracle_lib):
    """L-shaped master (wire cut in two, via, upper wire) on a 50 nm grid."""
    for split in (False, True):
        st = W.c2_multibox_structure(split)
        _check_surface(oracle_lib, st, 0, 0.05, 0.05)
        _check_surface(oracle_lib, st, 1, 0.05, 0.05)


@pytest.mark.parametrize("seed", range(6))
def test_gauss_surface_random_box_unions(oracle_lib, seed):
    """Random overlapping and abutting boxes of one net (grid 1/32, g = 2/32)."""
    st = W.random_multibox_net(seed)
    _check_surface(oracle_lib, st, 0, 1.0 / 32, 2.0 / 32)


def test_gauss_surface_orientation(oracle_lib):
    """Every rectangle has the union on its inner side only."""
    st = W.random_multibox_net(11)
    g, _, faces = oracle_lib.gauss(st, 0)
    grown = [np.concatenate([b[:3] - g, b[3:] + g]) for b in st.cond[st.cond_net == 0].astype(np.float64)]

    def inside(x):
        return any(all(b[a] < x[a] < b[3 + a] for a in range(3)) for b in grown)

    for f in faces:
        a, s = int(f[0]), int(f[1])
        c = 0.5 * (f[3:6] + f[6:9])
        e = np.zeros(3)
        e[a] = 1e-4 if s else -1e-4
        assert inside(c - e) and not inside(c + e)


@pytest.mark.parametrize("split", [False, True])
def test_sandwich_plates_closed_form(oracle_lib, split):
    """A master net of two plates around a grounded plate: C_00 = -C_01 =
    two parallel-plate capacitances (cut plates give the same)."""
    st = W.sandwich_plates(split)
    exact = W.sandwich_plates_exact()
    r = oracle_lib.frw_extract(st, 0, 40000, seed=21, threads=8)
    assert abs(r["row"][0] - exact) < 3 * r["se"][0] + 1e-3 * exact, (r["row"], r["se"], exact)
    assert abs(r["row"][1] + exact) < 3 * r["se"][1] + 1e-3 * exact
    assert r["row"][2] == 0.0


def test_split_non_master_net_changes_no_walk(oracle_lib):
    """Cutting net 1's wire into two abutting boxes leaves every walk of the
    multi-box master unchanged (same distances, same absorbing net)."""
    a = oracle_lib.frw_extract(W.c2_multibox_structure(False), 0, 3000, seed=8, threads=8, scores=True)
    b = oracle_lib.frw_extract(W.c2_multibox_structure(True), 0, 3000, seed=8, threads=8, scores=True)
    assert (a["net"] == b["net"]).all()
    assert (a["w"] == b["w"]).all()
