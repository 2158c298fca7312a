"""Oracle pins: Philox words, integer thresholds, lattice indexing, Eq. (6)."""
import os
import subprocess
from fractions import Fraction

import numpy as np
import pytest

HERE = os.path.dirname(os.path.abspath(__file__))
GOLD = os.path.join(HERE, "golden")


def _golden(name):
    out = []
    for line in open(os.path.join(GOLD, name)):
        line = line.strip()
        if line and not line.startswith("#"):
            out.append(line.split())
    return out


def test_philox_known_answers(oracle_lib):
    for row in _golden("philox4x32_10_kat.txt"):
        v = [int(x, 16) for x in row]
        out = oracle_lib.philox(v[0:4], v[4:6])
        assert [int(x) for x in out] == v[6:10]


@pytest.fixture(scope="module")
def torch_philox_shim(tmp_path_factory):
    """Philox from PyTorch's header-only engine, driven with raw key/counter."""
    import torch
    inc = os.path.join(os.path.dirname(torch.__file__), "include")
    d = tmp_path_factory.mktemp("shim")
    src = d / "shim.cpp"
    src.write_text(
        "#include <ATen/core/PhiloxRNGEngine.h>\n#include <cstdio>\n#include <cstdlib>\n"
        "int main(int c, char** v){ unsigned long long s=strtoull(v[1],0,0), k[4];"
        " for(int i=0;i<4;++i) k[i]=strtoull(v[2+i],0,0);"
        " at::philox_engine e(s, k[2] | (k[3]<<32), 0); e.set_offset(k[0] | (k[1]<<32));"
        " for(int i=0;i<4;++i) printf(\"%u\\n\", e()); }\n")
    exe = d / "shim"
    r = subprocess.run(["g++", "-O1", "-std=c++17", "-I", inc, "-o", str(exe), str(src)],
                       capture_output=True)
    if r.returncode:
        pytest.skip("torch Philox header does not compile here")
    return str(exe)


def test_philox_matches_torch_engine(oracle_lib, torch_philox_shim):
    rng = np.random.default_rng(7)
    for _ in range(20):
        seed = int(rng.integers(0, 2 ** 63))
        ctr = [int(x) for x in rng.integers(0, 2 ** 32, size=4)]
        out = subprocess.run([torch_philox_shim, str(seed)] + [str(c) for c in ctr],
                             capture_output=True, text=True, check=True).stdout.split()
        key = [seed & 0xffffffff, seed >> 32]
        assert [int(x) for x in oracle_lib.philox(ctr, key)] == [int(x) for x in out]


def test_rng_counter_layout(oracle_lib):
    """Word s of (seed, c1, walk, purpose) is word s&3 of the block with
    counter (s>>2, c1, walk lo, walk hi24 | purpose<<24)."""
    seed, c1, walk, purpose = 0x123456789ABCDEF, 77, (5 << 32) | 99, 3
    words = oracle_lib.rng_words(seed, c1, walk, purpose, 8, 8)
    key = [seed & 0xffffffff, seed >> 32]
    for blk in (2, 3):
        ctr = [blk, c1, walk & 0xffffffff, ((walk >> 32) & 0xffffff) | (purpose << 24)]
        ref = oracle_lib.philox(ctr, key)
        assert list(words[(blk - 2) * 4:(blk - 1) * 4]) == list(ref)


def test_uniform_vertex_thresholds_are_one_sixth(oracle_lib):
    """Uniform permittivity: every interior node of the vertex lattice moves to
    each neighbour with probability 1/6 (T_k = ceil((k+1) 2^32 / 6))."""
    for eps in (1e-3, 3.9, 25.0, 1e3):
        e = np.full((8, 8, 8), eps, dtype=np.float32)
        links, T = oracle_lib.vertex_thresholds(e)
        expect = [-(-((k + 1) << 32) // 6) for k in range(5)]
        assert (T == np.array(expect, dtype=np.uint32)).all()
        assert (links == links[0, 0]).all()


def _cell_probs(T):
    t = [0] + [int(x) for x in T] + [1 << 32]
    return [Fraction(t[d + 1] - t[d], 1 << 32) for d in range(6)]


def test_cell_lattice_eq6_closed_forms(oracle_lib):
    """Eq. (6) at uniform permittivity on the cell-centred lattice."""
    gold = {r[0]: Fraction(r[1]) for r in _golden("paper_constants.txt") if "/" in r[1]}
    N = 5
    e = np.full((N, N, N), 2.5, dtype=np.float32)
    links, T = oracle_lib.cell_thresholds(e)
    tol = Fraction(1, 1 << 31)

    def probs(i, j, k):
        return _cell_probs(T[(k * N + j) * N + i])

    p = probs(2, 2, 2)
    assert all(abs(x - Fraction(1, 6)) <= tol for x in p)
    p = probs(0, 2, 2)  # face node: -x is a panel
    assert abs(p[0] - gold["face_boundary"]) <= tol
    assert all(abs(x - gold["face_interior"]) <= tol for x in p[1:])
    p = probs(0, 0, 2)  # edge node
    assert abs(p[0] - gold["edge_boundary"]) <= tol and abs(p[2] - gold["edge_boundary"]) <= tol
    assert abs(p[1] - gold["edge_interior"]) <= tol and abs(p[5] - gold["edge_interior"]) <= tol
    p = probs(N - 1, N - 1, N - 1)  # corner node
    for d in (1, 3, 5):
        assert abs(p[d] - gold["corner_boundary"]) <= tol
    for d in (0, 2, 4):
        assert abs(p[d] - gold["corner_interior"]) <= tol


def test_cell_lattice_interface_coefficients(oracle_lib):
    """Eq. (6): alpha_i = eps_i / (eps_i + eps_v) towards an interior neighbour."""
    N = 3
    e = np.full((N, N, N), 2.0, dtype=np.float32)
    e[1, 1, 2] = 6.0  # +x neighbour of the centre
    links, T = oracle_lib.cell_thresholds(e)
    alpha = [Fraction(1, 2)] * 6
    alpha[1] = Fraction(6, 8)
    s = sum(alpha)
    p = _cell_probs(T[(1 * N + 1) * N + 1])
    for d in range(6):
        assert abs(p[d] - alpha[d] / s) <= Fraction(1, 1 << 31)


def test_threshold_rule_equals_mulhi_rule(oracle_lib):
    """d = #{k : u >= T_k} equals #{k : floor(u S_5 / 2^32) >= S_k} for random
    codes and words (the division-free form a kernel may use)."""
    rng = np.random.default_rng(3)
    for _ in range(300):
        g = rng.integers(1, 1 << 28, size=6).astype(np.uint64)
        S = np.cumsum(g)
        T = [int(((int(S[k]) << 32) + int(S[5]) - 1) // int(S[5])) for k in range(5)]
        us = list(rng.integers(0, 1 << 32, size=40)) + [t - 1 for t in T] + T
        for u in us:
            u = int(u) & 0xffffffff
            x = (u * int(S[5])) >> 32
            d_mulhi = sum(1 for k in range(5) if x >= int(S[k]))
            assert oracle_lib.choose_direction(u, T) == d_mulhi


def test_microwalk_step_uses_thresholds(oracle_lib):
    """A one-step walk: a 2-cell cube has a single interior node, so the hit
    is the neighbour chosen by word 0 against that node's thresholds."""
    rng = np.random.default_rng(5)
    for trial in range(20):
        e = rng.choice([1.0, 2.5, 7.0, 25.0], size=(2, 2, 2)).astype(np.float32)
        links, T = oracle_lib.vertex_thresholds(e)
        hits, steps = oracle_lib.microwalk(e, 0, 64, seed=trial, cube_index=9)
        words = [oracle_lib.rng_words(trial, 9, w, 0, 0, 1)[0] for w in range(64)]
        assert (steps == 1).all()
        # M = 1: hit index = face index = direction
        assert [oracle_lib.choose_direction(u, T[0]) for u in words] == list(hits)


def test_hit_index_layout(oracle_lib):
    """Hit indices cover [0, 6 M^2) and faces follow f = 2*axis + side."""
    from oracle.pins import vertex_boundary_nodes
    n = 6
    nodes = vertex_boundary_nodes(n)
    assert len({tuple(x) for x in nodes}) == 6 * (n - 1) ** 2
    e = np.full((n, n, n), 3.0, dtype=np.float32)
    hits, _ = oracle_lib.microwalk(e, 0, 4000, seed=1)
    assert hits.min() >= 0 and hits.max() < 6 * (n - 1) ** 2
