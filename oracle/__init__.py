"""CPU oracle for FRW capacitance extraction with MicroWalk transitions.

TEST INFRASTRUCTURE ONLY: a plain, slow binary64 reference (``mwo.cpp``) and
its ctypes wrapper.  Only the test suite, ``__graft_entry__.smoke()`` and the
CPU-baseline leg of ``bench.py`` may import this package.  It shares no code
with the GPU library ``paper_2507_09730_amd`` and never imports it.

Functions mirror the passages of the paper they implement (Huang & Yu,
arXiv 2507.09730): Alg. 3 (MicroWalk), Eqs. (6)-(8) and (11) (finite-difference
SGF and expected walk length), Alg. 1 (FRW extraction).
"""
import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SO = os.path.join(_HERE, "libmwo.so")
_SRC = os.path.join(_HERE, "mwo.cpp")

_lib = None


def build(force=False):
    """Compile mwo.cpp into libmwo.so (g++, binary64, no FMA contraction)."""
    if not force and os.path.exists(_SO) and os.path.getmtime(_SO) >= os.path.getmtime(_SRC):
        return _SO
    tmp = _SO + ".tmp"
    cmd = ["g++", "-O2", "-std=c++17", "-ffp-contract=off", "-fPIC", "-shared",
           "-pthread", "-o", tmp, _SRC]
    subprocess.run(cmd, check=True)
    os.replace(tmp, _SO)
    return _SO


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(_SO):
            build()
        _lib = ctypes.CDLL(_SO)
    return _lib


def _p(a):
    return a.ctypes.data_as(ctypes.c_void_p) if a is not None else None


U64, I32, DBL = ctypes.c_uint64, ctypes.c_int, ctypes.c_double


def philox(ctr, key):
    """Philox4x32-10 block (Salmon et al., SC'11)."""
    c = np.asarray(ctr, dtype=np.uint32)
    k = np.asarray(key, dtype=np.uint32)
    out = np.zeros(4, dtype=np.uint32)
    lib().mwo_philox4x32_10(_p(c), _p(k), _p(out))
    return out


def rng_words(seed, c1, walk, purpose, s0, count):
    out = np.zeros(count, dtype=np.uint32)
    lib().mwo_rng_words(U64(seed), ctypes.c_uint32(c1), U64(walk), ctypes.c_uint32(purpose),
                        U64(s0), ctypes.c_int64(count), _p(out))
    return out


def vertex_codes(eps):
    e = np.ascontiguousarray(eps, dtype=np.float32).ravel()
    out = np.zeros(e.size, dtype=np.uint64)
    lib().mwo_vertex_codes(_p(e), ctypes.c_int64(e.size), _p(out))
    return out


def vertex_thresholds(eps):
    """Link codes (NI x 6) and thresholds (NI x 5) of the vertex lattice."""
    e = np.ascontiguousarray(eps, dtype=np.float32)
    n = e.shape[0]
    ni = (n - 1) ** 3
    links = np.zeros((ni, 6), dtype=np.uint64)
    T = np.zeros((ni, 5), dtype=np.uint32)
    rc = lib().mwo_vertex_thresholds(_p(e), I32(n), _p(links), _p(T))
    if rc:
        raise ValueError("vertex lattice needs even n")
    return links, T


def cell_thresholds(eps):
    """Link codes (N^3 x 6) and thresholds (N^3 x 5) of the cell lattice (Eq. 6)."""
    e = np.ascontiguousarray(eps, dtype=np.float32)
    n = e.shape[0]
    links = np.zeros((n ** 3, 6), dtype=np.uint64)
    T = np.zeros((n ** 3, 5), dtype=np.uint32)
    rc = lib().mwo_cell_thresholds(_p(e), I32(n), _p(links), _p(T))
    if rc:
        raise ValueError("cell lattice needs odd N")
    return links, T


def choose_direction(u, T):
    t = np.ascontiguousarray(T, dtype=np.uint32)
    return lib().mwo_choose_direction(ctypes.c_uint32(int(u)), _p(t))


def microwalk(eps, lattice, n_walks, first_walk=0, seed=0, cube_index=0):
    """Alg. 3: boundary hit indices and step counts of n_walks walks."""
    e = np.ascontiguousarray(eps, dtype=np.float32)
    n = e.shape[0]
    hits = np.zeros(n_walks, dtype=np.int32)
    steps = np.zeros(n_walks, dtype=np.int32)
    rc = lib().mwo_microwalk(_p(e), I32(n), I32(lattice), U64(n_walks), U64(first_walk),
                             U64(seed), ctypes.c_uint32(cube_index), _p(hits), _p(steps))
    if rc:
        raise ValueError("invalid lattice size for this lattice")
    return hits, steps


def sgf_vertex(codes, src=None):
    """Exact exit distribution (Eq. 8) and E(tau) (Eq. 11) on the vertex lattice."""
    c = np.ascontiguousarray(codes, dtype=np.uint64)
    n = c.shape[0]
    if src is None:
        src = (n // 2,) * 3
    s = np.asarray(src, dtype=np.int32)
    M = n - 1
    P = np.zeros(6 * M * M)
    et = ctypes.c_double(0)
    rc = lib().mwo_sgf_vertex(_p(c), I32(n), _p(s), _p(P), ctypes.byref(et))
    if rc:
        raise RuntimeError("sgf solve failed (%d)" % rc)
    return P, et.value


def _plane_seq(planes, lattice):
    if lattice == 1:
        # cell lattice: the planes' permittivities, passed as float bits
        return np.ascontiguousarray(np.asarray(planes, dtype=np.float32).view(np.uint32), dtype=np.uint64)
    return np.ascontiguousarray(planes, dtype=np.uint64)


def sgf_cell(eps, src=None):
    """Exact exit distribution (6 N^2, hit-index order) and E(tau) on the
    cell-centred lattice (Sec. III-A, Eq. 6 codes) of an (N, N, N) [k, j, i]
    permittivity grid, N odd, from cell src (default the centre)."""
    e = np.ascontiguousarray(eps, dtype=np.float32)
    N = e.shape[0]
    if src is None:
        src = ((N - 1) // 2,) * 3
    s = np.asarray(src, dtype=np.int32)
    P = np.zeros(6 * N * N)
    et = ctypes.c_double(0)
    rc = lib().mwo_sgf_cell(_p(e), I32(N), _p(s), _p(P), ctypes.byref(et))
    if rc:
        raise RuntimeError("cell sgf solve failed (%d)" % rc)
    return P, et.value


def hop_table(plane_codes, axis, lattice=0):
    """Exit distribution (hit-index order) from the centre of a cube
    stratified along `axis` (Sec. III-C, Eq. 8): 6 M^2 entries of the vertex
    lattice from its plane codes, or with lattice=1, 6 N^2 entries of the
    cell-centred lattice from its plane permittivities."""
    seq = _plane_seq(plane_codes, lattice)
    n = int(seq.size)
    P = np.zeros(6 * (n - 1) ** 2 if lattice == 0 else 6 * n * n)
    rc = lib().mwo_hop_table(I32(lattice), I32(n), I32(axis), _p(seq), _p(P))
    if rc:
        raise ValueError("hop table failed (%d)" % rc)
    return P


def first_table(plane_codes, axis, normal_axis, lattice=0):
    """First-transition ingredients of a stratified cube: exit distributions
    from the centre c and from c +- e_normal, and the link conductances G+, G-
    of c along the normal (eps units).  lattice=1: the cell-centred lattice,
    planes given by their permittivities."""
    seq = _plane_seq(plane_codes, lattice)
    n = int(seq.size)
    nb = 6 * (n - 1) ** 2 if lattice == 0 else 6 * n * n
    Pc, Pp, Pm = np.zeros(nb), np.zeros(nb), np.zeros(nb)
    gp, gm = ctypes.c_double(0), ctypes.c_double(0)
    rc = lib().mwo_first_table(I32(lattice), I32(n), I32(axis), I32(normal_axis), _p(seq), _p(Pc), _p(Pp),
                               _p(Pm), ctypes.byref(gp), ctypes.byref(gm))
    if rc:
        raise ValueError("first table failed (%d)" % rc)
    return Pc, Pp, Pm, gp.value, gm.value


def _structure_args(st):
    cond = np.zeros((st.n_cond, 7))
    cond[:, :6] = st.cond.astype(np.float64)
    cond[:, 6] = st.cond_net
    diel = np.zeros((max(st.n_diel, 1), 7))
    if st.n_diel:
        diel[:st.n_diel, :6] = st.diel.astype(np.float64)
        diel[:st.n_diel, 6] = st.diel_eps.astype(np.float64)
    z0 = st.layer_z0.astype(np.float64)
    le = st.layer_eps.astype(np.float64)
    win = np.concatenate([st.win_lo, st.win_hi]).astype(np.float64)
    bc = np.asarray(st.bc, dtype=np.int32)
    keep = (cond, diel, z0, le, win, bc)
    args = [_p(cond), I32(st.n_cond), I32(st.n_nets), _p(diel), I32(st.n_diel),
            _p(z0), _p(le), I32(len(z0)), _p(win), _p(bc)]
    return args, keep


def build_cube(st, centre, R, n):
    """Voxelised cube codes (n^3) and (class, axis): 0 uniform, 1 stratified, 2 other."""
    args, keep = _structure_args(st)
    c = np.asarray(centre, dtype=np.float64)
    codes = np.zeros(n ** 3, dtype=np.uint64)
    cls = np.zeros(2, dtype=np.int32)
    lib().mwo_build_cube(*args, _p(c), DBL(R), I32(n), _p(codes), _p(cls))
    return codes.reshape(n, n, n), (int(cls[0]), int(cls[1]))


def dist(st, p):
    args, keep = _structure_args(st)
    pp = np.asarray(p, dtype=np.float64)
    d = ctypes.c_double(0)
    who = ctypes.c_int32(0)
    lib().mwo_dist(args[0], args[1], args[2], args[8], args[9], _p(pp), ctypes.byref(d),
                   ctypes.byref(who))
    return d.value, who.value


def gauss(st, master, cap=4096):
    """Gaussian surface of net `master`: g, total area and its rectangles as
    rows [axis, side, plane, lo3, hi3, area]."""
    args, keep = _structure_args(st)
    g = ctypes.c_double(0)
    area = ctypes.c_double(0)
    faces = np.zeros((cap, 10))
    nf = ctypes.c_int32(0)
    rc = lib().mwo_gauss(args[0], args[1], args[2], args[8], args[9], I32(master), ctypes.byref(g),
                         ctypes.byref(area), _p(faces), I32(cap), ctypes.byref(nf))
    if rc == -2:
        raise ValueError("Gaussian surface has more than %d rectangles" % cap)
    if rc:
        raise ValueError("no Gaussian surface (touching conductors?)")
    return g.value, area.value, faces[:nf.value]


STAT_KEYS = ("walks", "hops", "micro_steps", "cls_uniform", "cls_stratified", "cls_other",
             "first_uniform", "first_normal", "first_other_axis", "first_homogenised",
             "cache_miss", "env_absorbed", "hop_cap")


def frw_extract(st, master, n_walks, seed=0, first_walk=0, n_cells=16, hybrid=1,
                abs_tol_rel=1e-6, threads=1, scores=False, expand=1.0, kernel_limits=False, gauss_is=0.0,
                lattice=0):
    """Alg. 1: capacitance row (fF, last entry env) and standard errors.
    expand > 1: MicroWalk-E transitions with that expansion factor.
    gauss_is > 0: importance sampling of the Gaussian-surface point over
    patches of edge at most gauss_is x g, each weighted by its area times the
    first-transition kernel sum K at its centre (0: uniform by area).
    Transition cubes are the largest conductor-free cubes (expanded by the
    MicroWalk-E rule when expand > 1).  kernel_limits=True reproduces the GPU
    kernel's capacity rule instead (a cube is halved while more than 16
    dielectric boxes, or for MicroWalk-E 7 conductors, touch it); it exists
    only so that single walks can be compared with the kernel's one by one.
    lattice=1: every cube on the cell-centred lattice of Sec. III-A (n_cells
    odd; walks start in the centre cell and leave through panel centres)."""
    args, keep = _structure_args(st)
    K = st.n_nets + 1
    row = np.zeros(K)
    se = np.zeros(K)
    nets = np.zeros(n_walks, dtype=np.int32) if scores else None
    w = np.zeros(n_walks) if scores else None
    stats = np.zeros(13, dtype=np.uint64)
    rc = lib().mwo_frw_extract(*args, I32(master), U64(n_walks), U64(first_walk), U64(seed),
                               I32(n_cells), I32(hybrid), DBL(abs_tol_rel), DBL(expand),
                               I32(1 if kernel_limits else 0), DBL(gauss_is), I32(lattice), I32(threads),
                               _p(row), _p(se), _p(nets), _p(w), _p(stats))
    if rc:
        raise RuntimeError("oracle frw_extract failed (%d)" % rc)
    out = {"row": row, "se": se, "stats": dict(zip(STAT_KEYS, (int(x) for x in stats)))}
    if scores:
        out["net"] = nets
        out["w"] = w
    return out


def microwalk_e_cube(st, centre, R, n, n_walks, seed=0, first_walk=0, c1=0):
    """MicroWalk-E (Sec. III-B) on one expanded cube of structure st (centre,
    half-size R, n cells): per walk the boundary hit index, or -2 with the
    absorbing net (n_nets for the grounded enclosure), and the step count."""
    args, keep = _structure_args(st)
    c = np.asarray(centre, dtype=np.float64)
    hits = np.zeros(n_walks, dtype=np.int32)
    nets = np.zeros(n_walks, dtype=np.int32)
    steps = np.zeros(n_walks, dtype=np.int32)
    rc = lib().mwo_microwalk_e_cube(*args, _p(c), DBL(R), I32(n), U64(n_walks), U64(first_walk), U64(seed),
                                    ctypes.c_uint32(c1), _p(hits), _p(nets), _p(steps))
    if rc == -2:
        raise ValueError("the cube's centre node is absorbing")
    if rc:
        raise ValueError("vertex lattice needs even n")
    return hits, nets, steps
