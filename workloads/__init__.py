"""Seeded synthetic inputs shared by the tests, the benchmark and the oracle.

This module holds geometry and permittivity descriptions only (no part of the
method's arithmetic).  The paper's test structures are proprietary industrial
layouts; the generators here stand in for them with the same ingredients: IC
interconnect wires as axis-aligned boxes, layered inter-layer dielectrics
(eps 2.7 / 3.9), conformal eps 7.0 coatings and eps 25 high-k fills.

All coordinates are float32 micrometres; boxes are half-open [lo, hi).
"""
from dataclasses import dataclass, field

import numpy as np

DIRICHLET, NEUMANN = 0, 1


@dataclass
class Structure:
    cond: np.ndarray          # (n_cond, 6) float32: lo xyz, hi xyz
    cond_net: np.ndarray      # (n_cond,) int32
    n_nets: int
    diel: np.ndarray          # (n_diel, 6) float32
    diel_eps: np.ndarray      # (n_diel,) float32
    layer_z0: np.ndarray      # (n_layers,) float32 (entry 0 unused: first layer from -inf)
    layer_eps: np.ndarray     # (n_layers,) float32
    win_lo: np.ndarray        # (3,) float32
    win_hi: np.ndarray        # (3,) float32
    bc: tuple = (DIRICHLET,) * 6
    name: str = ""
    meta: dict = field(default_factory=dict)

    @property
    def n_cond(self):
        return int(self.cond.shape[0])

    @property
    def n_diel(self):
        return int(self.diel.shape[0])


def _f32(a):
    return np.asarray(a, dtype=np.float32)


def make_structure(cond, nets, diel, diel_eps, layer_z0, layer_eps, win_lo, win_hi, bc, name="",
                   meta=None):
    cond = _f32(cond).reshape(-1, 6)
    diel = _f32(diel).reshape(-1, 6)
    return Structure(cond=cond, cond_net=np.asarray(nets, dtype=np.int32), n_nets=int(max(nets) + 1),
                     diel=diel, diel_eps=_f32(diel_eps).reshape(-1), layer_z0=_f32(layer_z0),
                     layer_eps=_f32(layer_eps), win_lo=_f32(win_lo), win_hi=_f32(win_hi),
                     bc=tuple(int(b) for b in bc), name=name, meta=meta or {})


def _grow(b, t):
    b = np.asarray(b, dtype=np.float64)
    return np.concatenate([b[:3] - t, b[3:] + t])


# ---------------------------------------------------------------------------
# Single transition cubes
# ---------------------------------------------------------------------------
def c1_eps():
    """8^3-cell cube, eps 3.9 with an off-centre 3x4x5-cell eps 7.0 block at
    cells x in [1,4), y in [1,5), z in [3,8); layout eps[k, j, i]."""
    e = np.full((8, 8, 8), 3.9, dtype=np.float32)
    e[3:8, 1:5, 1:4] = 7.0
    return e


C3_EPS = (2.5, 3.9, 7.0, 25.0)


def random_cube(n, rng, k_max=6, eps_choices=C3_EPS, background=3.9):
    """n^3 cube with 1..k_max random box inclusions (later boxes win)."""
    e = np.full((n, n, n), background, dtype=np.float32)
    k = int(rng.integers(1, k_max + 1))
    half = (n + 1) // 2
    for _ in range(k):
        ext = rng.integers(1, half + 1, size=3)
        org = np.array([rng.integers(0, n - ext[a] + 1) for a in range(3)])
        val = eps_choices[int(rng.integers(0, len(eps_choices)))]
        e[org[2]:org[2] + ext[2], org[1]:org[1] + ext[1], org[0]:org[0] + ext[0]] = val
    return e


def fig3a_cubes(n, count=500, seed=6, k_max=6, eps_min=1e-2):
    """Fig. 3(a) study: n^3 cubes whose background and 1..k_max randomly
    placed blocks take permittivities drawn from an exponential distribution
    of rate 0.1 (mean 10), clipped below at eps_min so that every cell code
    rint(eps * 2^16) is positive."""
    rng = np.random.Generator(np.random.PCG64([seed, n]))
    cubes = []
    half = (n + 1) // 2
    for _ in range(count):
        e = np.full((n, n, n), max(rng.exponential(10.0), eps_min), dtype=np.float32)
        for _ in range(int(rng.integers(1, k_max + 1))):
            ext = rng.integers(1, half + 1, size=3)
            org = np.array([rng.integers(0, n - ext[a] + 1) for a in range(3)])
            e[org[2]:org[2] + ext[2], org[1]:org[1] + ext[1], org[0]:org[0] + ext[0]] = \
                max(rng.exponential(10.0), eps_min)
        cubes.append(e)
    return cubes


def c3_sizes(count=4096, seed=3):
    """(n, walks) of the batched-transition workload: n even, log-uniform in
    [8, 32]; walks log-uniform in [1e3, 1e5]."""
    rng = np.random.Generator(np.random.PCG64(seed))
    out = []
    for _ in range(count):
        n = int(2 * round(np.exp(rng.uniform(np.log(8), np.log(32))) / 2))
        w = int(round(np.exp(rng.uniform(np.log(1e3), np.log(1e5)))))
        out.append((n, w))
    return out


def c3_cubes(count=4096, seed=3):
    """Batched-transition workload: list of (eps grid, walks)."""
    rng = np.random.Generator(np.random.PCG64(seed))
    cubes = []
    for _ in range(count):
        n = int(2 * round(np.exp(rng.uniform(np.log(8), np.log(32))) / 2))
        w = int(round(np.exp(rng.uniform(np.log(1e3), np.log(1e5)))))
        cubes.append((random_cube(n, rng), w))
    return cubes


# ---------------------------------------------------------------------------
# Structures
# ---------------------------------------------------------------------------
def parallel_plates(variant="uniform"):
    """1x1x1 um window with symmetry walls, plates z in [0, 0.1] (net 0) and
    z in [0.9, 1.0] (net 1); gap 0.8 um."""
    cond = [[0, 0, 0, 1, 1, 0.1], [0, 0, 0.9, 1, 1, 1.0]]
    diel, deps = [], []
    z0, le = [0.0], [3.9]
    if variant == "columns":
        diel, deps = [[0.5, 0, 0, 1, 1, 1]], [7.0]
    elif variant == "columns_highk":
        # the largest permittivity the library accepts, against both plates
        diel, deps = [[0.5, 0, 0, 1, 1, 1]], [1000.0]
    elif variant == "checkerboard":
        diel, deps = [[0.5, 0, 0, 1, 0.5, 1], [0, 0.5, 0, 0.5, 1, 1]], [7.0, 7.0]
    elif variant == "series":
        z0, le = [0.0, 0.5], [3.9, 2.7]
    elif variant == "stack":
        # twelve layers: the gap cut into twelve slabs of 0.8/12 um
        z0 = [0.0] + [0.1 + q * 0.8 / 12 for q in range(1, 12)]
        le = [STACK_EPS[q % 4] for q in range(12)]
    elif variant != "uniform":
        raise ValueError(variant)
    return make_structure(cond, [0, 1], diel, deps, z0, le, [0, 0, 0], [1, 1, 1], (NEUMANN,) * 6,
                          name="plates-" + variant)


EPS0 = 8.8541878128e-3  # fF/um
STACK_EPS = (3.9, 2.7, 7.0, 2.2)


def parallel_plates_exact(variant="uniform"):
    """Closed-form C_00 (= -C_01) of parallel_plates(variant), fF."""
    d, A = 0.8, 1.0
    if variant == "uniform":
        return EPS0 * 3.9 * A / d
    if variant in ("columns", "checkerboard"):
        return EPS0 * (0.5 * 3.9 + 0.5 * 7.0) * A / d
    if variant == "columns_highk":
        return EPS0 * (0.5 * 3.9 + 0.5 * 1000.0) * A / d
    if variant == "series":
        return EPS0 * A / (0.4 / 3.9 + 0.4 / 2.7)
    if variant == "stack":
        return EPS0 * A / sum((d / 12) / STACK_EPS[q % 4] for q in range(12))
    raise ValueError(variant)


def sandwich_plates(split=False):
    """Multi-box nets: 1x1x1 um window with symmetry walls and eps 3.9; net 0
    is two plates, z in [0, 0.1] and [0.9, 1.0], around net 1, a plate at
    z in [0.45, 0.55] (gaps 0.35 um).  split: every plate is also cut into
    boxes (net 0 into quadrants, net 1 into two halves), which leaves the
    conductors, and so the capacitances, unchanged."""
    if not split:
        cond = [[0, 0, 0, 1, 1, 0.1], [0, 0, 0.9, 1, 1, 1.0], [0, 0, 0.45, 1, 1, 0.55]]
        nets = [0, 0, 1]
    else:
        cond, nets = [], []
        for z0, z1 in ((0.0, 0.1), (0.9, 1.0)):
            for x0, x1 in ((0.0, 0.5), (0.5, 1.0)):
                for y0, y1 in ((0.0, 0.375), (0.375, 1.0)):
                    cond.append([x0, y0, z0, x1, y1, z1])
                    nets.append(0)
        cond += [[0, 0, 0.45, 0.625, 1, 0.55], [0.625, 0, 0.45, 1, 1, 0.55]]
        nets += [1, 1]
    return make_structure(cond, nets, [], [], [0.0], [3.9], [0, 0, 0], [1, 1, 1], (NEUMANN,) * 6,
                          name="sandwich-plates" + ("-split" if split else ""))


def sandwich_plates_exact():
    """Closed-form C_00 (= -C_01) of sandwich_plates(), fF: two parallel-plate
    gaps of 0.35 um over 1 um^2 in parallel."""
    return 2 * EPS0 * 3.9 * 1.0 / 0.35


def c2_structure():
    """Crossing wires in a 2x2x1 um grounded window: two x-directed wires at
    z in [0.30, 0.40] (nets 0, 1) under two y-directed wires at z in
    [0.60, 0.70] (nets 2, 3), 100 nm wide and thick, each with a 20 nm eps 7.0
    coating; background eps 3.9 below z = 0.5 and 2.7 above."""
    wires = [[0.2, 0.85, 0.30, 1.8, 0.95, 0.40],
             [0.2, 1.05, 0.30, 1.8, 1.15, 0.40],
             [0.85, 0.2, 0.60, 0.95, 1.8, 0.70],
             [1.05, 0.2, 0.60, 1.15, 1.8, 0.70]]
    coat = [_grow(w, 0.02) for w in wires]
    return make_structure(wires, [0, 1, 2, 3], coat, [7.0] * 4, [0.0, 0.5], [3.9, 2.7],
                          [0, 0, 0], [2, 2, 1], (DIRICHLET,) * 6, name="c2-crossing-wires")


def c2_multibox_structure(split_net1=False):
    """C2 with a multi-box master: net 0 is its x-wire cut at x = 1.0 into two
    abutting boxes, a via (x in [1.6, 1.7], z in [0.40, 0.60]) up from the
    wire's end and a y-directed wire (y in [0.85, 1.4]) on the upper level,
    all coated like the other wires.  split_net1: net 1's wire is also cut
    into two abutting boxes (same conductors)."""
    net0 = [[0.2, 0.85, 0.30, 1.0, 0.95, 0.40],
            [1.0, 0.85, 0.30, 1.8, 0.95, 0.40],
            [1.6, 0.85, 0.40, 1.7, 0.95, 0.60],
            [1.6, 0.85, 0.60, 1.7, 1.40, 0.70]]
    net1 = ([[0.2, 1.05, 0.30, 1.3, 1.15, 0.40], [1.3, 1.05, 0.30, 1.8, 1.15, 0.40]] if split_net1
            else [[0.2, 1.05, 0.30, 1.8, 1.15, 0.40]])
    others = [[0.85, 0.2, 0.60, 0.95, 1.8, 0.70],
              [1.05, 0.2, 0.60, 1.15, 1.8, 0.70]]
    cond = net0 + net1 + others
    nets = [0] * len(net0) + [1] * len(net1) + [2, 3]
    # coatings follow the conductors, not how they are cut into boxes
    coat = [_grow(w, 0.02) for w in net0 + [[0.2, 1.05, 0.30, 1.8, 1.15, 0.40]] + others]
    return make_structure(cond, nets, coat, [7.0] * len(coat), [0.0, 0.5], [3.9, 2.7],
                          [0, 0, 0], [2, 2, 1], (DIRICHLET,) * 6,
                          name="c2-multibox" + ("-split1" if split_net1 else ""),
                          meta={"master": 0})


def random_multibox_net(seed, n_boxes=5):
    """Unit window with symmetry walls and eps 3.9 holding net 1, a small box
    at the origin corner, and net 0, a union of n_boxes random boxes on a 1/32
    grid (overlapping, and one abutting another).  The box at (8, 8, 8)/32 is
    4/32 from net 1 in every axis and every other box is at least that far, so
    the Gaussian surface of net 0 grows its boxes by 2/32."""
    rng = np.random.default_rng(seed)
    q = 1.0 / 32
    boxes = [[8, 8, 8, 8 + int(rng.integers(2, 8)), 8 + int(rng.integers(2, 8)), 8 + int(rng.integers(2, 8))]]
    while len(boxes) < n_boxes - 1:
        lo = [int(rng.integers(8, 24)), int(rng.integers(2, 24)), int(rng.integers(2, 24))]
        hi = [min(30, lo[a] + int(rng.integers(1, 9))) for a in range(3)]
        boxes.append(lo + hi)
    # one box abutting the previous one along x
    b = boxes[-1]
    lo = [b[3], b[1] + int(rng.integers(0, 2)), b[2]]
    hi = [min(31, lo[0] + int(rng.integers(1, 6))), b[4] + int(rng.integers(0, 3)), b[5]]
    hi[1] = min(31, max(hi[1], lo[1] + 1))
    boxes.append(lo + hi)
    cond = [[c * q for c in bx] for bx in boxes] + [[0, 0, 0, 4 * q, 4 * q, 4 * q]]
    nets = [0] * len(boxes) + [1]
    return make_structure(cond, nets, [], [], [0.0], [3.9], [0, 0, 0], [1, 1, 1], (NEUMANN,) * 6,
                          name="random-multibox-%d" % seed)


C4_STACK_Z0 = (0.0, 0.4, 0.6, 0.9, 1.1, 1.4, 1.6)
C4_STACK_EPS = (3.9, 2.7, 3.9, 2.7, 3.9, 2.7, 3.9)


def interconnect(side, tracks_per_layer, rng, height=2.0, highk_p=0.1, coat=0.02):
    """Three metal layers (z in [0.45,0.55], [0.95,1.05], [1.45,1.55]; directions
    x, y, x) of `tracks_per_layer` wires each, pitch U[0.08, 0.20] um, width
    pitch/2, random length U[1, 20] um clamped to the window; 20 nm eps 7.0
    coatings; each gap between neighbouring tracks gets an eps 25 fill over the
    common length with probability highk_p."""
    metal = ((0.45, 0.55, 0), (0.95, 1.05, 1), (1.45, 1.55, 0))
    cond, diel, deps = [], [], []
    fills = []
    for (z_lo, z_hi, along) in metal:
        pitch = rng.uniform(0.08, 0.20, size=tracks_per_layer)
        width = pitch / 2
        span = float(np.sum(pitch))
        pos = side / 2 - span / 2
        tracks = []
        for t in range(tracks_per_layer):
            lo_c = pos + (pitch[t] - width[t]) / 2
            hi_c = lo_c + width[t]
            pos += pitch[t]
            L = min(rng.uniform(1.0, 20.0), side - 0.2)
            start = 0.1 + rng.uniform() * (side - 0.2 - L)
            if along == 0:
                box = [start, lo_c, z_lo, start + L, hi_c, z_hi]
            else:
                box = [lo_c, start, z_lo, hi_c, start + L, z_hi]
            tracks.append((box, start, start + L, lo_c, hi_c))
            cond.append(box)
        for t in range(tracks_per_layer - 1):
            if rng.uniform() < highk_p:
                a, b = tracks[t], tracks[t + 1]
                s0, s1 = max(a[1], b[1]), min(a[2], b[2])
                if s1 <= s0:
                    continue
                g0, g1 = a[4], b[3]
                if along == 0:
                    fills.append([s0, g0, z_lo, s1, g1, z_hi])
                else:
                    fills.append([g0, s0, z_lo, g1, s1, z_hi])
    for box in cond:
        diel.append(_grow(box, coat))
        deps.append(7.0)
    for f in fills:
        diel.append(f)
        deps.append(25.0)
    return cond, diel, deps


def c4_structure(seed=4):
    """20x20x2 um three-layer interconnect window, 64 wires per layer (192
    nets), layered ILD 3.9/2.7, conformal eps 7.0 coatings and eps 25 fills."""
    rng = np.random.Generator(np.random.PCG64(seed))
    side = 20.0
    cond, diel, deps = interconnect(side, 64, rng)
    st = make_structure(cond, list(range(len(cond))), diel, deps, C4_STACK_Z0, C4_STACK_EPS,
                        [0, 0, 0], [side, side, 2.0], (DIRICHLET,) * 6, name="c4-interconnect")
    # master: middle-layer wire nearest to the window centre
    mid = [i for i, b in enumerate(st.cond) if b[2] > 0.9 and b[5] < 1.1]
    cen = [(st.cond[i][:3] + st.cond[i][3:]) / 2 for i in mid]
    d = [max(abs(c[0] - 10), abs(c[1] - 10)) for c in cen]
    st.meta["master"] = int(mid[int(np.argmin(d))])
    return st


def request_structure(K, rng):
    """A serving request: a window built like the large structure with
    ceil(K/3) tracks per layer and side max(2, 20*sqrt(K/192)) um."""
    tracks = int(np.ceil(K / 3))
    side = float(max(2.0, 20.0 * np.sqrt(K / 192.0)))
    cond, diel, deps = interconnect(side, tracks, rng)
    return make_structure(cond, list(range(len(cond))), diel, deps, C4_STACK_Z0, C4_STACK_EPS,
                          [0, 0, 0], [side, side, 2.0], (DIRICHLET,) * 6, name="req-%d" % K)


def c5_requests(count=2000, seed=5):
    """Serving workload: (structure, master, walk budget, seed) per request."""
    rng = np.random.Generator(np.random.PCG64(seed))
    out = []
    for i in range(count):
        K = int(round(np.exp(rng.uniform(np.log(4), np.log(200)))))
        st = request_structure(K, rng)
        master = int(rng.integers(0, st.n_nets))
        budget = int(round(np.exp(rng.uniform(np.log(1e5), np.log(1e7)))))
        out.append((st, master, budget, i))
    return out
