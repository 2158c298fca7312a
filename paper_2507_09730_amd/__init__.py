"""libmwalk: FRW capacitance extraction with MicroWalk transitions on MI355X.

Thin ctypes binding of the C ABI declared in ``include/libmwalk.h`` (same
names, argument marshalling only).  Device memory and streams come from
PyTorch; every step of the method runs in the library's HIP kernels.  Importing
this package raises ImportError when the built library is missing: there is
no fallback implementation.
"""
import ctypes
import os

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libmwalk.so")

if not os.path.exists(LIB_PATH):
    raise ImportError("libmwalk.so is not built (run __graft_entry__.build() or "
                      "python paper_2507_09730_amd/build.py)")

_lib = ctypes.CDLL(LIB_PATH)

MW_OK, MW_EINVAL, MW_ENOMEM, MW_EDEVICE, MW_EBUSY, MW_ENOTREADY, MW_EGEOM, MW_ELIMIT = \
    0, -1, -2, -3, -4, -5, -6, -7
MW_LATTICE_VERTEX, MW_LATTICE_CELL = 0, 1
MW_MAX_REGIONS = 16
_NAMES = {-1: "MW_EINVAL", -2: "MW_ENOMEM", -3: "MW_EDEVICE", -4: "MW_EBUSY",
          -5: "MW_ENOTREADY", -6: "MW_EGEOM", -7: "MW_ELIMIT"}


class MWError(RuntimeError):
    def __init__(self, status, msg):
        super().__init__("%s: %s" % (_NAMES.get(status, status), msg))
        self.status = status


_lib.mw_last_error.restype = ctypes.c_char_p
_lib.mw_structure_create.argtypes = [ctypes.c_void_p, ctypes.c_void_p]
_lib.mw_batch_plan_run.argtypes = [ctypes.c_void_p, ctypes.c_uint64, ctypes.c_void_p]
_lib.mw_batch_plan_destroy.argtypes = [ctypes.c_void_p]
_lib.mw_structure_destroy.argtypes = [ctypes.c_void_p]


def mw_last_error():
    return _lib.mw_last_error().decode()


def _check(rc):
    if rc != MW_OK:
        raise MWError(rc, mw_last_error())


def _stream(stream):
    import torch
    s = stream if stream is not None else torch.cuda.current_stream()
    return ctypes.c_void_p(s.cuda_stream)


def _ptr(t):
    return ctypes.c_void_p(t.data_ptr()) if t is not None else None


U64, I32, U32 = ctypes.c_uint64, ctypes.c_int32, ctypes.c_uint32


def mw_init(device=0):
    _check(_lib.mw_init(I32(device)))


class mw_tune(ctypes.Structure):
    _fields_ = [("tile_form", ctypes.c_int32), ("waves_per_wg", ctypes.c_int32),
                ("refill_every", ctypes.c_int32), ("item_walks", ctypes.c_int32),
                ("walks_per_lane", ctypes.c_int32)]


def mw_transition(eps, n_walks, lattice=MW_LATTICE_VERTEX, first_walk=0, seed=0, cube_index=0,
                  hits=None, steps=None, want_steps=True, stream=None):
    """Alg. 3 on one cube.  eps: CUDA float32 tensor (n, n, n) indexed
    [k, j, i].  Returns (hits, steps) int32 CUDA tensors."""
    import torch
    assert eps.is_cuda and eps.dtype == torch.float32 and eps.is_contiguous()
    n = int(eps.shape[0])
    assert eps.shape == (n, n, n)
    if hits is None:
        hits = torch.empty(n_walks, dtype=torch.int32, device=eps.device)
    if steps is None and want_steps:
        steps = torch.empty(n_walks, dtype=torch.int32, device=eps.device)
    _check(_lib.mw_transition(_ptr(eps), I32(n), I32(lattice), U64(n_walks), U64(first_walk),
                              U64(seed), U32(cube_index), _ptr(hits), _ptr(steps), _stream(stream)))
    return hits, steps


def mw_transition_noalloc(eps, n_walks, lattice=MW_LATTICE_VERTEX, first_walk=0, seed=0, cube_index=0,
                          hits=None, steps=None, want_steps=True, stream=None):
    """mw_transition through the entry point that allocates no device memory
    (static per-device scratch).  The caller passes the outputs to keep the
    call allocation-free; when they are None they are created here."""
    import torch
    assert eps.is_cuda and eps.dtype == torch.float32 and eps.is_contiguous()
    n = int(eps.shape[0])
    assert eps.shape == (n, n, n)
    if hits is None:
        hits = torch.empty(n_walks, dtype=torch.int32, device=eps.device)
    if steps is None and want_steps:
        steps = torch.empty(n_walks, dtype=torch.int32, device=eps.device)
    _check(_lib.mw_transition_noalloc(_ptr(eps), I32(n), I32(lattice), U64(n_walks), U64(first_walk),
                                      U64(seed), U32(cube_index), _ptr(hits), _ptr(steps), _stream(stream)))
    return hits, steps


def pack_cubes(eps_list, device="cuda"):
    """Concatenates cube grids into one device buffer: (eps_cat, n_cells, eps_off)."""
    import torch
    ns = np.array([int(e.shape[0]) for e in eps_list], dtype=np.int32)
    cells = ns.astype(np.int64) ** 3
    eps_off = np.zeros(len(eps_list), dtype=np.int64)
    if len(eps_list):
        eps_off[1:] = np.cumsum(cells)[:-1]
        flat = np.concatenate([np.asarray(e, dtype=np.float32).reshape(-1) for e in eps_list])
        eps_cat = torch.from_numpy(flat).to(device)
    else:
        eps_cat = torch.empty(1, device=device)
    return eps_cat, ns, eps_off


def mw_transition_batch(eps_list, walks, lattice=MW_LATTICE_VERTEX, seed=0, tune=None,
                        want_steps=True, device="cuda", stream=None, packed=None, out=None):
    """Many cubes in one persistent launch.  eps_list: list of (n, n, n)
    float32 arrays (or packed=(eps_cat, n_cells, eps_off) from pack_cubes);
    walks: walks per cube.  Returns (hits_cat, steps_cat, out_off) with cube
    c's results at out_off[c]."""
    import torch
    eps_cat, ns, eps_off = packed if packed is not None else pack_cubes(eps_list, device)
    n_cubes = len(ns)
    walks = np.asarray(walks, dtype=np.uint64)
    out_off = np.zeros(n_cubes, dtype=np.int64)
    if n_cubes:
        out_off[1:] = np.cumsum(walks.astype(np.int64))[:-1]
    total = int(walks.sum())
    if out is not None:
        hits, steps = out
    else:
        hits = torch.empty(max(total, 1), dtype=torch.int32, device=eps_cat.device)
        steps = (torch.empty(max(total, 1), dtype=torch.int32, device=eps_cat.device)
                 if want_steps else None)
    t = None
    if tune is not None:
        t = mw_tune(*[int(tune.get(k, 0)) for k, _ in mw_tune._fields_])
    _check(_lib.mw_transition_batch(
        I32(n_cubes), _ptr(eps_cat), eps_off.ctypes.data_as(ctypes.c_void_p),
        ns.ctypes.data_as(ctypes.c_void_p), I32(lattice), walks.ctypes.data_as(ctypes.c_void_p),
        out_off.ctypes.data_as(ctypes.c_void_p), U64(seed), _ptr(hits), _ptr(steps),
        ctypes.byref(t) if t is not None else None, _stream(stream)))
    return hits[:total], (steps[:total] if steps is not None else None), out_off


def _batch_arrays(eps_list, walks, device, packed):
    eps_cat, ns, eps_off = packed if packed is not None else pack_cubes(eps_list, device)
    walks = np.asarray(walks, dtype=np.uint64)
    out_off = np.zeros(len(ns), dtype=np.int64)
    if len(ns):
        out_off[1:] = np.cumsum(walks.astype(np.int64))[:-1]
    return eps_cat, ns, eps_off, walks, out_off


def _vp(a):
    return a.ctypes.data_as(ctypes.c_void_p)


def mw_autotune_batch(eps_list, walks, lattice=MW_LATTICE_VERTEX, device="cuda", packed=None,
                      stream=None):
    """Times candidate launch settings on this batch; returns the fastest as a
    dict (also remembered for later untuned batches of the same shape)."""
    import torch
    eps_cat, ns, eps_off, walks, out_off = _batch_arrays(eps_list, walks, device, packed)
    total = int(walks.sum())
    hits = torch.empty(max(total, 1), dtype=torch.int32, device=eps_cat.device)
    steps = torch.empty(max(total, 1), dtype=torch.int32, device=eps_cat.device)
    best = mw_tune()
    _check(_lib.mw_autotune_batch(I32(len(ns)), _ptr(eps_cat), _vp(eps_off), _vp(ns), I32(lattice),
                                  _vp(walks), _vp(out_off), _ptr(hits), _ptr(steps),
                                  ctypes.byref(best), _stream(stream)))
    return {k: int(getattr(best, k)) for k, _ in mw_tune._fields_}


def mw_tune_lookup(n_cells, walks, lattice=MW_LATTICE_VERTEX):
    """The tuned setting a batch of this shape would use, or None."""
    ns = np.ascontiguousarray(n_cells, dtype=np.int32)
    w = np.ascontiguousarray(walks, dtype=np.uint64)
    t = mw_tune()
    found = ctypes.c_int32(0)
    _check(_lib.mw_tune_lookup(I32(len(ns)), _vp(ns), _vp(w), I32(lattice), ctypes.byref(t), ctypes.byref(found)))
    return {k: int(getattr(t, k)) for k, _ in mw_tune._fields_} if found.value else None


class BatchPlan:
    """mw_batch_plan_*: a batch captured as a HIP graph, replayed per seed."""

    def __init__(self, eps_list, walks, lattice=MW_LATTICE_VERTEX, tune=None, device="cuda",
                 packed=None, want_steps=True):
        import torch
        self.eps_cat, ns, eps_off, walks, self.out_off = _batch_arrays(eps_list, walks, device, packed)
        total = int(walks.sum())
        self.hits = torch.empty(max(total, 1), dtype=torch.int32, device=self.eps_cat.device)
        self.steps = (torch.empty(max(total, 1), dtype=torch.int32, device=self.eps_cat.device)
                      if want_steps else None)
        self.total = total
        t = None
        if tune is not None:
            t = mw_tune(*[int(tune.get(k, 0)) for k, _ in mw_tune._fields_])
        h = ctypes.c_void_p()
        _check(_lib.mw_batch_plan_create(I32(len(ns)), _ptr(self.eps_cat), _vp(eps_off), _vp(ns),
                                         I32(lattice), _vp(walks), _vp(self.out_off), _ptr(self.hits),
                                         _ptr(self.steps), ctypes.byref(t) if t is not None else None,
                                         ctypes.byref(h)))
        self.handle = h

    def run(self, seed, stream=None):
        _check(_lib.mw_batch_plan_run(self.handle, U64(seed), _stream(stream)))
        return self.hits[:self.total], (self.steps[:self.total] if self.steps is not None else None)

    def close(self):
        if self.handle:
            _check(_lib.mw_batch_plan_destroy(self.handle))
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def mw_batch_plan_create(eps_list, walks, **kw):
    return BatchPlan(eps_list, walks, **kw)


def mw_batch_plan_run(plan, seed, stream=None):
    return plan.run(seed, stream)


def mw_batch_plan_destroy(plan):
    plan.close()


# ---------------------------------------------------------------------------
# Geometry and FRW extraction (Alg. 1)
# ---------------------------------------------------------------------------
F3 = ctypes.c_float * 3


class mw_cond_box(ctypes.Structure):
    _fields_ = [("lo", F3), ("hi", F3), ("net", ctypes.c_int32)]


class mw_diel_box(ctypes.Structure):
    _fields_ = [("lo", F3), ("hi", F3), ("eps", ctypes.c_float)]


class mw_structure_desc(ctypes.Structure):
    _fields_ = [("n_cond", ctypes.c_int32), ("cond", ctypes.POINTER(mw_cond_box)),
                ("n_nets", ctypes.c_int32), ("n_diel", ctypes.c_int32),
                ("diel", ctypes.POINTER(mw_diel_box)), ("n_layers", ctypes.c_int32),
                ("layer_z0", ctypes.POINTER(ctypes.c_float)),
                ("layer_eps", ctypes.POINTER(ctypes.c_float)), ("win_lo", F3), ("win_hi", F3),
                ("bc", ctypes.c_uint8 * 6)]


class frw_options(ctypes.Structure):
    _fields_ = [("n_cells", ctypes.c_int32), ("hybrid", ctypes.c_int32),
                ("expand", ctypes.c_int32), ("plain", ctypes.c_int32),
                ("target_rel_3sigma", ctypes.c_double), ("abs_tol_rel", ctypes.c_double),
                ("first_walk", ctypes.c_uint64), ("batch_walks", ctypes.c_uint64),
                ("gauss_is", ctypes.c_double), ("lattice", ctypes.c_int32)]


class frw_stats(ctypes.Structure):
    _fields_ = [("walks", ctypes.c_uint64), ("hops", ctypes.c_uint64),
                ("micro_steps", ctypes.c_uint64), ("hop_class", ctypes.c_uint64 * 3),
                ("first_branch", ctypes.c_uint64 * 4), ("cache_miss", ctypes.c_uint64),
                ("env_absorbed", ctypes.c_uint64), ("hop_cap", ctypes.c_uint64),
                ("launches", ctypes.c_uint64), ("seconds", ctypes.c_double),
                ("walker_seconds", ctypes.c_double), ("gauss_g", ctypes.c_double),
                ("gauss_area", ctypes.c_double), ("gauss_faces", ctypes.c_uint64),
                ("cube_halved", ctypes.c_uint64), ("walks_launched", ctypes.c_uint64)]

    def as_dict(self):
        return {"walks": self.walks, "hops": self.hops, "micro_steps": self.micro_steps,
                "hop_class": list(self.hop_class), "first_branch": list(self.first_branch),
                "cache_miss": self.cache_miss, "env_absorbed": self.env_absorbed,
                "hop_cap": self.hop_cap, "launches": self.launches, "seconds": self.seconds,
                "walker_seconds": self.walker_seconds, "gauss_g": self.gauss_g,
                "gauss_area": self.gauss_area, "gauss_faces": self.gauss_faces,
                "cube_halved": self.cube_halved, "walks_launched": self.walks_launched}


def make_desc(st):
    """mw_structure_desc for a structure object with the fields of
    workloads.Structure (cond (n,6), cond_net, n_nets, diel (m,6), diel_eps,
    layer_z0, layer_eps, win_lo, win_hi, bc).  Returns (desc, keepalive)."""
    nc, nd = int(st.cond.shape[0]), int(st.diel.shape[0])
    cond = (mw_cond_box * max(nc, 1))()
    for i in range(nc):
        b = st.cond[i]
        cond[i] = mw_cond_box(F3(*b[:3]), F3(*b[3:]), int(st.cond_net[i]))
    diel = (mw_diel_box * max(nd, 1))()
    for i in range(nd):
        b = st.diel[i]
        diel[i] = mw_diel_box(F3(*b[:3]), F3(*b[3:]), float(st.diel_eps[i]))
    nl = len(st.layer_z0)
    z0 = (ctypes.c_float * nl)(*[float(x) for x in st.layer_z0])
    le = (ctypes.c_float * nl)(*[float(x) for x in st.layer_eps])
    d = mw_structure_desc(nc, cond, int(st.n_nets), nd, diel, nl, z0, le,
                          F3(*[float(x) for x in st.win_lo]), F3(*[float(x) for x in st.win_hi]),
                          (ctypes.c_uint8 * 6)(*[int(b) for b in st.bc]))
    return d, (cond, diel, z0, le)


class StructureHandle:
    """Owns an mw_structure (device-resident geometry and its grid index)."""

    def __init__(self, st):
        desc, keep = make_desc(st)
        h = ctypes.c_void_p()
        _check(_lib.mw_structure_create(ctypes.byref(desc), ctypes.byref(h)))
        self.handle = h
        self.n_nets = int(st.n_nets)

    def close(self):
        if self.handle:
            _lib.mw_structure_destroy(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def mw_structure_create(st):
    return StructureHandle(st)


def mw_structure_destroy(handle):
    handle.close()


def frw_extract(structure, master, walk_budget, seed=0, n_cells=16, hybrid=1,
                target_rel_3sigma=0.0, abs_tol_rel=1e-6, first_walk=0, batch_walks=0,
                scores=False, device="cuda", expand=0, plain=0, gauss_is=0.0, lattice=MW_LATTICE_VERTEX):
    """Alg. 1: one capacitance row (fF, last entry = grounded enclosure) and
    its standard errors.  With scores=True also returns the per-walk net and
    fp32 weight (CUDA tensors).  lattice=MW_LATTICE_CELL: cubes on the
    cell-centred lattice (odd n_cells)."""
    import torch
    if not isinstance(structure, StructureHandle):
        structure = StructureHandle(structure)
    K = structure.n_nets + 1
    row = (ctypes.c_double * K)()
    se = (ctypes.c_double * K)()
    stats = frw_stats()
    opt = frw_options(n_cells, hybrid, expand, plain, target_rel_3sigma, abs_tol_rel, first_walk,
                      batch_walks, gauss_is, lattice)
    net = w = None
    if scores:
        net = torch.empty(walk_budget, dtype=torch.int32, device=device)
        w = torch.empty(walk_budget, dtype=torch.float32, device=device)
        torch.cuda.synchronize()
    _check(_lib.frw_extract(structure.handle, I32(master), U64(walk_budget), U64(seed),
                            ctypes.byref(opt), row, se, ctypes.byref(stats), _ptr(net), _ptr(w)))
    out = {"row": np.array(row[:]), "se": np.array(se[:]), "stats": stats.as_dict()}
    if scores:
        n = stats.walks
        out["net"], out["w"] = net[:n], w[:n]
    return out



def frw_autotune(structure, master, walks, seed=0, n_cells=16, hybrid=1, expand=0, lattice=MW_LATTICE_VERTEX):
    """Tunes the FRW walker's resident waves per CU on this extraction and
    keeps the choice (returned) for later calls with the same lattice."""
    if not isinstance(structure, StructureHandle):
        structure = StructureHandle(structure)
    opt = frw_options(n_cells, hybrid, expand, 0, 0.0, 1e-6, 0, 0, 0.0, lattice)
    w = ctypes.c_int32(0)
    _check(_lib.frw_autotune(structure.handle, I32(master), U64(walks), U64(seed), ctypes.byref(opt),
                             ctypes.byref(w)))
    return int(w.value)


def mw_table_cache_clear(n_cells):
    """Empties the device's transition-table cache of this lattice size."""
    _check(_lib.mw_table_cache_clear(I32(n_cells)))


def mw_sgf_table(plane_codes, axis, kind=0, normal_axis=0, lattice=MW_LATTICE_VERTEX):
    """One transition table of the device cache (built if missing): the
    stratified cube's plane codes along `axis`; kind 0 hop table, kind 1
    first-transition table for `normal_axis`.  Returns {"cdf": uint32[6 M^2],
    "sign": bool[6 M^2] (kind 1), "kh": float (kind 1)}.  With
    lattice=MW_LATTICE_CELL the planes are given by their permittivities
    (odd count) and M = n."""
    if lattice == MW_LATTICE_CELL:
        codes = np.ascontiguousarray(np.asarray(plane_codes, dtype=np.float32).view(np.uint32))
    else:
        codes = np.ascontiguousarray(plane_codes, dtype=np.uint32)
    n = int(codes.size)
    nb = 6 * (n - 1) ** 2 if lattice == MW_LATTICE_VERTEX else 6 * n * n
    cdf = np.zeros(nb, dtype=np.uint32)
    bits = np.zeros((nb + 31) // 32, dtype=np.uint32)
    kh = ctypes.c_float(0)
    _check(_lib.mw_sgf_table(I32(n), I32(kind), I32(axis), I32(normal_axis), _vp(codes), _vp(cdf),
                             _vp(bits), ctypes.byref(kh)))
    sign = ((bits[np.arange(nb) >> 5] >> (np.arange(nb) & 31).astype(np.uint32)) & 1).astype(bool)
    return {"cdf": cdf, "sign": sign, "kh": float(kh.value)}


def frw_extract_matrix(structure, walks_per_master, seed=0, masters=None, n_cells=16, hybrid=1,
                       target_rel_3sigma=0.0, abs_tol_rel=1e-6, first_walk=0, batch_walks=0, expand=0,
                       plain=0, gauss_is=0.0, lattice=MW_LATTICE_VERTEX):
    """Capacitance-matrix rows for several masters (default: every net) in
    shared rounds.  Returns {"cap": (M, K) rows, "se": (M, K), "sym": (M, M)
    symmetrised block, "masters": list, "stats": dict}; master i uses seed + i."""
    if not isinstance(structure, StructureHandle):
        structure = StructureHandle(structure)
    K = structure.n_nets + 1
    if masters is None:
        masters = list(range(structure.n_nets))
    m = np.ascontiguousarray(masters, dtype=np.int32)
    M = int(m.size)
    cap = np.zeros((M, K))
    se = np.zeros((M, K))
    sym = np.zeros((M, M))
    stats = frw_stats()
    opt = frw_options(n_cells, hybrid, expand, plain, target_rel_3sigma, abs_tol_rel, first_walk, batch_walks,
                      gauss_is, lattice)
    _check(_lib.frw_extract_matrix(structure.handle, I32(M), _vp(m), U64(walks_per_master), U64(seed),
                                   ctypes.byref(opt), _vp(cap), _vp(se), _vp(sym), ctypes.byref(stats)))
    return {"cap": cap, "se": se, "sym": sym, "masters": [int(x) for x in m], "stats": stats.as_dict()}


# ---------------------------------------------------------------------------
# Serving (continuous batching)
# ---------------------------------------------------------------------------
class mw_server_stats(ctypes.Structure):
    _fields_ = [(k, ctypes.c_uint64) for k in ("submitted", "completed", "failed", "rounds", "walks",
                                                "resident_bytes", "max_resident_bytes",
                                                "max_concurrent")]

    def as_dict(self):
        return {k: int(getattr(self, k)) for k, _ in self._fields_}


_lib.mw_server_create.argtypes = [ctypes.c_size_t, ctypes.c_void_p, ctypes.c_void_p]
_lib.mw_server_submit.argtypes = [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_int32, ctypes.c_uint64,
                                  ctypes.c_uint64, ctypes.c_void_p]
_lib.mw_server_poll.argtypes = [ctypes.c_void_p, ctypes.c_uint64, ctypes.c_void_p, ctypes.c_void_p,
                                ctypes.c_void_p, ctypes.c_void_p]
_lib.mw_server_get_stats.argtypes = [ctypes.c_void_p, ctypes.c_void_p]
_lib.mw_server_destroy.argtypes = [ctypes.c_void_p]


class Server:
    """Request loop over the device (mw_server_*): submit structures, poll rows."""

    def __init__(self, hbm_budget_bytes, n_cells=16, hybrid=1, target_rel_3sigma=0.0,
                 abs_tol_rel=1e-6, expand=0, plain=0, gauss_is=0.0, lattice=MW_LATTICE_VERTEX):
        opt = frw_options(n_cells, hybrid, expand, plain, target_rel_3sigma, abs_tol_rel, 0, 0, gauss_is,
                          lattice)
        h = ctypes.c_void_p()
        _check(_lib.mw_server_create(ctypes.c_size_t(int(hbm_budget_bytes)), ctypes.byref(opt),
                                     ctypes.byref(h)))
        self.handle = h
        self._nets = {}

    def submit(self, st, master, walk_budget, seed=0):
        desc, keep = make_desc(st)
        t = ctypes.c_uint64()
        _check(_lib.mw_server_submit(self.handle, ctypes.byref(desc), master, walk_budget, seed,
                                     ctypes.byref(t)))
        self._nets[t.value] = int(st.n_nets)
        return t.value

    def poll(self, ticket):
        """None while running; else dict(row, se, latency, walks)."""
        K = self._nets[ticket] + 1
        row = (ctypes.c_double * K)()
        se = (ctypes.c_double * K)()
        stats = frw_stats()
        lat = ctypes.c_double()
        rc = _lib.mw_server_poll(self.handle, ticket, row, se, ctypes.byref(stats), ctypes.byref(lat))
        if rc == MW_ENOTREADY:
            return None
        _check(rc)
        return {"row": np.array(row[:]), "se": np.array(se[:]), "latency": lat.value,
                "walks": stats.walks}

    def wait(self, ticket, timeout=600.0, interval=0.0005):
        import time
        t0 = time.time()
        while True:
            r = self.poll(ticket)
            if r is not None:
                return r
            if time.time() - t0 > timeout:
                raise TimeoutError("request %d not done" % ticket)
            time.sleep(interval)

    def stats(self):
        s = mw_server_stats()
        _check(_lib.mw_server_get_stats(self.handle, ctypes.byref(s)))
        return s.as_dict()

    def close(self):
        if self.handle:
            _check(_lib.mw_server_destroy(self.handle))
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def mw_server_create(hbm_budget_bytes, **options):
    return Server(hbm_budget_bytes, **options)


def mw_server_submit(server, st, master, walk_budget, seed=0):
    return server.submit(st, master, walk_budget, seed)


def mw_server_poll(server, ticket):
    return server.poll(ticket)


def mw_server_get_stats(server):
    return server.stats()


def mw_server_destroy(server):
    server.close()


EXPORTS = ("mw_last_error", "mw_init", "mw_transition", "mw_transition_batch",
           "mw_structure_create", "mw_structure_destroy", "frw_extract")
