// frw.hip — Alg. 1 (FRW capacitance extraction) on the GPU: geometry store,
// lazily voxelised transition cubes, the hybrid transition strategy of
// Sec. III-C (exact SGF tables for stratified cubes, MicroWalk (Alg. 3) for
// the rest), the first transition, MicroWalk-E (expanded cubes that may hold
// conductors, Sec. III-B), the score reductions, capacitance-matrix rows and
// the serving loop.
//
// First transitions run in their own kernel, one lane per walk.  The walker
// kernel then takes walks in wave-sized chunks; every lane owns one walk at
// a time.  A lane's transition cube is never materialised: the lane keeps in
// LDS, per axis, a bitmask per cell index of the dielectric boxes (priority
// order, at most 16) whose interval holds that cell's centre, the boxes'
// codes, and the background layer code of each z cell.  A cell's code is the
// code of the highest set bit of the AND of its three masks, else its z
// cell's background code; a MicroWalk step derives the six link codes of its
// node from the eight cells around it and reads the two masks of the moved
// axis when it moves.  Lanes of a wave that need MicroWalk step together
// while at least half of the working lanes do; the others take their next
// hop meanwhile.
//
// Cubes of an odd lattice size n use the cell-centred lattice of Sec. III-A
// (nodes at the voxel centres, Eq. (6) coefficients from the cells'
// permittivities, exits at panel centres) with the same cube description;
// even n use the vertex lattice described above.
//
// Stratified cubes (every region present in the cube spans whole planes
// normal to one axis) are sampled from cached exact SGF tables of the same
// lattice.  A missing table parks the walk in a queue; the table is built by
// build_tables_kernel between walker launches, and parked walks resume from
// their saved position (their random numbers depend only on walk id and hop
// index, so parking does not change any result).
#include <algorithm>
#include <atomic>
#include <chrono>
#include <cstring>
#include <cmath>
#include <map>
#include <memory>
#include <mutex>
#include <tuple>
#include <vector>

#include "common.h"

namespace mw {
namespace {

constexpr float EPS0 = 8.8541878128e-3f;  // vacuum permittivity, fF/um
constexpr uint32_t HOP_CAP = 100000;
constexpr int MAX_REGIONS = MW_MAX_REGIONS;
constexpr int FRW_THREADS = 256;   // first-transition kernel
constexpr int WALK_THREADS = 64;   // walker kernel: one-wave blocks pack the LDS of a CU
constexpr uint32_t KEY_HDR = 4;
constexpr uint32_t NO_INDEX = 0xffffffffu;
constexpr uint32_t FULL_INDEX = 0xfffffffeu;  // slot of a key that found the table cache full

enum ErrBits : uint32_t { ERR_REGIONS = 1, ERR_TABLE_CAP = 2, ERR_PARK_CAP = 4, ERR_STEP_CAP = 8 };
constexpr uint32_t MW_STEP_CAP = 1u << 26;
// MicroWalk-E: expanded cubes reach at most EXP_LIST_FACTOR times the
// conductor-free half-size and hold at most EXP_MAX_COND conductors.
constexpr float EXP_LIST_FACTOR = 4.f;
constexpr int EXP_MAX_COND = 7;

// -------------------------------------------------------------------------
// Device structure descriptor.
// -------------------------------------------------------------------------
struct StructDev {
    int32_t n_cond, n_nets, n_diel, n_layers;
    const float4* cond_lo;  // xyz lo, w = net (bits)
    const float4* cond_hi;
    const float4* diel_lo;  // xyz lo, w = eps
    const float4* diel_hi;  // xyz hi, w = vertex cell code (bits)
    const float* layer_z0;
    const uint32_t* layer_code;
    const uint32_t* layer_eps;  // layer permittivities as float bits (cell lattice)
    float wlo[3], whi[3];
    int32_t bc[6];
    // uniform grid
    int32_t gdim[3];
    float gorg[3], ginv[3], gcell[3];
    const uint32_t* gc_off;
    const uint32_t* gc_list;
    const uint32_t* gd_off;
    const uint32_t* gd_list;
    // candidates of expanded (MicroWalk-E) cubes: conductors and dielectric
    // boxes within EXP_LIST_FACTOR times the cell's conductor-free distance
    const uint32_t* ge_off;
    const uint32_t* ge_list;
    const uint32_t* gx_off;
    const uint32_t* gx_list;
    // the boxes of gc_list, gd_list, ge_list and gx_list in place (lo, hi
    // per entry): one load per candidate instead of an index and then the box
    const float4* gc_rec;
    const float4* gd_rec;
    const float4* ge_rec;
    const float4* gx_rec;
    float delta_abs;
};

// One rectangle of a Gaussian surface, or one importance-sampling patch of
// it: p = {plane, cumulative sampling weight, axis | side << 2 (bits), weight
// factor}, t = {lo, hi} along the lower tangent axis, then {lo, hi} along the
// higher one.  Uniform sampling: the weight is the area and the factor |G|;
// importance sampling: the weight is q = area K(centre) and the factor
// Q area / q.
struct GaussFace {
    float4 p, t;
};

struct GaussDev {
    float g, area;  // area: the total sampling weight (|G| or Q)
    int32_t n_faces, pad;
    const GaussFace* faces;
};

// Table cache for one lattice size.
struct CacheDev {
    unsigned long long* slot;  // (hash32 << 32) | table index; 0 = empty
    uint32_t* ready;
    uint32_t* keys;
    uint32_t* data;
    uint32_t* n_tables;
    uint32_t* pending;
    uint32_t* n_pending;
    uint32_t slot_mask, capacity, key_words, tab_words, n, nb;
    uint32_t key_stride;  // key_words rounded up to whole 16-byte rows (zero padded)
};

struct Parked {
    unsigned long long walk;
    float px, py, pz, omega;
    uint32_t t;
    int32_t seg;
};
static_assert(sizeof(Parked) == 32, "Parked moves as two 16-byte vectors");

struct Counters {
    unsigned long long hops, micro_steps, hop_class[3], first_branch[4], env, hop_cap;
    uint32_t err, park_count, first_missing, pad;
    unsigned long long resume_next, walk_next;
    // transitions whose cube the capacity rule made smaller than the
    // conductor-free (or expanded) size
    unsigned long long halved;
    // the parked walks the next walker launch resumes, from park[resume_side]
    uint32_t resume_count, resume_side;
    // device-driven rounds: tables they built, 1 once they handed over to
    // the host, 1 when their first-transition launch has walks to redo
    uint32_t tables_built, dev_stop, need_first;
    // set between launches: the next walker launch has no walk to resume
    // and no fresh walk left (every block of it ends at once)
    uint32_t launch_idle;
};

// A contiguous range of walks of one extraction request.  One launch of the
// first-transition or walker kernel serves a list of segments (one for
// frw_extract, several requests for the server); the walks of the list are
// numbered 0..total-1 in segment order.
struct Segment {
    const StructDev* S;
    const GaussDev* G;
    unsigned long long walk_begin;  // walk id of the segment's first walk
    unsigned long long offset;      // list index of the segment's first walk
    unsigned long long count;
    int32_t* score_net;             // indexed by walk - walk_begin
    float* score_w;
    float4* first_state;
    uint32_t* first_done;
    uint32_t k0, k1;                // Philox key (seed)
};

__device__ __forceinline__ int find_segment(const Segment* segs, int n_segs, unsigned long long g) {
    int lo = 0, hi = n_segs - 1;
    while (lo < hi) {
        const int mid = (lo + hi + 1) >> 1;
        if (segs[mid].offset <= g)
            lo = mid;
        else
            hi = mid - 1;
    }
    return lo;
}

struct WalkArgs {
    const Segment* segs;
    int32_t n_segs, pad0;
    unsigned long long total;
    CacheDev cache;
    int32_t n, hybrid;
    Parked* park[2];        // parked-walk queues: resume from park[resume_side], park to the other
    uint32_t park_cap;
    Counters* ctr;
    uint32_t lane_stride;   // dwords of LDS per lane (odd)
    uint32_t uniform_index; // table of the uniform cube
    int32_t expand_m;       // MicroWalk-E: expanded half-size n d / (2 m) (EXP kernels)
    int32_t plain;          // 1: every walk makes one transition per launch, then parks
    // single-segment launches: a copy of the structure header, read through
    // the kernel-argument segment (uniform scalar loads) instead of memory
    // that the kernel also writes
    StructDev S0;
};

// First transitions of a batch of walks (one lane per walk).
struct FirstArgs {
    const Segment* segs;
    const float4* eval;  // non-null: evaluate K / h at these points (xyz, w = axis | side << 2 bits)
    int32_t n_segs, pad0;
    unsigned long long total;
    CacheDev cache;
    int32_t n;
    Counters* ctr;
    uint32_t lane_stride;
    int32_t round;  // 0: every walk is processed and its done flag written
    int32_t dev_round;  // 1: a device-driven round (runs only when the counters ask for it)
    StructDev S0;  // single-segment launches: the structure header (kernel arguments)
};

// The walker reads device-struct data through global views (gp/gpw).
using SRef = const GAS StructDev&;
__device__ __forceinline__ float4 ldf4(const float4* p) {
    const gvec4 v = *(const GAS gvec4*)p;
    return make_float4(v.x, v.y, v.z, v.w);
}
// Candidate records rec[2 q] (lo), rec[2 q + 1] (hi) for q in [b, e), handed
// to f in list order; the loads of CAND_BATCH records are issued together (a
// batch running past e repeats the last record, which f does not see).  f
// returns false to stop.
constexpr int CAND_BATCH = 4;
template <class F>
__device__ __forceinline__ void for_each_record(const float4* rec, uint32_t b, uint32_t e, F&& f) {
    for (uint32_t q0 = b; q0 < e; q0 += CAND_BATCH) {
        float4 lo[CAND_BATCH], hi[CAND_BATCH];
#pragma unroll
        for (int j = 0; j < CAND_BATCH; ++j) {
            const uint32_t q = min(q0 + (uint32_t)j, e - 1);
            lo[j] = ldf4(rec + 2 * (size_t)q);
            hi[j] = ldf4(rec + 2 * (size_t)q + 1);
        }
        bool go = true;
#pragma unroll
        for (int j = 0; j < CAND_BATCH; ++j)
            if (go && q0 + (uint32_t)j < e) go = f(lo[j], hi[j]);
        if (!go) return;
    }
}
// The same over the entries b + i of a list for the set bits i of mask (list
// order).
template <class F>
__device__ __forceinline__ void for_each_marked(const float4* rec, uint32_t b, unsigned long long mask, F&& f) {
    while (mask) {
        uint32_t q[CAND_BATCH];
        bool v[CAND_BATCH];
#pragma unroll
        for (int j = 0; j < CAND_BATCH; ++j) {
            v[j] = mask != 0ull;
            q[j] = v[j] ? b + (uint32_t)__builtin_ctzll(mask) : b;
            mask &= mask - 1ull;
        }
        float4 lo[CAND_BATCH], hi[CAND_BATCH];
#pragma unroll
        for (int j = 0; j < CAND_BATCH; ++j) {
            const uint32_t qq = v[j] ? q[j] : q[0];
            lo[j] = ldf4(rec + 2 * (size_t)qq);
            hi[j] = ldf4(rec + 2 * (size_t)qq + 1);
        }
        bool go = true;
#pragma unroll
        for (int j = 0; j < CAND_BATCH; ++j)
            if (go && v[j]) go = f(lo[j], hi[j]);
        if (!go) return;
    }
}
__device__ __forceinline__ Parked ldpark(const Parked* p) {
    const GAS guvec4* q = (const GAS guvec4*)p;
    const guvec4 a = q[0], b = q[1];
    Parked r;
    __builtin_memcpy(&r, &a, 16);
    __builtin_memcpy(reinterpret_cast<char*>(&r) + 16, &b, 16);
    return r;
}
__device__ __forceinline__ void stpark(Parked* p, const Parked& v) {
    guvec4 a, b;
    __builtin_memcpy(&a, &v, 16);
    __builtin_memcpy(&b, reinterpret_cast<const char*>(&v) + 16, 16);
    GAS guvec4* q = (GAS guvec4*)p;
    q[0] = a;
    q[1] = b;
}
__device__ __forceinline__ void stf4(float4* p, float4 v) {
    gvec4 w;
    w.x = v.x;
    w.y = v.y;
    w.z = v.z;
    w.w = v.w;
    *(GAS gvec4*)p = w;
}

// -------------------------------------------------------------------------
// Geometry helpers.
// -------------------------------------------------------------------------
__device__ __forceinline__ float box_dist(float4 lo, float4 hi, float3 p) {
    const float dx = fmaxf(fmaxf(lo.x - p.x, p.x - hi.x), 0.f);
    const float dy = fmaxf(fmaxf(lo.y - p.y, p.y - hi.y), 0.f);
    const float dz = fmaxf(fmaxf(lo.z - p.z, p.z - hi.z), 0.f);
    return fmaxf(dx, fmaxf(dy, dz));
}

__device__ __forceinline__ float axis_of(float3 p, int a) { return a == 0 ? p.x : (a == 1 ? p.y : p.z); }

template <class SR>
__device__ __forceinline__ int grid_cell(SR& S, float3 p) {
    int c[3];
#pragma unroll
    for (int a = 0; a < 3; ++a) {
        int v = (int)floorf((axis_of(p, a) - S.gorg[a]) * S.ginv[a]);
        c[a] = min(max(v, 0), S.gdim[a] - 1);
    }
    return (c[2] * S.gdim[1] + c[1]) * S.gdim[0] + c[0];
}

// Largest conductor-free cube: L-infinity distance to the nearest conductor
// or grounded window face; nearest = net, or n_nets for a grounded face.
template <class SR>
__device__ __forceinline__ float query_dist(SR& S, float3 p, int cell, int* nearest) {
    float best = INFINITY;
    int who = S.n_nets;
    const uint32_t b = gp(S.gc_off)[cell], e = gp(S.gc_off)[cell + 1];
    for_each_record(S.gc_rec, b, e, [&](const float4& lo, const float4& hi) {
        const float d = box_dist(lo, hi, p);
        if (d < best) {
            best = d;
            who = __float_as_int(lo.w);
        }
        return true;
    });
#pragma unroll
    for (int a = 0; a < 3; ++a) {
        const float x = axis_of(p, a);
        if (S.bc[2 * a] == MW_BC_DIRICHLET && x - S.wlo[a] < best) {
            best = x - S.wlo[a];
            who = S.n_nets;
        }
        if (S.bc[2 * a + 1] == MW_BC_DIRICHLET && S.whi[a] - x < best) {
            best = S.whi[a] - x;
            who = S.n_nets;
        }
    }
    *nearest = who;
    return best;
}

template <class SR>
__device__ __forceinline__ float fold(SR& S, int a, float x) {
    if (S.bc[2 * a] == MW_BC_NEUMANN && x < S.wlo[a]) x = 2.f * S.wlo[a] - x;
    if (S.bc[2 * a + 1] == MW_BC_NEUMANN && x > S.whi[a]) x = 2.f * S.whi[a] - x;
    return x;
}

template <class SR>
__device__ __forceinline__ float3 fold3(SR& S, float3 p) {
    return make_float3(fold(S, 0, p.x), fold(S, 1, p.y), fold(S, 2, p.z));
}

// -------------------------------------------------------------------------
// Per-lane cube description in LDS: masks[3][n] (u16, dielectric boxes),
// box codes[16] (u32, box bit b at codes[15 - b]), background codes bz[n]
// (u32, per z cell) directly after them.  The pointers carry the LDS address
// space, so that functions the compiler does not inline still use LDS
// instructions on them.
// -------------------------------------------------------------------------
#define LAS __attribute__((address_space(3)))
struct LaneCube {
    LAS uint16_t* mask;   // mask[a * n + i]: bit b = box b's interval holds cell i's centre
    LAS uint32_t* codes;  // codes[15 - b]: code of box bit b
    LAS uint32_t* bz;     // background (layer) code of z cell k (= codes + 16)
};

__device__ __forceinline__ LaneCube lane_cube(uint32_t* my, int n) {
    LAS uint32_t* m = (LAS uint32_t*)my;
    LaneCube L;
    L.mask = reinterpret_cast<LAS uint16_t*>(m);
    L.codes = m + ((3 * n + 1) / 2);
    L.bz = L.codes + MAX_REGIONS;
    return L;
}

__device__ __forceinline__ int hb16(uint32_t m) { return 31 - __clz(m | 1u); }

// Code of a cell with box-membership m and background code b.  The read is
// unconditional (bit 0's slot when m = 0) so that no branch splits the eight
// reads of a step.
__device__ __forceinline__ uint32_t cell_code(LaneCube L, uint32_t m, uint32_t b) {
    const uint32_t v = L.codes[MAX_REGIONS - 1 - hb16(m)];
    return m ? v : b;
}

// MicroWalk-E additions to a lane's LDS, after the LaneCube arrays:
// nmask[a * (n + 1) + i]: bit b < EXP_MAX_COND: conductor bit b (closed box)
// holds coordinate i of axis a; bit 7: coordinate i of axis a lies at or
// beyond a grounded window face.  cnet[b]: net of conductor bit b.
// theta[(b * 3 + a) * 2 + side] / 65535: fraction of the link from the free
// node next to object b (b = 7: the grounded faces) along axis a at which it
// enters the object — side 0 through the object's low face (a +a move),
// side 1 through its high face (a -a move).
struct LaneExp {
    LAS uint8_t* nmask;
    LAS uint16_t* cnet;
    LAS uint16_t* theta;
};

__device__ __forceinline__ int lane_base_words(int n) { return (3 * n + 1) / 2 + MAX_REGIONS + n; }
__host__ __device__ __forceinline__ int lane_exp_words(int n) { return (3 * (n + 1) + 3) / 4 + 4 + 24; }

__device__ __forceinline__ LaneExp lane_exp(uint32_t* my, int n) {
    LaneExp E;
    LAS uint32_t* q = (LAS uint32_t*)my + lane_base_words(n);
    E.nmask = reinterpret_cast<LAS uint8_t*>(q);
    q += (3 * (n + 1) + 3) / 4;
    E.cnet = reinterpret_cast<LAS uint16_t*>(q);
    E.theta = reinterpret_cast<LAS uint16_t*>(q + 4);
    return E;
}

__device__ __forceinline__ uint16_t theta_q(float th) {
    return (uint16_t)fminf(65535.f, fmaxf(4096.f, rintf(th * 65535.f)));  // theta >= 1/16
}

// Bit toggles of 16-bit and 8-bit LDS entries (dword-aligned arrays) as LDS
// atomics on the containing dword: they return nothing, so a run of toggles
// issues without waiting for read-modify-write round trips.
__device__ __forceinline__ void lds_xor(LAS uint32_t* p, uint32_t v) {
    __hip_atomic_fetch_xor(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
}
__device__ __forceinline__ void toggle16(LAS uint16_t* base, int k, uint32_t bits) {
    lds_xor(reinterpret_cast<LAS uint32_t*>(base) + (k >> 1), bits << (16 * (k & 1)));
}
__device__ __forceinline__ void toggle8(LAS uint8_t* base, int k, uint32_t bits) {
    lds_xor(reinterpret_cast<LAS uint32_t*>(base) + (k >> 2), bits << (8 * (k & 3)));
}

struct CubeInfo {
    uint32_t present, A[3];
    int n_layers;  // background layers holding at least one cell centre
    int cls;       // 0 uniform, 1 stratified, 2 other
    int axis;      // stratification axis
    bool overflow;
};

constexpr int LAYER_LDS = 8;  // stacks of up to this many layers: a copy in LDS

// Background layer of every z cell of a cube: layer(k) = #{q >= 1 : z_k >=
// z0[q]} for the cell centre z_k (z0 ascending), walking the boundaries once
// since the centres rise with k.  Z and C index z0 and the layer codes (global
// memory, or a copy in LDS).
template <class Z, class C>
__device__ __forceinline__ void layer_walk(Z z0, C lcode, int nl, float zlo, float h, int n, LaneCube L, int* lmin,
                                           int* lmax) {
    // layers of the lowest and the highest centre
    int l = 0;
    while (l + 1 < nl && zlo + 0.5f * h >= z0[l + 1]) ++l;
    int lt = l;
    while (lt + 1 < nl && zlo + ((float)(n - 1) + 0.5f) * h >= z0[lt + 1]) ++lt;
    *lmin = l;
    *lmax = lt;
    uint32_t code = lcode[l];
    LAS uint32_t* bz2 = L.bz;
    if (l == lt) {
        // one layer holds every centre (n is even)
        for (int k = 0; k < n; k += 2) {
            bz2[k] = code;
            bz2[k + 1] = code;
        }
        return;
    }
    // the same count for every lane; a boundary is crossed a few times
    float zb = z0[l + 1];
    for (int k = 0; k < n; ++k) {
        const float z = zlo + ((float)k + 0.5f) * h;
        while (z >= zb) {
            ++l;
            zb = l + 1 < nl ? z0[l + 1] : INFINITY;
            code = lcode[l];
        }
        L.bz[k] = code;
    }
}

// Builds the region description of the cube centred at c with half-size R.
// Regions are the dielectric boxes (bits, priority = list order) and the
// background layers (per-z-cell codes); a region is present when it holds at
// least one cell centre.
// lt: when not null, an LDS copy of the structure's layer boundaries (words
// 0..7, as float bits) and codes (words 8..15), for at most LAYER_LDS layers.
// dr: when not null, the cell's dielectric candidate range (gd_off[cell],
// gd_off[cell + 1]) read ahead by the caller (ordinary cubes only).
// marked: only the list entries b + i for the set bits i of marks are
// visited (the boxes exp_fit found touching this cube).
// CELL: a cube of the cell-centred lattice (n odd): the region codes are the
// permittivities (float bits) and the mask rows lie n + 1 apart, so that
// every axis starts on a dword (the extra row past the last cell repeats the
// last cell's mask and is never read as a cell).
template <bool CELL = false, class SR>
__device__ __forceinline__ CubeInfo build_cube(SR& S, int cell, float3 c, float R, int n, LaneCube L,
                                              bool expanded = false, const uint32_t* lt = nullptr,
                                              const uint2* dr = nullptr, bool marked = false,
                                              unsigned long long marks = 0ull) {
    CubeInfo info{};
    const int ns = CELL ? n + 1 : n;  // mask row stride (even)
    const float h = 2.f * R / (float)n;
    const float lo0[3] = {c.x - R, c.y - R, c.z - R};
    LAS uint32_t* mask32 = reinterpret_cast<LAS uint32_t*>(L.mask);  // 3 ns is even
    for (int q = 0; q < 3 * ns / 2; ++q) mask32[q] = 0u;
    // background layer of every z cell: layer(k) = #{q >= 1 : z_k >= z0[q]}
    // for the cell centre z_k (layer_z0 ascends)
    int lmin, lmax;
    const GAS float* z0 = gp(S.layer_z0);
    const GAS uint32_t* lcode = gp(CELL ? S.layer_eps : S.layer_code);
    const bool zfold = (S.bc[4] == MW_BC_NEUMANN && lo0[2] < S.wlo[2]) ||
                       (S.bc[5] == MW_BC_NEUMANN && lo0[2] + 2.f * R > S.whi[2]);
    if (!zfold && lt) {
        layer_walk(reinterpret_cast<const float*>(lt), lt + LAYER_LDS, S.n_layers, lo0[2], h, n, L, &lmin, &lmax);
    } else if (!zfold) {
        layer_walk(z0, lcode, S.n_layers, lo0[2], h, n, L, &lmin, &lmax);
    } else {
        lmin = 1 << 30;
        lmax = -1;
        for (int k = 0; k < n; ++k) {
            const float z = fold(S, 2, lo0[2] + ((float)k + 0.5f) * h);
            int l = 0;
            for (int q = 1; q < S.n_layers; ++q)
                if (z >= z0[q]) l = q;
            lmin = min(lmin, l);
            lmax = max(lmax, l);
            L.bz[k] = lcode[l];
        }
    }
    info.n_layers = lmax - lmin + 1;
    // dielectric boxes touching the cube, in priority order
    int nbits = 0;
    const uint32_t* doff = expanded ? S.gx_off : S.gd_off;
    const uint32_t b = dr ? dr->x : gp(doff)[cell], e = dr ? dr->y : gp(doff)[cell + 1];
    // the cube's extent inside the window along each axis, and whether it
    // crosses a symmetry wall (then cells fold back into the window)
    float clo[3], chi[3];
    bool crosses[3];
#pragma unroll
    for (int a = 0; a < 3; ++a) {
        clo[a] = lo0[a];
        chi[a] = lo0[a] + 2.f * R;
        if (S.bc[2 * a] == MW_BC_NEUMANN) clo[a] = fmaxf(clo[a], S.wlo[a]);
        if (S.bc[2 * a + 1] == MW_BC_NEUMANN) chi[a] = fminf(chi[a], S.whi[a]);
        crosses[a] = (S.bc[2 * a] == MW_BC_NEUMANN && lo0[a] < S.wlo[a]) ||
                     (S.bc[2 * a + 1] == MW_BC_NEUMANN && lo0[a] + 2.f * R > S.whi[a]);
    }
    const float inv_h = (float)n / (2.f * R);
    auto box = [&](const float4& blo, const float4& bhi) {
        const float bl[3] = {blo.x, blo.y, blo.z}, bh[3] = {bhi.x, bhi.y, bhi.z};
        bool touch = true;
#pragma unroll
        for (int a = 0; a < 3; ++a)
            if (!(bl[a] <= chi[a] && bh[a] >= clo[a])) touch = false;
        if (!touch) return true;
        if (nbits >= MAX_REGIONS) {
            info.overflow = true;
            return false;
        }
        const uint16_t bit = (uint16_t)(1u << nbits);
        L.codes[MAX_REGIONS - 1 - nbits] = __float_as_uint(CELL ? blo.w : bhi.w);
        ++nbits;
#pragma unroll
        for (int a = 0; a < 3; ++a) {
            // masks hold toggles here (bit b flips where box b's run of
            // cells starts or ends); the pass below turns them into masks
            if (!crosses[a]) {
                // cells whose centre lo0 + (i + 1/2) h lies in [bl, bh)
                const float f0 = fminf(fmaxf((bl[a] - lo0[a]) * inv_h - 0.5f, -1.f), (float)n + 1.f);
                const float f1 = fminf(fmaxf((bh[a] - lo0[a]) * inv_h - 0.5f, -1.f), (float)n + 1.f);
                const int i0 = max((int)ceilf(f0), 0), i1 = min((int)ceilf(f1), n);
                if (i0 < i1) {
                    toggle16(L.mask, a * ns + i0, bit);
                    if (i1 < n) toggle16(L.mask, a * ns + i1, bit);
                }
            } else {
                bool prev = false;
                for (int i = 0; i < n; ++i) {
                    const float x = fold(S, a, lo0[a] + ((float)i + 0.5f) * h);
                    const bool in = x >= bl[a] && x < bh[a];
                    if (in != prev) toggle16(L.mask, a * ns + i, bit);
                    prev = in;
                }
            }
        }
        return true;
    };
    if (marked)
        for_each_marked(expanded ? S.gx_rec : S.gd_rec, b, marks, box);
    else
        for_each_record(expanded ? S.gx_rec : S.gd_rec, b, e, box);
    // toggles -> masks (prefix xor along each axis); aggregate masks:
    // present boxes and boxes spanning all cells per axis
    uint32_t O[3];
    // two cells per dword (ns is even, so every axis starts on a dword)
    auto prefix = [&](int a, int i, uint32_t w, uint32_t& m, uint32_t& A, uint32_t& Oa) {
        const uint32_t m0 = m ^ (w & 0xffffu);
        const uint32_t m1 = m0 ^ (w >> 16);
        mask32[a * (ns / 2) + i] = m0 | (m1 << 16);
        A &= m0 & m1;
        Oa |= m0 | m1;
        m = m1;
    };
    if (ns == 16) {
        // all 24 dwords are read before any is written back: one LDS round
        // trip instead of one per dword
        uint32_t w[24];
#pragma unroll
        for (int q = 0; q < 24; ++q) w[q] = mask32[q];
#pragma unroll
        for (int a = 0; a < 3; ++a) {
            uint32_t A = 0xffffu, Oa = 0, m = 0;
#pragma unroll
            for (int i = 0; i < 8; ++i) prefix(a, i, w[a * 8 + i], m, A, Oa);
            info.A[a] = A;
            O[a] = Oa;
        }
    } else {
#pragma unroll
        for (int a = 0; a < 3; ++a) {
            uint32_t A = 0xffffu, Oa = 0, m = 0;
            for (int i = 0; i < ns / 2; ++i) prefix(a, i, mask32[a * (ns / 2) + i], m, A, Oa);
            info.A[a] = A;
            O[a] = Oa;
        }
    }
    info.present = O[0] & O[1] & O[2];
    // layers span every x and y cell; they span every z cell only when a
    // single layer is present
    const bool one_layer = info.n_layers == 1;
    const bool full0 = (info.present & ~info.A[0]) == 0;
    const bool full1 = (info.present & ~info.A[1]) == 0;
    const bool full2 = (info.present & ~info.A[2]) == 0 && one_layer;
    if (full0 && full1 && full2) {
        info.cls = 0;
        info.axis = 2;
    } else if (full0 && full1) {
        info.cls = 1;
        info.axis = 2;
    } else if (full1 && full2) {
        info.cls = 1;
        info.axis = 0;
    } else if (full0 && full2) {
        info.cls = 1;
        info.axis = 1;
    } else {
        info.cls = 2;
        info.axis = -1;
    }
    return info;
}

// Absorbing nodes of an expanded cube centred at c with half-size R (the
// cube never crosses a symmetry wall): grounded faces first, then the
// conductors holding part of the open cube, in candidate-list (index) order.
// False when more than EXP_MAX_COND conductors do.  marked, marks: as for
// build_cube.
template <class SR>
__device__ __forceinline__ bool build_conductors(SR& S, int cell, float3 c, float R, int n, LaneExp E,
                                                 bool marked = false, unsigned long long marks = 0ull) {
    const float h = 2.f * R / (float)n;
    const float o[3] = {c.x - R, c.y - R, c.z - R};
    const int np = n + 1;
    LAS uint32_t* m32 = reinterpret_cast<LAS uint32_t*>(E.nmask);
    for (int q = 0; q < (3 * np + 3) / 4; ++q) m32[q] = 0u;
    // toggles (bit flips where a run of nodes starts or ends), then prefix xor
#pragma unroll
    for (int a = 0; a < 3; ++a) {
        if (S.bc[2 * a] == MW_BC_DIRICHLET && o[a] <= S.wlo[a]) {
            const float u = (S.wlo[a] - o[a]) / h;  // nodes i <= u are at/beyond the face
            const int iw = min((int)floorf(u), n);
            toggle8(E.nmask, a * np, 0x80u);
            if (iw + 1 <= n) toggle8(E.nmask, a * np + iw + 1, 0x80u);
            E.theta[(7 * 3 + a) * 2 + 1] = theta_q((float)(iw + 1) - u);
        }
        if (S.bc[2 * a + 1] == MW_BC_DIRICHLET && o[a] + 2.f * R >= S.whi[a]) {
            const float u = (S.whi[a] - o[a]) / h;  // nodes i >= u
            const int iw = max((int)ceilf(u), 0);
            if (iw <= n) toggle8(E.nmask, a * np + iw, 0x80u);
            E.theta[(7 * 3 + a) * 2 + 0] = theta_q(u - (float)(iw - 1));
        }
    }
    int nb = 0;
    const uint32_t b = gp(S.ge_off)[cell], e = gp(S.ge_off)[cell + 1];
    bool fits = true;
    auto box = [&](const float4& lo4, const float4& hi4) {
        const float bl[3] = {lo4.x, lo4.y, lo4.z}, bh[3] = {hi4.x, hi4.y, hi4.z};
        bool touch = true;
#pragma unroll
        for (int a = 0; a < 3; ++a)
            if (!(bl[a] < o[a] + 2.f * R && bh[a] > o[a])) touch = false;
        if (!touch) return true;
        if (nb >= EXP_MAX_COND) {
            fits = false;
            return false;
        }
        const uint8_t bit = (uint8_t)(1u << nb);
        E.cnet[nb] = (uint16_t)__float_as_int(lo4.w);
#pragma unroll
        for (int a = 0; a < 3; ++a) {
            const float u0 = (bl[a] - o[a]) / h, u1 = (bh[a] - o[a]) / h;
            const int i0 = max((int)ceilf(u0), 0), i1 = min((int)floorf(u1), n);
            if (i0 <= i1) {
                toggle8(E.nmask, a * np + i0, bit);
                if (i1 + 1 <= n) toggle8(E.nmask, a * np + i1 + 1, bit);
            }
            E.theta[(nb * 3 + a) * 2 + 0] = theta_q(u0 - (float)(i0 - 1));
            E.theta[(nb * 3 + a) * 2 + 1] = theta_q((float)(i1 + 1) - u1);
        }
        ++nb;
        return true;
    };
    if (marked)
        for_each_marked(S.ge_rec, b, marks, box);
    else
        for_each_record(S.ge_rec, b, e, box);
    if (!fits) return false;
    // prefix xor along each axis, four nodes per dword (the axes follow each
    // other without padding: the running value restarts at nodes np and 2 np)
    int idx = 0;
    uint32_t m = 0;
    auto prefix = [&](int w, uint32_t v) {
        uint32_t out = 0;
#pragma unroll
        for (int j = 0; j < 4; ++j, ++idx) {
            if (idx == np || idx == 2 * np) m = 0;
            m ^= (v >> (8 * j)) & 0xffu;
            out |= m << (8 * j);
        }
        m32[w] = out;
    };
    if (n == 16) {
        // all 13 dwords are read before any is written back
        uint32_t v[13];
#pragma unroll
        for (int w = 0; w < 13; ++w) v[w] = m32[w];
#pragma unroll
        for (int w = 0; w < 13; ++w) prefix(w, v[w]);
    } else {
        for (int w = 0; w < (3 * np + 3) / 4; ++w) prefix(w, m32[w]);
    }
    return true;
}

// Half-size of the expanded cube (before the halving rule): n d / (2 m),
// stopped at symmetry walls, never below d.
template <class SR>
__device__ __forceinline__ float expanded_size(SR& S, float3 c, float d, int n, int m) {
    float R = (float)n * d / (float)(2 * m);
    const float cc[3] = {c.x, c.y, c.z};
#pragma unroll
    for (int a = 0; a < 3; ++a) {
        if (S.bc[2 * a] == MW_BC_NEUMANN) R = fminf(R, cc[a] - S.wlo[a]);
        if (S.bc[2 * a + 1] == MW_BC_NEUMANN) R = fminf(R, S.whi[a] - cc[a]);
    }
    return fmaxf(R, d);
}

// Expanded cubes are halved while they touch more than MAX_REGIONS dielectric
// boxes or more than EXP_MAX_COND conductors: R -> max(R / 2, d) while R > d,
// then R / 2.  exp_fit counts, in one pass over both candidate lists and with
// the comparisons build_cube and build_conductors make, the boxes touched at
// the first EXP_LEVELS sizes of that sequence and returns the first size that
// fits (else the last one, from which halving goes on), so that the cube is
// built once instead of once per size tried.  *level: its index.  When that
// size fits, both lists have at most 64 entries and one more than 8, *marked
// is set and *mdiel, *mcond mark (bit i: list entry b + i) the boxes the
// cube touches, so that the builds visit only those.
constexpr int EXP_LEVELS = 3;
template <class SR>
__device__ __forceinline__ float exp_fit(SR& S, int cell, float3 c, float R0, float d, int* level, bool* marked,
                                         unsigned long long* mdiel, unsigned long long* mcond) {
    const float cc[3] = {c.x, c.y, c.z};
    float Rk[EXP_LEVELS];
    // per size and axis: the cube's extent [lo, lo + 2R] and its part
    // inside the window at symmetry walls
    float lo[EXP_LEVELS][3], hi[EXP_LEVELS][3], clo[EXP_LEVELS][3], chi[EXP_LEVELS][3];
    Rk[0] = R0;
#pragma unroll
    for (int k = 1; k < EXP_LEVELS; ++k)
        Rk[k] = Rk[k - 1] > d ? fmaxf(0.5f * Rk[k - 1], d) : 0.5f * Rk[k - 1];
#pragma unroll
    for (int k = 0; k < EXP_LEVELS; ++k)
#pragma unroll
        for (int a = 0; a < 3; ++a) {
            lo[k][a] = cc[a] - Rk[k];
            hi[k][a] = lo[k][a] + 2.f * Rk[k];
            clo[k][a] = S.bc[2 * a] == MW_BC_NEUMANN ? fmaxf(lo[k][a], S.wlo[a]) : lo[k][a];
            chi[k][a] = S.bc[2 * a + 1] == MW_BC_NEUMANN ? fminf(hi[k][a], S.whi[a]) : hi[k][a];
        }
    int nd[EXP_LEVELS] = {}, nc[EXP_LEVELS] = {};
    unsigned long long md[EXP_LEVELS] = {}, mc[EXP_LEVELS] = {};
    const uint32_t db = gp(S.gx_off)[cell], de = gp(S.gx_off)[cell + 1];
    const uint32_t cb = gp(S.ge_off)[cell], ce = gp(S.ge_off)[cell + 1];
    uint32_t i = 0;
    for_each_record(S.gx_rec, db, de, [&](const float4& bl, const float4& bh) {
        const unsigned long long bit = i < 64 ? 1ull << i : 0ull;
#pragma unroll
        for (int k = 0; k < EXP_LEVELS; ++k) {
            const bool t = bl.x <= chi[k][0] && bh.x >= clo[k][0] && bl.y <= chi[k][1] && bh.y >= clo[k][1] &&
                           bl.z <= chi[k][2] && bh.z >= clo[k][2];
            nd[k] += t ? 1 : 0;
            md[k] |= t ? bit : 0ull;
        }
        ++i;
        return true;
    });
    i = 0;
    for_each_record(S.ge_rec, cb, ce, [&](const float4& bl, const float4& bh) {
        const unsigned long long bit = i < 64 ? 1ull << i : 0ull;
#pragma unroll
        for (int k = 0; k < EXP_LEVELS; ++k) {
            const bool t = bl.x < hi[k][0] && bh.x > lo[k][0] && bl.y < hi[k][1] && bh.y > lo[k][1] &&
                           bl.z < hi[k][2] && bh.z > lo[k][2];
            nc[k] += t ? 1 : 0;
            mc[k] |= t ? bit : 0ull;
        }
        ++i;
        return true;
    });
    int lv = EXP_LEVELS - 1;
    float R = Rk[EXP_LEVELS - 1];
    bool fits = nd[EXP_LEVELS - 1] <= MAX_REGIONS && nc[EXP_LEVELS - 1] <= EXP_MAX_COND;
    unsigned long long mdv = md[EXP_LEVELS - 1], mcv = mc[EXP_LEVELS - 1];
#pragma unroll
    for (int k = EXP_LEVELS - 2; k >= 0; --k)
        if (nd[k] <= MAX_REGIONS && nc[k] <= EXP_MAX_COND) {
            lv = k;
            R = Rk[k];
            fits = true;
            mdv = md[k];
            mcv = mc[k];
        }
    *level = lv;
    // (short lists are scanned in full: marking them saves nothing)
    *marked = fits && (de - db > 8 || ce - cb > 8) && de - db <= 64 && ce - cb <= 64;
    *mdiel = mdv;
    *mcond = mcv;
    return R;
}

__device__ __forceinline__ bool stratified_along(const CubeInfo& I, int s) {
    if (I.cls == 0) return true;
    const int a1 = (s + 1) % 3, a2 = (s + 2) % 3;
    const bool f1 = (I.present & ~I.A[a1]) == 0 && (a1 != 2 || I.n_layers == 1);
    const bool f2 = (I.present & ~I.A[a2]) == 0 && (a2 != 2 || I.n_layers == 1);
    return f1 && f2;
}

// Code of plane p normal to s of a cube stratified along s (ns: the mask
// row stride; the permittivity bits on the cell lattice).
__device__ __forceinline__ uint32_t plane_code(LaneCube L, const CubeInfo& I, int ns, int s, int p) {
    return cell_code(L, L.mask[s * ns + p] & I.present, L.bz[s == 2 ? p : 0]);
}

// Cell lattice (n odd, mask rows ns = n + 1 apart): mean permittivity of
// each plane normal to a, rounded to float, written as float bits to
// out[0..n).  Cells are summed by runs of equal masks (and background) in
// binary64; every partial sum is exact (at most 2^10 cells of permittivity
// in [1e-3, 1e3] times run lengths below 2^5), so the result does not depend
// on the order.
__device__ void plane_mean_eps(LaneCube L, int n, int a, LAS uint32_t* out) {
    const int ns = n + 1;
    const int u = a == 0 ? 1 : 0, v = a == 2 ? 1 : 2;
    uint32_t ubnd = 1u, vbnd = 1u;
    {
        uint32_t pu = L.mask[u * ns], pv = L.mask[v * ns], pb = a == 2 ? 0u : L.bz[0];
        for (int i = 1; i < n; ++i) {
            const uint32_t cu = L.mask[u * ns + i], cv = L.mask[v * ns + i], cb = a == 2 ? 0u : L.bz[i];
            ubnd |= (cu != pu ? 1u : 0u) << i;
            vbnd |= (cv != pv || cb != pb ? 1u : 0u) << i;
            pu = cu;
            pv = cv;
            pb = cb;
        }
    }
    const double area = (double)(n * n);
    uint32_t prev_ma = 0xffffffffu, prev_b = 0, prev = 0;
    for (int p = 0; p < n; ++p) {
        const uint32_t ma = L.mask[a * ns + p];
        const uint32_t bp = a == 2 ? L.bz[p] : 0u;
        if (ma == prev_ma && bp == prev_b) {
            out[p] = prev;
            continue;
        }
        double sum = 0.0;
        for (uint32_t ur = ubnd; ur;) {
            const int i = __builtin_ctz(ur);
            ur &= ur - 1u;
            const int li = (ur ? __builtin_ctz(ur) : n) - i;
            const uint32_t mau = ma & L.mask[u * ns + i];
            double row = 0.0;
            for (uint32_t vr = vbnd; vr;) {
                const int j = __builtin_ctz(vr);
                vr &= vr - 1u;
                const int lj = (vr ? __builtin_ctz(vr) : n) - j;
                const uint32_t bv = a == 2 ? bp : L.bz[j];
                row += (double)lj * (double)__uint_as_float(cell_code(L, mau & L.mask[v * ns + j], bv));
            }
            sum += (double)li * row;
        }
        prev_ma = ma;
        prev_b = bp;
        prev = __float_as_uint((float)(sum / area));
        out[p] = prev;
    }
}

// Mean codes of the planes normal to a (rounded half to even) written to
// out[0..n): each plane sums its cells by runs of equal masks (and
// background codes) along the two in-plane axes; planes whose own mask and
// background equal the previous plane's repeat it.  When a is not z, the
// second in-plane axis v is z.
__device__ void plane_mean_codes(LaneCube L, int n, int a, LAS uint32_t* out) {
    const int u = a == 0 ? 1 : 0, v = a == 2 ? 1 : 2;
    const unsigned long long area = (unsigned long long)n * n;
    // runs of equal masks along u, and of equal masks and background codes
    // along v (bit i: a run starts at i), found once for all planes
    uint32_t ubnd = 1u, vbnd = 1u;
    {
        uint32_t pu = L.mask[u * n], pv = L.mask[v * n], pb = a == 2 ? 0u : L.bz[0];
        for (int i = 1; i < n; ++i) {
            const uint32_t cu = L.mask[u * n + i], cv = L.mask[v * n + i], cb = a == 2 ? 0u : L.bz[i];
            ubnd |= (cu != pu ? 1u : 0u) << i;
            vbnd |= (cv != pv || cb != pb ? 1u : 0u) << i;
            pu = cu;
            pv = cv;
            pb = cb;
        }
    }
    const uint32_t full = n == 32 ? 0xffffffffu : ((1u << n) - 1u);
    uint32_t prev_ma = 0xffffffffu, prev_b = 0, prev = 0;
    for (int p = 0; p < n; ++p) {
        const uint32_t ma = L.mask[a * n + p];
        const uint32_t bp = a == 2 ? L.bz[p] : 0u;
        if (ma == prev_ma && bp == prev_b) {
            out[p] = prev;
            continue;
        }
        unsigned long long sum = 0;
        for (uint32_t ur = ubnd; ur;) {
            const int i = __builtin_ctz(ur);
            ur &= ur - 1u;
            const int li = (ur ? __builtin_ctz(ur) : n) - i;
            const uint32_t mau = ma & L.mask[u * n + i];
            unsigned long long row = 0;
            for (uint32_t vr = vbnd & full; vr;) {
                const int j = __builtin_ctz(vr);
                vr &= vr - 1u;
                const int lj = (vr ? __builtin_ctz(vr) : n) - j;
                const uint32_t bv = a == 2 ? bp : L.bz[j];
                row += (unsigned long long)lj * cell_code(L, mau & L.mask[v * n + j], bv);
            }
            sum += (unsigned long long)li * row;
        }
        unsigned long long qt, rem;
        if ((n & (n - 1)) == 0) {
            // the area n^2 is a power of two
            qt = sum >> (2 * __builtin_ctz((unsigned)n));
            rem = sum & (area - 1ull);
        } else {
            qt = sum / area;
            rem = sum % area;
        }
        if (2 * rem > area || (2 * rem == area && (qt & 1))) ++qt;
        prev_ma = ma;
        prev_b = bp;
        prev = (uint32_t)qt;
        out[p] = prev;
    }
}

// -------------------------------------------------------------------------
// Table cache.
// -------------------------------------------------------------------------
enum LookupResult { LOOKUP_HIT = 0, LOOKUP_PARK = 1, LOOKUP_FULL = 2 };
constexpr unsigned long long SLOT_HASH_MASK = 0xffffffff00000000ull;

// Finds the table of a key (words produced by key(q), q < key_words) or
// queues it for building.  Slot words pack a 32-bit key hash with the table
// index; the full key is compared before a hit is reported.
// Table layout: [last positive index, Kh bits, guide[2^GUIDE_BITS + 1],
// CDF[nb], sign bits[ceil(nb/32)]].  guide[g] = first b with CDF[b] >
// g * 2^GUIDE_SHIFT, so the answer for a word u lies in [guide[u >>
// GUIDE_SHIFT], guide[(u >> GUIDE_SHIFT) + 1]].  With 2048 buckets for the
// 6 (n-1)^2 entries of a 16-cell cube most buckets hold at most one entry.
constexpr uint32_t GUIDE_BITS = 11, GUIDE_SHIFT = 32 - GUIDE_BITS;
constexpr uint32_t TAB_GUIDE = 2, TAB_CDF = 2 + (1u << GUIDE_BITS) + 1;

__device__ __forceinline__ uint32_t key_hash_step(uint32_t h, uint32_t w) {
    h ^= w;
    h *= 0x01000193u;
    return h ^ (h >> 15);
}
constexpr uint32_t KEY_HASH_SEED = 0x811c9dc5u;

template <class KeyF>
__device__ uint32_t key_hash(uint32_t words, KeyF key) {
    uint32_t h = KEY_HASH_SEED;
#pragma unroll 4
    for (uint32_t q = 0; q < words; ++q) h = key_hash_step(h, key(q));
    return h;
}

// hash: key_hash of the key (computed by the caller).  On a hit, *glo and
// *ghi receive the guide pair of word u's bucket in the table (loaded with the
// key comparison).  A new key is queued for building (pending list); a
// table is ready when its ready word is nonzero.
template <class KeyF>
__device__ __forceinline__ int lookup_or_insert(const CacheDev& C, KeyF key, uint32_t hash, uint32_t* out_index,
                                               uint32_t u = 0, uint32_t* glo = nullptr, uint32_t* ghi = nullptr) {
    const uint32_t words = C.key_words;
    uint32_t h = hash;
    if (h == 0u) h = 1u;
    const unsigned long long hh = (unsigned long long)h << 32;
    uint32_t slot = (h * 0x9E3779B1u) & C.slot_mask;
    // The slot and ready words are read at workgroup scope (through the
    // compute unit's cache): a stale empty slot only sends the lane to the
    // CAS, which returns the current word; a stale "being inserted" slot
    // parks the walk, as the current word would (tables are built between
    // launches); ready words do not change during a launch, and each launch
    // starts with the compute units' caches invalidated.
    for (uint32_t probe = 0; probe <= C.slot_mask; ++probe) {
        unsigned long long cur =
            __hip_atomic_load(gpw(C.slot) + slot, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
        if (cur == 0ull) {
            const unsigned long long old = atomicCAS(&C.slot[slot], 0ull, hh | NO_INDEX);
            if (old == 0ull) {
                const uint32_t idx = atomicAdd(C.n_tables, 1u);
                if (idx >= C.capacity) {
                    // no room: the slot says so to every later lookup of
                    // this key until the cache is emptied
                    __hip_atomic_store(&C.slot[slot], hh | FULL_INDEX, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
                    return LOOKUP_FULL;
                }
                uint32_t* dst = C.keys + (size_t)idx * C.key_stride;
                for (uint32_t q = 0; q < words; ++q) dst[q] = key(q);
                for (uint32_t q = words; q < C.key_stride; ++q) dst[q] = 0u;
                __threadfence();
                __hip_atomic_store(&C.slot[slot], hh | idx, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
                const uint32_t pos = atomicAdd(C.n_pending, 1u);
                C.pending[pos] = idx;
                return LOOKUP_PARK;
            }
            cur = old;
        }
        if ((cur & SLOT_HASH_MASK) == hh) {
            const uint32_t idx = (uint32_t)cur;
            if (idx == NO_INDEX) return LOOKUP_PARK;
            if (idx == FULL_INDEX) return LOOKUP_FULL;
            const uint32_t rdy =
                __hip_atomic_load(gpw(C.ready) + idx, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
            uint32_t g0 = 0, g1 = 0;
            if (glo) {
                // the table's guide pair, read with the key (unused unless
                // the table is ready)
                const GAS uint32_t* tab = gp(C.data) + (size_t)idx * C.tab_words + TAB_GUIDE + (u >> GUIDE_SHIFT);
                g0 = tab[0];
                g1 = tab[1];
            }
            // the stored key in 16-byte rows (padding words are zero)
            const GAS guvec4* k4 = reinterpret_cast<const GAS guvec4*>(gp(C.keys) + (size_t)idx * C.key_stride);
            bool same = true;
#pragma unroll 2
            for (uint32_t c = 0; c < C.key_stride / 4; ++c) {
                const guvec4 v = k4[c];
                const uint32_t q = 4 * c;
                same &= v.x == (q < words ? key(q) : 0u);
                same &= v.y == (q + 1 < words ? key(q + 1) : 0u);
                same &= v.z == (q + 2 < words ? key(q + 2) : 0u);
                same &= v.w == (q + 3 < words ? key(q + 3) : 0u);
            }
            if (same) {
                if (!rdy) return LOOKUP_PARK;
                *out_index = idx;
                if (glo) {
                    *glo = g0;
                    *ghi = g1;
                }
                return LOOKUP_HIT;
            }
        }
        slot = (slot + 1) & C.slot_mask;
    }
    return LOOKUP_FULL;
}


// Sample for word u given the guide pair of its bucket (g = u >> GUIDE_SHIFT):
// glo = guide[g], ghi = guide[g + 1].  The first b with cdf[b] > u lies in
// [glo, ghi] (ghi itself when no b below it qualifies), so bisection over
// [glo, ghi) finds it, with no load at all when the bucket holds no entry
// boundary (glo = ghi).  nb: the answer when no entry qualifies.
__device__ __forceinline__ int table_sample_guided(const GAS uint32_t* tab, uint32_t nb, uint32_t u, uint32_t glo,
                                                   uint32_t ghi) {
    const GAS uint32_t* cdf = tab + TAB_CDF;
    uint32_t lo = glo, hi = ghi;
    while (lo < hi) {
        const uint32_t mid = (lo + hi) >> 1;
        if (cdf[mid] > u)
            hi = mid;
        else
            lo = mid + 1;
    }
    return lo < nb ? (int)lo : (int)tab[0];
}

__device__ __forceinline__ int table_sample(const GAS uint32_t* tab, uint32_t nb, uint32_t u) {
    const uint32_t g = u >> GUIDE_SHIFT;
    return table_sample_guided(tab, nb, u, tab[TAB_GUIDE + g], tab[TAB_GUIDE + g + 1]);
}

// Vertex-lattice boundary node of hit index b.
__device__ __forceinline__ void node_of_hit(int n, int b, int node[3]) {
    const int M = n - 1;
    const int f = b / (M * M), rem = b - f * M * M;
    const int bb = rem / M + 1, aa = rem - (bb - 1) * M + 1;
    const int ax = f >> 1, side = f & 1;
    const int face = side ? n : 0;
    // the two in-plane axes in ascending order take aa and bb (selects: no
    // indexed private array)
    node[0] = ax == 0 ? face : aa;
    node[1] = ax == 1 ? face : (ax == 0 ? aa : bb);
    node[2] = ax == 2 ? face : bb;
}

// Where a cell-lattice walk leaves cube (c, R): cell coordinates (i, j, k)
// with one of them -1 or n name the boundary panel, whose centre is returned.
__device__ __forceinline__ float3 cell_exit_point(float3 c, float R, float h, int n, int i, int j, int k) {
    auto coord = [&](float cc, int q) {
        return q < 0 ? cc - R : (q >= n ? cc + R : cc - R + ((float)q + 0.5f) * h);
    };
    return make_float3(coord(c.x, i), coord(c.y, j), coord(c.z, k));
}

// Cell coordinates (one of them -1 or n) of boundary panel b of the cell
// lattice, hit index (2 ax + side) n^2 + b1 n + a1 with (a1, b1) the panel's
// cells along the two other axes in ascending order.
__device__ __forceinline__ void cell_panel_of_hit(int n, int b, int* i, int* j, int* k) {
    const int f = b / (n * n), rem = b - f * n * n;
    const int b1 = rem / n, a1 = rem - b1 * n;
    const int ax = f >> 1, side = f & 1;
    const int out = side ? n : -1;
    *i = ax == 0 ? out : a1;
    *j = ax == 1 ? out : (ax == 0 ? a1 : b1);
    *k = ax == 2 ? out : b1;
}

// Looks up (or queues) the table of the key in key[0 .. C.key_words);
// out[0] = status, out[1] = table index.
__global__ void key_table_kernel(CacheDev C, const uint32_t* key, uint32_t* out) {
    if (threadIdx.x || blockIdx.x) return;
    uint32_t idx = NO_INDEX;
    auto kf = [&](uint32_t q) { return key[q]; };
    const int res = lookup_or_insert(C, kf, key_hash(C.key_words, kf), &idx);
    out[0] = (uint32_t)res;
    out[1] = idx;
}

// Looks up (or queues) the hop table of the uniform cube; out[0] = status,
// out[1] = table index.  Its exit distribution does not depend on the
// permittivity: the key holds code 1 (vertex lattice) or permittivity 1
// (cell lattice, odd n) in every plane.
__global__ void uniform_table_kernel(CacheDev C, int n, uint32_t* out) {
    if (threadIdx.x || blockIdx.x) return;
    uint32_t idx = NO_INDEX;
    const bool cell = (n & 1) != 0;
    auto key = [&](uint32_t q) {
        if (q == 0) return cell ? 2u : 0u;
        return q == 1 ? (uint32_t)n : (q == 2 ? 2u : (q < KEY_HDR ? 0u : (cell ? 0x3f800000u : 1u)));
    };
    const int res = lookup_or_insert(C, key, key_hash(C.key_words, key), &idx);
    out[0] = (uint32_t)res;
    out[1] = idx;
}

// -------------------------------------------------------------------------
// First transitions (Alg. 1: GaussianSurfaceSampling + FirstTransition).
// Every walk of a batch starts here, one lane per walk, so the per-walk work
// (Gaussian-surface sample, first cube, homogenisation, weight) runs with
// full lanes.  A walk whose first-cube table is missing is retried after the
// table is built.
// -------------------------------------------------------------------------
__device__ __forceinline__ float sel3(float3 v, int a) { return a == 0 ? v.x : (a == 1 ? v.y : v.z); }

// CELL: cubes of the cell-centred lattice (n odd).
template <bool MULTI, bool CELL = false>
__global__ void __launch_bounds__(FRW_THREADS) first_kernel(FirstArgs A) {
    extern __shared__ uint32_t lds[];
    if (A.dev_round && A.ctr->need_first == 0u) return;
    const int n = A.n;
    const int ns = CELL ? n + 1 : n;  // mask row stride
    uint32_t* my = lds + threadIdx.x * A.lane_stride;
    const LaneCube L = lane_cube(my, ns);
    LAS uint32_t* kbuf = L.bz + ns;
    unsigned long long c_br[4] = {0, 0, 0, 0}, c_halved = 0;
    uint32_t err = 0, missing = 0;
    // one structure per launch: its layer table goes to LDS once
    uint32_t* lt_lds = lds + FRW_THREADS * A.lane_stride;
    const uint32_t* lt = nullptr;
    if (!MULTI) {
        if (A.S0.n_layers <= LAYER_LDS) {
            if (threadIdx.x < 2 * LAYER_LDS) {
                const int q = min((int)(threadIdx.x % LAYER_LDS), A.S0.n_layers - 1);
                lt_lds[threadIdx.x] = threadIdx.x < LAYER_LDS ? __float_as_uint(gp(A.S0.layer_z0)[q])
                                                              : gp(CELL ? A.S0.layer_eps : A.S0.layer_code)[q];
            }
            lt = lt_lds;
        }
        __syncthreads();
    }
    for (unsigned long long g = blockIdx.x * (unsigned long long)blockDim.x + threadIdx.x; g < A.total;
         g += (unsigned long long)gridDim.x * blockDim.x) {
        const GAS Segment& SG = gp(A.segs)[MULTI ? find_segment(A.segs, A.n_segs, g) : 0];
        const unsigned long long k = g - SG.offset;
        if (A.round > 0 && gp(SG.first_done)[k]) continue;
        auto& S = [&]() -> decltype(auto) {
            if constexpr (MULTI)
                return *gp(SG.S);
            else
                return (A.S0);
        }();
        const GAS GaussDev& G = *gp(SG.G);
        const unsigned long long walk = SG.walk_begin + k;
        float3 c;
        int a_norm, side;
        float factor = 0.f;
        if (A.eval) {
            // evaluation of the kernel sum at a given point of G
            const float4 e = ldf4(A.eval + k);
            c = make_float3(e.x, e.y, e.z);
            const uint32_t fbits = __float_as_uint(e.w);
            a_norm = (int)(fbits & 3u);
            side = (int)(fbits >> 2);
        } else {
            // GaussianSurfaceSampling(G): rectangle (or patch) by its sampling
            // weight (the first whose cumulative weight exceeds the draw),
            // uniform point on it
            const Rand4 r = philox10(0u, 0u, (uint32_t)walk, ctr_hi(walk, PURPOSE_GAUSS), SG.k0, SG.k1);
            const float xa = ((float)r.x + 0.5f) * 2.3283064365386963e-10f * G.area;
            const GAS GaussFace* gf = gp(G.faces);
            const int nf = G.n_faces;
            int f_lo = 0;
            if (nf <= 8) {
                // few rectangles: count those whose cumulative weight is <=
                // the draw (independent loads)
#pragma unroll
                for (int q = 0; q < 7; ++q) {
                    const float cq = gf[min(q, nf - 1)].p.y;
                    f_lo += (q < nf - 1 && !(xa < cq)) ? 1 : 0;
                }
            } else {
                int f_hi = nf - 1;
                while (f_lo < f_hi) {
                    const int mid = (f_lo + f_hi) >> 1;
                    if (xa < gf[mid].p.y)
                        f_hi = mid;
                    else
                        f_lo = mid + 1;
                }
            }
            const float4 fp = ldf4(&G.faces[f_lo].p), ft = ldf4(&G.faces[f_lo].t);
            const uint32_t fbits = __float_as_uint(fp.z);
            a_norm = (int)(fbits & 3u);
            side = (int)(fbits >> 2);
            factor = fp.w;
            const float ua = ft.x + ((float)r.y + 0.5f) * 2.3283064365386963e-10f * (ft.y - ft.x);
            const float ub = ft.z + ((float)r.z + 0.5f) * 2.3283064365386963e-10f * (ft.w - ft.z);
            const float pl = fp.x;
            c = make_float3(a_norm == 0 ? pl : ua, a_norm == 1 ? pl : (a_norm == 0 ? ua : ub), a_norm == 2 ? pl : ub);
        }
        const int cell = grid_cell(S, c);
        const uint2 drange = make_uint2(gp(S.gd_off)[cell], gp(S.gd_off)[cell + 1]);
        int who;
        float R = fminf(query_dist(S, c, cell, &who), G.g);
        // FirstTransition: cube touching the master (Sec. III-C, Fig. 4
        // branches; homogenised along the normal when not stratified)
        CubeInfo I = build_cube<CELL>(S, cell, c, R, n, L, false, lt, &drange);
        const bool halved = I.overflow;
        for (int it = 0; it < 40 && I.overflow; ++it) {
            R *= 0.5f;  // capacity rule: halve while more than 16 boxes touch
            I = build_cube<CELL>(S, cell, c, R, n, L, false, lt, &drange);
        }
        if (I.overflow) {
            err |= ERR_REGIONS;
            gpw(SG.first_done)[k] = 1u;
            stf4(SG.first_state + k, make_float4(c.x, c.y, c.z, 0.f));
            continue;
        }
        const float h = 2.f * R / (float)n;
        int br, sax;
        if (I.cls == 0) {
            br = 0;
            sax = a_norm;
        } else if (stratified_along(I, a_norm)) {
            br = 1;
            sax = a_norm;
        } else if (I.cls == 1) {
            br = 2;
            sax = I.axis;
        } else {
            br = 3;
            sax = a_norm;
        }
        kbuf[0] = CELL ? 3u : 1u;  // first-transition table (of the cell lattice)
        kbuf[1] = (uint32_t)n;
        kbuf[2] = (uint32_t)sax;
        kbuf[3] = (uint32_t)a_norm;
        if (br == 3) {
            if (CELL)
                plane_mean_eps(L, n, a_norm, kbuf + KEY_HDR);
            else
                plane_mean_codes(L, n, a_norm, kbuf + KEY_HDR);
        } else {
            for (int p = 0; p < n; ++p) kbuf[KEY_HDR + p] = plane_code(L, I, ns, sax, p);
        }
        uint32_t idx, glo = 0, ghi = 0;
        const Rand4 r2 = philox10(0u, 0u, (uint32_t)walk, ctr_hi(walk, PURPOSE_FIRST), SG.k0, SG.k1);
        auto key = [&](uint32_t q) { return kbuf[q]; };
        const int res = lookup_or_insert(A.cache, key, key_hash(A.cache.key_words, key), &idx, r2.x, &glo, &ghi);
        if (res != LOOKUP_HIT) {
            if (res == LOOKUP_FULL) err |= ERR_TABLE_CAP;
            if (A.round == 0) gpw(SG.first_done)[k] = 0u;
            ++missing;
            continue;
        }
        const GAS uint32_t* tab = gp(A.cache.data) + (size_t)idx * A.cache.tab_words;
        const float Kh = __uint_as_float(tab[1]);
        if (A.eval) {
            stf4(SG.first_state + k, make_float4(Kh / h, 0.f, 0.f, 0.f));
            gpw(SG.first_done)[k] = 1u;
            continue;
        }
#pragma unroll
        for (int q = 0; q < 4; ++q) c_br[q] += br == q ? 1ull : 0ull;  // constant indices: registers
        c_halved += halved ? 1ull : 0ull;
        const int b = table_sample_guided(tab, A.cache.nb, r2.x, glo, ghi);
        const uint32_t sb = (tab[TAB_CDF + A.cache.nb + (b >> 5)] >> (b & 31)) & 1u;
        float sgn = sb ? 1.f : -1.f;
        if (!side) sgn = -sgn;
        const float omega = EPS0 * factor * (Kh / h) * sgn;
        float3 x;
        if (CELL) {
            int ci, cj, ck;
            cell_panel_of_hit(n, b, &ci, &cj, &ck);
            x = cell_exit_point(c, R, h, n, ci, cj, ck);
        } else {
            int nd[3];
            node_of_hit(n, b, nd);
            x = make_float3(c.x - R + (float)nd[0] * h, c.y - R + (float)nd[1] * h, c.z - R + (float)nd[2] * h);
        }
        const float3 xf = fold3(S, x);
        stf4(SG.first_state + k, make_float4(xf.x, xf.y, xf.z, omega));
        gpw(SG.first_done)[k] = 1u;
    }
    Counters& K = *A.ctr;
    for (int q = 0; q < 4; ++q)
        if (c_br[q]) atomicAdd(&K.first_branch[q], c_br[q]);
    if (c_halved) atomicAdd(&K.halved, c_halved);
    if (err) atomicOr(&K.err, err);
    if (missing) atomicAdd(&K.first_missing, missing);
}

// -------------------------------------------------------------------------
// MicroWalk on a lazily described cube (Alg. 3 with the link codes of the
// eight cells around the current node taken from the per-axis masks).
// -------------------------------------------------------------------------
struct MwState {
    int ni, nj, nk;
    uint32_t s;  // steps taken
    uint32_t mx0, mx1, my0, my1, mz0, mz1, bz0, bz1;
    // n <= 16: the masks of the cell rows around the node with the box bits
    // moved to bits 16..31; x and y rows set bits 0..15, a z row k sets bit
    // 15 - k (its background)
    uint32_t px0, px1, py0, py1, pz0, pz1;
};

// n <= 16: the code of a cell whose prepared masks meet in m sits at
// codes[clz(m)]: a box bit 16 + b gives codes[15 - b], the background bit
// 15 - k of z row k gives codes[16 + k] = bz[k].  One read, no select.
__device__ __forceinline__ uint32_t cell_code16(LaneCube L, uint32_t m) { return L.codes[__builtin_clz(m)]; }

__device__ __forceinline__ uint32_t prep_xy(uint32_t v) { return (v << 16) | 0xffffu; }
__device__ __forceinline__ uint32_t prep_z(uint32_t v, int k) { return (v << 16) | (1u << (15 - k)); }

__device__ __forceinline__ void mw_begin16(MwState& M, LaneCube L, int n) {
    M.ni = M.nj = M.nk = n / 2;
    M.s = 0;
    M.px0 = prep_xy(L.mask[M.ni - 1]);
    M.px1 = prep_xy(L.mask[M.ni]);
    M.py0 = prep_xy(L.mask[n + M.nj - 1]);
    M.py1 = prep_xy(L.mask[n + M.nj]);
    M.pz0 = prep_z(L.mask[2 * n + M.nk - 1], M.nk - 1);
    M.pz1 = prep_z(L.mask[2 * n + M.nk], M.nk);
}

// mw_block for n <= 16 (the same steps and moves; the cell codes come from
// cell_code16).
__device__ __forceinline__ bool mw_block16(MwState& M, LaneCube L, int n, const Rand4& r) {
    const uint32_t us[4] = {r.x, r.y, r.z, r.w};
    bool alive = true;
    // node coordinates packed in bytes 0, 1, 2 (a coordinate never drops
    // below 0, so a move is one shifted add)
    uint32_t co = (uint32_t)M.ni | ((uint32_t)M.nj << 8) | ((uint32_t)M.nk << 16);
#pragma unroll
    for (int q = 0; q < 4; ++q) {
        if (alive) {
            const uint32_t c000 = cell_code16(L, M.px0 & M.py0 & M.pz0), c001 = cell_code16(L, M.px1 & M.py0 & M.pz0);
            const uint32_t c010 = cell_code16(L, M.px0 & M.py1 & M.pz0), c011 = cell_code16(L, M.px1 & M.py1 & M.pz0);
            const uint32_t c100 = cell_code16(L, M.px0 & M.py0 & M.pz1), c101 = cell_code16(L, M.px1 & M.py0 & M.pz1);
            const uint32_t c110 = cell_code16(L, M.px0 & M.py1 & M.pz1), c111 = cell_code16(L, M.px1 & M.py1 & M.pz1);
            const uint32_t a0 = c000 + c100, a1 = c010 + c110;
            const uint32_t b0 = c001 + c101, b1 = c011 + c111;
            const uint32_t gmx = a0 + a1, total = gmx + b0 + b1;
            const uint32_t gmy = a0 + b0, gmz = c000 + c001 + c010 + c011;
            const uint32_t S2 = total + gmy, S3 = total + total, S4 = S3 + gmz, S5 = S3 + total;
            const uint32_t xq = __umulhi(us[q], S5);
            // the move #{k : xq >= S_k} of the five thresholds, decoded from
            // the comparisons: x while xq < total (up when xq >= gmx), y while
            // xq < S3 (up when xq >= S2), z otherwise (up when xq >= S4)
            const bool t2 = xq >= total, t4 = xq >= S3;
            const bool ux = xq >= gmx, uy = xq >= S2, uz = xq >= S4;
            const bool up = (t4 & uz) | (t2 & !t4 & uy) | (!t2 & ux);  // lane masks: scalar logic
            const uint32_t sh = t4 ? 16u : (t2 ? 8u : 0u);
            ++M.s;
            co += (up ? 1u : 0xffffffffu) << sh;
            const int cnew = (int)((co >> sh) & 0xffu);
            alive = cnew != 0 && cnew != n;
            // prepared masks of the two cell rows around the new node along
            // ax (the index is clamped; a walk that left is not stepped again)
            const int cc = min(max(cnew, 1), n - 1);
            // rows cc - 1 and cc of the move's axis (row0 points at row -1 of
            // x; n is even, so the three axes start n u16 apart)
            const LAS uint16_t* rr = (t4 ? L.mask + 2 * n : (t2 ? L.mask + n : L.mask)) - 1 + cc;
            const uint32_t lo = rr[0], hi = rr[1];
            const uint32_t bgz = 1u << (15 - cc);  // background bit of z row cc
            const uint32_t plo = t4 ? (lo << 16) | (bgz << 1) : prep_xy(lo);
            const uint32_t phi = t4 ? (hi << 16) | bgz : prep_xy(hi);
            const bool xm = !t2, ym = t2 && !t4;
            M.px0 = xm ? plo : M.px0;
            M.px1 = xm ? phi : M.px1;
            M.py0 = ym ? plo : M.py0;
            M.py1 = ym ? phi : M.py1;
            M.pz0 = t4 ? plo : M.pz0;
            M.pz1 = t4 ? phi : M.pz1;
        }
    }
    M.ni = (int)(co & 0xffu);
    M.nj = (int)((co >> 8) & 0xffu);
    M.nk = (int)((co >> 16) & 0xffu);
    return alive;
}

__device__ __forceinline__ void mw_begin(MwState& M, LaneCube L, int n) {
    M.ni = M.nj = M.nk = n / 2;
    M.s = 0;
    M.mx0 = L.mask[M.ni - 1];
    M.mx1 = L.mask[M.ni];
    M.my0 = L.mask[n + M.nj - 1];
    M.my1 = L.mask[n + M.nj];
    M.mz0 = L.mask[2 * n + M.nk - 1];
    M.mz1 = L.mask[2 * n + M.nk];
    M.bz0 = L.bz[M.nk - 1];
    M.bz1 = L.bz[M.nk];
}

// Up to four steps with the four words of one Philox block; false once the
// walk has reached a boundary node.  Straight-line code: the eight cell codes
// are always looked up (where all eight masks agree they are one code and the
// choice reduces to floor(6 u / 2^32), but a branch for that case would run
// beside the general one in most waves), and the move updates the masks with
// selects.
__device__ __forceinline__ bool mw_block(MwState& M, LaneCube L, int n, const Rand4& r) {
    const uint32_t us[4] = {r.x, r.y, r.z, r.w};
    bool alive = true;
#pragma unroll
    for (int q = 0; q < 4; ++q) {
        if (alive) {
            const uint32_t m000 = M.mx0 & M.my0 & M.mz0, m001 = M.mx1 & M.my0 & M.mz0;
            const uint32_t m010 = M.mx0 & M.my1 & M.mz0, m011 = M.mx1 & M.my1 & M.mz0;
            const uint32_t m100 = M.mx0 & M.my0 & M.mz1, m101 = M.mx1 & M.my0 & M.mz1;
            const uint32_t m110 = M.mx0 & M.my1 & M.mz1, m111 = M.mx1 & M.my1 & M.mz1;
            const uint32_t c000 = cell_code(L, m000, M.bz0), c001 = cell_code(L, m001, M.bz0);
            const uint32_t c010 = cell_code(L, m010, M.bz0), c011 = cell_code(L, m011, M.bz0);
            const uint32_t c100 = cell_code(L, m100, M.bz1), c101 = cell_code(L, m101, M.bz1);
            const uint32_t c110 = cell_code(L, m110, M.bz1), c111 = cell_code(L, m111, M.bz1);
            const uint32_t a0 = c000 + c100, a1 = c010 + c110;
            const uint32_t b0 = c001 + c101, b1 = c011 + c111;
            const uint32_t gmx = a0 + a1, total = gmx + b0 + b1;
            const uint32_t gmy = a0 + b0, gmz = c000 + c001 + c010 + c011;
            const uint32_t S2 = total + gmy, S3 = total + total, S4 = S3 + gmz, S5 = S3 + total;
            const uint32_t xq = __umulhi(us[q], S5);
            const uint32_t d = (uint32_t)(xq >= gmx) + (uint32_t)(xq >= total) + (uint32_t)(xq >= S2) +
                               (uint32_t)(xq >= S3) + (uint32_t)(xq >= S4);
            const int ax = (int)(d >> 1);
            const int dir = (d & 1u) ? 1 : -1;
            ++M.s;
            M.ni += ax == 0 ? dir : 0;
            M.nj += ax == 1 ? dir : 0;
            M.nk += ax == 2 ? dir : 0;
            const int cnew = ax == 0 ? M.ni : (ax == 1 ? M.nj : M.nk);
            alive = cnew != 0 && cnew != n;
            // masks of the two cell rows around the new node along ax (the
            // index is clamped; a walk that left is not stepped again)
            const int cc = min(max(cnew, 1), n - 1);
            const uint32_t lo = L.mask[ax * n + cc - 1], hi = L.mask[ax * n + cc];
            const uint32_t zlo = L.bz[cc - 1], zhi = L.bz[cc];
            M.mx0 = ax == 0 ? lo : M.mx0;
            M.mx1 = ax == 0 ? hi : M.mx1;
            M.my0 = ax == 1 ? lo : M.my0;
            M.my1 = ax == 1 ? hi : M.my1;
            M.mz0 = ax == 2 ? lo : M.mz0;
            M.mz1 = ax == 2 ? hi : M.mz1;
            M.bz0 = ax == 2 ? zlo : M.bz0;
            M.bz1 = ax == 2 ? zhi : M.bz1;
        }
    }
    return alive;
}

// -------------------------------------------------------------------------
// MicroWalk on the cell-centred lattice of Sec. III-A (nodes at the voxel
// centres; n odd, mask rows ns = n + 1 apart).  The walk stands on cell
// (ni, nj, nk) and starts in the centre cell.  The Eq. (6) coefficient
// towards a neighbour cell is eps_nb / (eps_nb + eps_v), kept as
// rint(. * 2^24) of a binary64 division (exactly 2^23 for equal
// permittivities), and 2^24 towards a boundary panel; the walk leaves the
// cube at the centre of that panel.
// -------------------------------------------------------------------------
__device__ __forceinline__ uint32_t eq6_code(uint32_t nb, uint32_t v) {
    if (nb == v) return 1u << 23;
    const double e = (double)__uint_as_float(nb), ev = (double)__uint_as_float(v);
    return (uint32_t)rint(e / (e + ev) * 16777216.0);
}

// n <= 15: the prepared masks (as for cell_code16, with the z rows' own
// background bits) of the rows i-1, i, i+1 of each axis are kept in
// registers, indices clamped into the cube, so that every cell read is one
// LDS load and a move reloads one row.  The six Eq. (6) codes need a
// binary64 division only at a cell whose neighbours differ from it.
struct CellRows {
    uint32_t x0, x1, x2, y0, y1, y2, z0, z1, z2;
    uint32_t b0, b1, b2;  // n > 15: background codes of z rows k-1, k, k+1
};

__device__ __forceinline__ void mw_begin_cell16(MwState& M, CellRows& C, LaneCube L, int n) {
    const int ns = n + 1, c = (n - 1) / 2;
    M.ni = M.nj = M.nk = c;
    M.s = 0;
    C.x0 = prep_xy(L.mask[c - 1]);
    C.x1 = prep_xy(L.mask[c]);
    C.x2 = prep_xy(L.mask[c + 1]);
    C.y0 = prep_xy(L.mask[ns + c - 1]);
    C.y1 = prep_xy(L.mask[ns + c]);
    C.y2 = prep_xy(L.mask[ns + c + 1]);
    C.z0 = prep_z(L.mask[2 * ns + c - 1], c - 1);
    C.z1 = prep_z(L.mask[2 * ns + c], c);
    C.z2 = prep_z(L.mask[2 * ns + c + 1], c + 1);
}

__device__ __forceinline__ bool mw_block_cell16(MwState& M, CellRows& C, LaneCube L, int n, const Rand4& r) {
    const int ns = n + 1;
    const uint32_t us[4] = {r.x, r.y, r.z, r.w};
    constexpr uint32_t PANEL = 1u << 24, HALF = 1u << 23;
    bool alive = true;
#pragma unroll
    for (int q = 0; q < 4; ++q) {
        if (alive) {
            const int i = M.ni, j = M.nj, k = M.nk;
            const uint32_t ev = cell_code16(L, C.x1 & C.y1 & C.z1);
            const uint32_t e0 = cell_code16(L, C.x0 & C.y1 & C.z1), e1 = cell_code16(L, C.x2 & C.y1 & C.z1);
            const uint32_t e2 = cell_code16(L, C.x1 & C.y0 & C.z1), e3 = cell_code16(L, C.x1 & C.y2 & C.z1);
            const uint32_t e4 = cell_code16(L, C.x1 & C.y1 & C.z0), e5 = cell_code16(L, C.x1 & C.y1 & C.z2);
            uint32_t g0 = HALF, g1 = HALF, g2 = HALF, g3 = HALF, g4 = HALF, g5 = HALF;
            if ((e0 != ev) | (e1 != ev) | (e2 != ev) | (e3 != ev) | (e4 != ev) | (e5 != ev)) {
                g0 = eq6_code(e0, ev);
                g1 = eq6_code(e1, ev);
                g2 = eq6_code(e2, ev);
                g3 = eq6_code(e3, ev);
                g4 = eq6_code(e4, ev);
                g5 = eq6_code(e5, ev);
            }
            // links out of the cube go to boundary panels (the clamped rows'
            // reads above are then ignored)
            g0 = i > 0 ? g0 : PANEL;
            g1 = i < n - 1 ? g1 : PANEL;
            g2 = j > 0 ? g2 : PANEL;
            g3 = j < n - 1 ? g3 : PANEL;
            g4 = k > 0 ? g4 : PANEL;
            g5 = k < n - 1 ? g5 : PANEL;
            const uint32_t S0 = g0, S1 = S0 + g1, S2 = S1 + g2, S3 = S2 + g3, S4 = S3 + g4, S5 = S4 + g5;
            const uint32_t xq = __umulhi(us[q], S5);
            const uint32_t d = (uint32_t)(xq >= S0) + (uint32_t)(xq >= S1) + (uint32_t)(xq >= S2) +
                               (uint32_t)(xq >= S3) + (uint32_t)(xq >= S4);
            const int ax = (int)(d >> 1);
            const bool up = (d & 1u) != 0;
            const int dir = up ? 1 : -1;
            ++M.s;
            M.ni += ax == 0 ? dir : 0;
            M.nj += ax == 1 ? dir : 0;
            M.nk += ax == 2 ? dir : 0;
            const int cnew = ax == 0 ? M.ni : (ax == 1 ? M.nj : M.nk);
            alive = cnew >= 0 && cnew < n;
            // the row that enters the window along ax (clamped; a walk that
            // left is not stepped again)
            const int rr = min(max(cnew + dir, 0), n - 1);
            const uint32_t raw = L.mask[ax * ns + rr];
            const uint32_t v = ax == 2 ? prep_z(raw, rr) : prep_xy(raw);
            // rows (r0, r1, r2) of the move's axis become (r1, r2, v) going
            // up and (v, r0, r1) going down (selects: no branch on the axis)
            auto shift = [&](bool on, uint32_t& r0, uint32_t& r1, uint32_t& r2) {
                const uint32_t a0 = r0, a1 = r1, a2 = r2;
                r0 = on ? (up ? a1 : v) : a0;
                r1 = on ? (up ? a2 : a0) : a1;
                r2 = on ? (up ? v : a1) : a2;
            };
            shift(ax == 0, C.x0, C.x1, C.x2);
            shift(ax == 1, C.y0, C.y1, C.y2);
            shift(ax == 2, C.z0, C.z1, C.z2);
        }
    }
    return alive;
}

// n > 15 (up to 31): the same steps with the rows' plain masks and the z
// rows' background codes in registers; a cell read is one LDS load of the
// top box's code and a select of the background code.
__device__ __forceinline__ void mw_begin_cell(MwState& M, CellRows& C, LaneCube L, int n) {
    const int ns = n + 1, c = (n - 1) / 2;
    M.ni = M.nj = M.nk = c;
    M.s = 0;
    C.x0 = L.mask[c - 1];
    C.x1 = L.mask[c];
    C.x2 = L.mask[c + 1];
    C.y0 = L.mask[ns + c - 1];
    C.y1 = L.mask[ns + c];
    C.y2 = L.mask[ns + c + 1];
    C.z0 = L.mask[2 * ns + c - 1];
    C.z1 = L.mask[2 * ns + c];
    C.z2 = L.mask[2 * ns + c + 1];
    C.b0 = L.bz[c - 1];
    C.b1 = L.bz[c];
    C.b2 = L.bz[c + 1];
}

__device__ __forceinline__ bool mw_block_cell(MwState& M, CellRows& C, LaneCube L, int n, const Rand4& r) {
    const int ns = n + 1;
    const uint32_t us[4] = {r.x, r.y, r.z, r.w};
    constexpr uint32_t PANEL = 1u << 24, HALF = 1u << 23;
    bool alive = true;
#pragma unroll
    for (int q = 0; q < 4; ++q) {
        if (alive) {
            const int i = M.ni, j = M.nj, k = M.nk;
            const uint32_t ev = cell_code(L, C.x1 & C.y1 & C.z1, C.b1);
            const uint32_t e0 = cell_code(L, C.x0 & C.y1 & C.z1, C.b1), e1 = cell_code(L, C.x2 & C.y1 & C.z1, C.b1);
            const uint32_t e2 = cell_code(L, C.x1 & C.y0 & C.z1, C.b1), e3 = cell_code(L, C.x1 & C.y2 & C.z1, C.b1);
            const uint32_t e4 = cell_code(L, C.x1 & C.y1 & C.z0, C.b0), e5 = cell_code(L, C.x1 & C.y1 & C.z2, C.b2);
            uint32_t g0 = HALF, g1 = HALF, g2 = HALF, g3 = HALF, g4 = HALF, g5 = HALF;
            if ((e0 != ev) | (e1 != ev) | (e2 != ev) | (e3 != ev) | (e4 != ev) | (e5 != ev)) {
                g0 = eq6_code(e0, ev);
                g1 = eq6_code(e1, ev);
                g2 = eq6_code(e2, ev);
                g3 = eq6_code(e3, ev);
                g4 = eq6_code(e4, ev);
                g5 = eq6_code(e5, ev);
            }
            g0 = i > 0 ? g0 : PANEL;
            g1 = i < n - 1 ? g1 : PANEL;
            g2 = j > 0 ? g2 : PANEL;
            g3 = j < n - 1 ? g3 : PANEL;
            g4 = k > 0 ? g4 : PANEL;
            g5 = k < n - 1 ? g5 : PANEL;
            const uint32_t S0 = g0, S1 = S0 + g1, S2 = S1 + g2, S3 = S2 + g3, S4 = S3 + g4, S5 = S4 + g5;
            const uint32_t xq = __umulhi(us[q], S5);
            const uint32_t d = (uint32_t)(xq >= S0) + (uint32_t)(xq >= S1) + (uint32_t)(xq >= S2) +
                               (uint32_t)(xq >= S3) + (uint32_t)(xq >= S4);
            const int ax = (int)(d >> 1);
            const bool up = (d & 1u) != 0;
            const int dir = up ? 1 : -1;
            ++M.s;
            M.ni += ax == 0 ? dir : 0;
            M.nj += ax == 1 ? dir : 0;
            M.nk += ax == 2 ? dir : 0;
            const int cnew = ax == 0 ? M.ni : (ax == 1 ? M.nj : M.nk);
            alive = cnew >= 0 && cnew < n;
            const int rr = min(max(cnew + dir, 0), n - 1);
            const uint32_t v = L.mask[ax * ns + rr];
            const uint32_t vb = L.bz[rr];  // used for z moves only
            auto shift = [&](bool on, uint32_t& r0, uint32_t& r1, uint32_t& r2, uint32_t nv) {
                const uint32_t a0 = r0, a1 = r1, a2 = r2;
                r0 = on ? (up ? a1 : nv) : a0;
                r1 = on ? (up ? a2 : a0) : a1;
                r2 = on ? (up ? nv : a1) : a2;
            };
            shift(ax == 0, C.x0, C.x1, C.x2, v);
            shift(ax == 1, C.y0, C.y1, C.y2, v);
            shift(ax == 2, C.z0, C.z1, C.z2, v);
            shift(ax == 2, C.b0, C.b1, C.b2, vb);
        }
    }
    return alive;
}

// MicroWalk-E steps: node masks of the current node and its two neighbours
// per axis, kept in registers.
struct MwStateE {
    uint32_t xm, xc, xp, ym, yc, yp, zm, zc, zp;
};

__device__ __forceinline__ void mw_begin_e(const MwState& M, MwStateE& Q, LaneExp E, int n) {
    const int np = n + 1;
    Q.xm = E.nmask[M.ni - 1];
    Q.xc = E.nmask[M.ni];
    Q.xp = E.nmask[M.ni + 1];
    Q.ym = E.nmask[np + M.nj - 1];
    Q.yc = E.nmask[np + M.nj];
    Q.yp = E.nmask[np + M.nj + 1];
    Q.zm = E.nmask[2 * np + M.nk - 1];
    Q.zc = E.nmask[2 * np + M.nk];
    Q.zp = E.nmask[2 * np + M.nk + 1];
}

// Code of a link cut at fraction tq / 65535 of its length: rint(g / theta),
// that is floor((65535 g + tq / 2) / tq), in integers.  g is at most four
// cell codes (< 2^28) and tq >= 4096, so the numerator x is below 2^44 and
// the quotient below 2^32; long division in two steps of 32-bit divisions:
// x = xh 2^16 + xl, q = (xh / tq) 2^16 + ((xh % tq) 2^16 + xl) / tq.
__device__ __forceinline__ uint32_t cut_link(uint32_t g, uint32_t tq) {
    const uint64_t x = (uint64_t)g * 65535u + (tq >> 1);
    const uint32_t xh = (uint32_t)(x >> 16), xl = (uint32_t)x & 0xffffu;
    const uint32_t q1 = xh / tq, r1 = xh - q1 * tq;
    const uint32_t q2 = ((r1 << 16) | xl) / tq;
    return (q1 << 16) + q2;
}

// The direction rule of Alg. 3 as comparisons: bit k (k = 0..4) is set when
// floor(u S5 / 2^32) >= S_k, S_k the prefix sums of the six link codes; the
// direction is the number of set bits.  Six uncut links sum to less than
// 2^31 (24 cell codes of at most rint(1e3 2^16)); cut links (wide) can carry
// the sums past 2^32, so they are formed in 64 bits and the product's high
// part is u (S5 >> 32) + mulhi(u, S5 mod 2^32).
__device__ __forceinline__ uint32_t step_bits(const uint32_t g[6], uint32_t u, bool wide) {
    if (!wide) {
        const uint32_t S0 = g[0], S1 = S0 + g[1], S2 = S1 + g[2], S3 = S2 + g[3], S4 = S3 + g[4];
        const uint32_t xq = __umulhi(u, S4 + g[5]);
        return (uint32_t)(xq >= S0) | ((uint32_t)(xq >= S1) << 1) | ((uint32_t)(xq >= S2) << 2) |
               ((uint32_t)(xq >= S3) << 3) | ((uint32_t)(xq >= S4) << 4);
    }
    const uint64_t S0 = g[0], S1 = S0 + g[1], S2 = S1 + g[2], S3 = S2 + g[3], S4 = S3 + g[4];
    const uint64_t S5 = S4 + g[5];
    const uint64_t xq = (uint64_t)u * (uint32_t)(S5 >> 32) + __umulhi(u, (uint32_t)S5);
    return (uint32_t)(xq >= S0) | ((uint32_t)(xq >= S1) << 1) | ((uint32_t)(xq >= S2) << 2) |
           ((uint32_t)(xq >= S3) << 3) | ((uint32_t)(xq >= S4) << 4);
}

// Up to four MicroWalk-E steps (one Philox block).  Returns 0 while the walk
// is inside, 1 when it reached a boundary node, 2 when it reached an
// absorbing node (*net: the conductor's net, or env_net beyond a grounded
// face).  Links into absorbing nodes are cut where they enter the object.
__device__ __forceinline__ int mw_block_e(MwState& M, MwStateE& Q, LaneCube L, LaneExp E, int n, const Rand4& r,
                                          int env_net, int* net) {
    const uint32_t us[4] = {r.x, r.y, r.z, r.w};
    const int np = n + 1;
    int st = 0;
#pragma unroll
    for (int q = 0; q < 4; ++q) {
        if (st == 0) {
            const uint32_t m000 = M.mx0 & M.my0 & M.mz0, m001 = M.mx1 & M.my0 & M.mz0;
            const uint32_t m010 = M.mx0 & M.my1 & M.mz0, m011 = M.mx1 & M.my1 & M.mz0;
            const uint32_t m100 = M.mx0 & M.my0 & M.mz1, m101 = M.mx1 & M.my0 & M.mz1;
            const uint32_t m110 = M.mx0 & M.my1 & M.mz1, m111 = M.mx1 & M.my1 & M.mz1;
            const uint32_t c000 = cell_code(L, m000, M.bz0), c001 = cell_code(L, m001, M.bz0);
            const uint32_t c010 = cell_code(L, m010, M.bz0), c011 = cell_code(L, m011, M.bz0);
            const uint32_t c100 = cell_code(L, m100, M.bz1), c101 = cell_code(L, m101, M.bz1);
            const uint32_t c110 = cell_code(L, m110, M.bz1), c111 = cell_code(L, m111, M.bz1);
            const uint32_t a0 = c000 + c100, a1 = c010 + c110;
            const uint32_t b0 = c001 + c101, b1 = c011 + c111;
            // links -x, +x, -y, +y, -z, +z
            uint32_t g[6] = {a0 + a1, b0 + b1, a0 + b0, a1 + b1, c000 + c001 + c010 + c011,
                             c100 + c101 + c110 + c111};
            const uint32_t nx[6] = {Q.xm, Q.xp, Q.xc, Q.xc, Q.xc, Q.xc};
            const uint32_t ny[6] = {Q.yc, Q.yc, Q.ym, Q.yp, Q.yc, Q.yc};
            const uint32_t nz[6] = {Q.zc, Q.zc, Q.zc, Q.zc, Q.zm, Q.zp};
            bool cut = false;
#pragma unroll
            for (int dd = 0; dd < 6; ++dd) {
                const uint32_t env = (nx[dd] | ny[dd] | nz[dd]) & 0x80u;
                const uint32_t cm = nx[dd] & ny[dd] & nz[dd] & 0x7fu;
                if (env | cm) {
                    const int b = env ? 7 : __ffs(cm) - 1;
                    g[dd] = cut_link(g[dd], E.theta[(b * 3 + (dd >> 1)) * 2 + ((dd & 1) ? 0 : 1)]);
                    cut = true;
                }
            }
            const uint32_t d = (uint32_t)__popc(step_bits(g, us[q], cut));
            const int ax = (int)(d >> 1);
            const bool up = (d & 1u) != 0;
            ++M.s;
            int cnew;
            if (ax == 0) {
                M.ni += up ? 1 : -1;
                cnew = M.ni;
                if (up) {
                    Q.xm = Q.xc;
                    Q.xc = Q.xp;
                    Q.xp = E.nmask[min(cnew + 1, n)];
                } else {
                    Q.xp = Q.xc;
                    Q.xc = Q.xm;
                    Q.xm = E.nmask[max(cnew - 1, 0)];
                }
            } else if (ax == 1) {
                M.nj += up ? 1 : -1;
                cnew = M.nj;
                if (up) {
                    Q.ym = Q.yc;
                    Q.yc = Q.yp;
                    Q.yp = E.nmask[np + min(cnew + 1, n)];
                } else {
                    Q.yp = Q.yc;
                    Q.yc = Q.ym;
                    Q.ym = E.nmask[np + max(cnew - 1, 0)];
                }
            } else {
                M.nk += up ? 1 : -1;
                cnew = M.nk;
                if (up) {
                    Q.zm = Q.zc;
                    Q.zc = Q.zp;
                    Q.zp = E.nmask[2 * np + min(cnew + 1, n)];
                } else {
                    Q.zp = Q.zc;
                    Q.zc = Q.zm;
                    Q.zm = E.nmask[2 * np + max(cnew - 1, 0)];
                }
            }
            if (cnew == 0 || cnew == n) {
                st = 1;
            } else {
                const uint32_t env = (Q.xc | Q.yc | Q.zc) & 0x80u;
                const uint32_t cm = Q.xc & Q.yc & Q.zc & 0x7fu;
                if (env) {
                    st = 2;
                    *net = env_net;
                } else if (cm) {
                    st = 2;
                    *net = E.cnet[__ffs(cm) - 1];
                } else {
                    // cell masks of the new node
                    const uint32_t lo = L.mask[ax * n + cnew - 1], hi = L.mask[ax * n + cnew];
                    if (ax == 0) {
                        M.mx0 = lo;
                        M.mx1 = hi;
                    } else if (ax == 1) {
                        M.my0 = lo;
                        M.my1 = hi;
                    } else {
                        M.mz0 = lo;
                        M.mz1 = hi;
                        M.bz0 = L.bz[cnew - 1];
                        M.bz1 = L.bz[cnew];
                    }
                }
            }
        }
    }
    return st;
}

// mw_block_e for n <= 16: the same steps, moves and absorptions, with the
// cell codes of cell_code16 and the move decoded from the comparisons as in
// mw_block16 (no branch on the axis).
__device__ __forceinline__ int mw_block_e16(MwState& M, MwStateE& Q, LaneCube L, LaneExp E, int n, const Rand4& r,
                                            int env_net, int* net) {
    const uint32_t us[4] = {r.x, r.y, r.z, r.w};
    const int np = n + 1;
    int st = 0;
    uint32_t co = (uint32_t)M.ni | ((uint32_t)M.nj << 8) | ((uint32_t)M.nk << 16);
#pragma unroll
    for (int q = 0; q < 4; ++q) {
        if (st == 0) {
            const uint32_t c000 = cell_code16(L, M.px0 & M.py0 & M.pz0), c001 = cell_code16(L, M.px1 & M.py0 & M.pz0);
            const uint32_t c010 = cell_code16(L, M.px0 & M.py1 & M.pz0), c011 = cell_code16(L, M.px1 & M.py1 & M.pz0);
            const uint32_t c100 = cell_code16(L, M.px0 & M.py0 & M.pz1), c101 = cell_code16(L, M.px1 & M.py0 & M.pz1);
            const uint32_t c110 = cell_code16(L, M.px0 & M.py1 & M.pz1), c111 = cell_code16(L, M.px1 & M.py1 & M.pz1);
            const uint32_t a0 = c000 + c100, a1 = c010 + c110;
            const uint32_t b0 = c001 + c101, b1 = c011 + c111;
            // links -x, +x, -y, +y, -z, +z
            uint32_t g[6] = {a0 + a1, b0 + b1, a0 + b0, a1 + b1, c000 + c001 + c010 + c011,
                             c100 + c101 + c110 + c111};
            // a link is cut only if its far node is absorbing: one of the
            // coordinates around the node lies beyond a grounded face, or
            // one conductor holds a coordinate of every axis
            const uint32_t near = (((Q.xm | Q.xc | Q.xp) & (Q.ym | Q.yc | Q.yp) & (Q.zm | Q.zc | Q.zp)) & 0x7fu) |
                                  ((Q.xm | Q.xc | Q.xp | Q.ym | Q.yc | Q.yp | Q.zm | Q.zc | Q.zp) & 0x80u);
            bool cut = false;
            if (near) {
                const uint32_t nx[6] = {Q.xm, Q.xp, Q.xc, Q.xc, Q.xc, Q.xc};
                const uint32_t ny[6] = {Q.yc, Q.yc, Q.ym, Q.yp, Q.yc, Q.yc};
                const uint32_t nz[6] = {Q.zc, Q.zc, Q.zc, Q.zc, Q.zm, Q.zp};
#pragma unroll
                for (int dd = 0; dd < 6; ++dd) {
                    const uint32_t env = (nx[dd] | ny[dd] | nz[dd]) & 0x80u;
                    const uint32_t cm = nx[dd] & ny[dd] & nz[dd] & 0x7fu;
                    if (env | cm) {
                        const int b = env ? 7 : __ffs(cm) - 1;
                        g[dd] = cut_link(g[dd], E.theta[(b * 3 + (dd >> 1)) * 2 + ((dd & 1) ? 0 : 1)]);
                        cut = true;
                    }
                }
            }
            // the move #{k : floor(u S5 / 2^32) >= S_k}: x while bit 1 is
            // clear (up when bit 0 is set), y while bit 3 is clear (up when
            // bit 2 is set), z otherwise (up when bit 4 is set)
            const uint32_t bits = step_bits(g, us[q], cut);
            const bool t2 = (bits & 2u) != 0, t4 = (bits & 8u) != 0;
            const bool ux = (bits & 1u) != 0, uy = (bits & 4u) != 0, uz = (bits & 16u) != 0;
            const bool up = (t4 & uz) | (t2 & !t4 & uy) | (!t2 & ux);
            const uint32_t sh = t4 ? 16u : (t2 ? 8u : 0u);
            ++M.s;
            co += (up ? 1u : 0xffffffffu) << sh;
            const int cnew = (int)((co >> sh) & 0xffu);
            const bool xm = !t2, ym = t2 && !t4;
            // node masks along the move's axis shift by one; the new far one
            // is read (index clamped as in mw_block_e)
            const LAS uint8_t* nrow = E.nmask + (t4 ? 2 * np : (t2 ? np : 0));
            const uint32_t ne = nrow[up ? min(cnew + 1, n) : max(cnew - 1, 0)];
            {
                const uint32_t m0 = Q.xm, c0 = Q.xc, p0 = Q.xp;
                Q.xm = xm ? (up ? c0 : ne) : m0;
                Q.xc = xm ? (up ? p0 : m0) : c0;
                Q.xp = xm ? (up ? ne : c0) : p0;
            }
            {
                const uint32_t m0 = Q.ym, c0 = Q.yc, p0 = Q.yp;
                Q.ym = ym ? (up ? c0 : ne) : m0;
                Q.yc = ym ? (up ? p0 : m0) : c0;
                Q.yp = ym ? (up ? ne : c0) : p0;
            }
            {
                const uint32_t m0 = Q.zm, c0 = Q.zc, p0 = Q.zp;
                Q.zm = t4 ? (up ? c0 : ne) : m0;
                Q.zc = t4 ? (up ? p0 : m0) : c0;
                Q.zp = t4 ? (up ? ne : c0) : p0;
            }
            if (cnew == 0 || cnew == n) {
                st = 1;
            } else {
                const uint32_t env = (Q.xc | Q.yc | Q.zc) & 0x80u;
                const uint32_t cm = Q.xc & Q.yc & Q.zc & 0x7fu;
                if (env) {
                    st = 2;
                    *net = env_net;
                } else if (cm) {
                    st = 2;
                    *net = E.cnet[__ffs(cm) - 1];
                }
            }
            // prepared masks of the two cell rows around the new node along
            // the move's axis (a walk that stopped is not stepped again)
            const int cc = min(max(cnew, 1), n - 1);
            const LAS uint16_t* rr = (t4 ? L.mask + 2 * n : (t2 ? L.mask + n : L.mask)) - 1 + cc;
            const uint32_t lo = rr[0], hi = rr[1];
            const uint32_t bgz = 1u << (15 - cc);
            const uint32_t plo = t4 ? (lo << 16) | (bgz << 1) : prep_xy(lo);
            const uint32_t phi = t4 ? (hi << 16) | bgz : prep_xy(hi);
            M.px0 = xm ? plo : M.px0;
            M.px1 = xm ? phi : M.px1;
            M.py0 = ym ? plo : M.py0;
            M.py1 = ym ? phi : M.py1;
            M.pz0 = t4 ? plo : M.pz0;
            M.pz1 = t4 ? phi : M.pz1;
        }
    }
    M.ni = (int)(co & 0xffu);
    M.nj = (int)((co >> 8) & 0xffu);
    M.nk = (int)((co >> 16) & 0xffu);
    return st;
}

// -------------------------------------------------------------------------
// Walker kernel: transitions after the first, until absorption.  A lane
// holds one walk; lanes whose next cube is not stratified run MicroWalk in
// the loop below, the others take table transitions, and the wave switches
// between the two while at least half of its working lanes walk.
// -------------------------------------------------------------------------
enum Phase : int { PH_IDLE = 0, PH_NEED = 1, PH_MW = 2, PH_EXHAUSTED = 3, PH_PARK = 4 };

// Consecutive indices handed to the lanes of a wave from a global counter,
// claimed CLAIM_CHUNK at a time: one device-scope atomic per chunk instead of
// one per refill (same-address atomics from every wave serialise).  Indices
// of a chunk are handed out in order, so a wave that stops taking work has
// used every index below the first invalid one it saw.  Call at points where
// the whole wave is active; state is wave-uniform.
constexpr uint32_t CLAIM_CHUNK = 64;

struct WaveClaim {
    unsigned long long base = 0;
    uint32_t left = 0;

    // One index for every lane of `want` (returned to those lanes).
    __device__ __forceinline__ unsigned long long take(unsigned long long* counter, uint64_t want, int lane) {
        const uint32_t cnt = __popcll(want);
        const uint32_t rank = __popcll(want & ((1ull << lane) - 1ull));
        unsigned long long idx = ~0ull;
        uint32_t served = 0;
        while (served < cnt) {
            if (left == 0) {
                unsigned long long b = 0;
                if (lane == 0) b = atomicAdd(counter, (unsigned long long)CLAIM_CHUNK);
                base = __shfl(b, 0);
                left = CLAIM_CHUNK;
            }
            const uint32_t n = min(cnt - served, left);
            if (rank >= served && rank < served + n) idx = base + (rank - served);
            base += n;
            left -= n;
            served += n;
        }
        return idx;
    }
};

// The structure a walker lane reads: the launch's copy for one segment, the
// lane's segment's otherwise.
template <bool MULTI>
__device__ __forceinline__ decltype(auto) walk_struct(const WalkArgs& A, const GAS Segment& SG) {
    if constexpr (MULTI)
        return *gp(SG.S);
    else
        return (A.S0);
}

// EXP: MicroWalk hops use expanded cubes (MicroWalk-E).
// N16: ordinary MicroWalk reads cell codes as cell_code16 (n <= 16; on
// the cell lattice n <= 15, with the row masks in registers).
// CELL: every cube on the cell-centred lattice (n odd; plain MicroWalk).
template <bool MULTI, bool EXP, bool N16 = false, bool CELL = false>
// three resident waves per SIMD (at most 168 VGPRs) for the plain MicroWalk
// kernels, whose LDS allows 11 waves per compute unit; two for MicroWalk-E
__global__ void __launch_bounds__(WALK_THREADS) __attribute__((amdgpu_waves_per_eu(EXP ? 2 : 3)))
frw_walk_kernel(WalkArgs A) {
    static_assert(!(CELL && EXP), "the cell lattice runs plain MicroWalk steps of its own");
    extern __shared__ uint32_t lds[];
    const int n = A.n;
    const int ns = CELL ? n + 1 : n;  // mask row stride
    const int lane = threadIdx.x & 63;
    // a launch with no parked walk to resume and no fresh walk left (a
    // device-driven round after a run that finished) ends at once
    if (A.ctr->launch_idle) return;
    uint32_t* my = lds + threadIdx.x * A.lane_stride;
    const LaneCube L = lane_cube(my, ns);
    const LaneExp E = lane_exp(my, n);  // used by EXP kernels only

    Counters& K = *A.ctr;
    unsigned long long c_hops = 0, c_steps = 0, c_cls[3] = {0, 0, 0}, c_env = 0, c_cap = 0, c_halved = 0;
    uint32_t err = 0;
    // one structure per launch: its layer table goes to LDS once
    uint32_t* lt_lds = lds + WALK_THREADS * A.lane_stride;
    const uint32_t* lt = nullptr;
    if (!MULTI) {
        const StructDev& S0 = A.S0;
        if (S0.n_layers <= LAYER_LDS) {
            if (threadIdx.x < 2 * LAYER_LDS) {
                const int q = min((int)(threadIdx.x % LAYER_LDS), S0.n_layers - 1);
                lt_lds[threadIdx.x] = threadIdx.x < LAYER_LDS ? __float_as_uint(gp(S0.layer_z0)[q])
                                                              : gp(CELL ? S0.layer_eps : S0.layer_code)[q];
            }
            lt = lt_lds;
        }
        __syncthreads();
    }

    // the parked walks this launch resumes (set by the kernel before it)
    const uint32_t n_resume = K.resume_count;
    const bool side1 = (K.resume_side & 1u) != 0u;
    const Parked* resume = side1 ? A.park[1] : A.park[0];
    Parked* park_out = side1 ? A.park[0] : A.park[1];

    int phase = PH_IDLE;
    WaveClaim claim_rc, claim_fr;  // wave-level claims of resumed and fresh walks
    bool resume_done = false;
    int sg = 0;  // segment of the lane's walk (always 0 for one segment)
    uint32_t wk0 = 0, wk1 = 0;  // the walk's Philox key (its segment's seed)
    unsigned long long walk = 0;
    float3 pos = make_float3(0.f, 0.f, 0.f);
    float omega = 0.f;
    uint32_t t = 0;
    // MicroWalk state
    float3 mc = pos;
    float mR = 0.f;
    MwState M{};
    MwStateE Q{};
    CellRows CR{};  // CELL kernels only
    int env_net = 0;

    for (;;) {
        // ---- walks that park for the next launch: in the plain form after
        // each transition, and fresh walks whose first transition is still
        // missing (t = 0); one queue slot range claimed per wave ----
        {
            const uint64_t bp = __ballot(phase == PH_PARK);
            if (bp) {
                uint32_t base = 0;
                if (lane == 0) base = atomicAdd(&K.park_count, (uint32_t)__popcll(bp));
                base = __shfl(base, 0);
                if (phase == PH_PARK) {
                    const uint32_t slot = base + (uint32_t)__popcll(bp & ((1ull << lane) - 1ull));
                    if (slot < A.park_cap) {
                        Parked P;
                        P.walk = walk;
                        P.px = pos.x;
                        P.py = pos.y;
                        P.pz = pos.z;
                        P.omega = omega;
                        P.t = t;
                        P.seg = sg;
                        stpark(park_out + slot, P);
                    } else {
                        err |= ERR_PARK_CAP;
                    }
                    phase = PH_IDLE;
                }
            }
        }
        // ---- take work: resumed walks first, then fresh walk ids ----
        {
            const uint64_t bal = __ballot(phase == PH_IDLE);
            if (bal) {
                bool got = false;
                if (n_resume && !resume_done) {
                    const unsigned long long ri = claim_rc.take(&K.resume_next, bal, lane);
                    if (phase == PH_IDLE) {
                        if (ri < n_resume) {
                            const Parked P = ldpark(resume + ri);
                            if (MULTI) sg = P.seg;
                            const GAS Segment& SG = gp(A.segs)[sg];
                            wk0 = SG.k0;
                            wk1 = SG.k1;
                            walk = P.walk;
                            phase = PH_NEED;
                            if (P.t == 0u) {
                                // parked before its first transition existed:
                                // start from it now, or park again while it
                                // is still missing
                                const unsigned long long k = walk - SG.walk_begin;
                                const float4 f = ldf4(SG.first_state + k);
                                pos = make_float3(f.x, f.y, f.z);
                                omega = f.w;
                                t = 1;
                                if (!gp(SG.first_done)[k]) {
                                    t = 0;
                                    phase = PH_PARK;
                                }
                            } else {
                                pos = make_float3(P.px, P.py, P.pz);
                                omega = P.omega;
                                t = P.t;
                            }
                            got = true;
                        }
                    }
                    resume_done = claim_rc.base >= n_resume;
                }
                const uint64_t bal2 = __ballot(phase == PH_IDLE && !got);
                if (bal2) {
                    const unsigned long long gi = claim_fr.take(&K.walk_next, bal2, lane);
                    if (phase == PH_IDLE && !got) {
                        if (gi < A.total) {
                            if (MULTI) sg = find_segment(A.segs, A.n_segs, gi);
                            const GAS Segment& SG = gp(A.segs)[sg];
                            wk0 = SG.k0;
                            wk1 = SG.k1;
                            const unsigned long long k = gi - SG.offset;
                            const float4 f = ldf4(SG.first_state + k);
                            const uint32_t fdone = gp(SG.first_done)[k];
                            walk = SG.walk_begin + k;
                            pos = make_float3(f.x, f.y, f.z);
                            omega = f.w;
                            t = fdone ? 1u : 0u;
                            // a walk whose first transition missed its table
                            // waits in the park queue (t = 0)
                            phase = fdone ? PH_NEED : PH_PARK;
                        } else {
                            phase = PH_EXHAUSTED;
                        }
                    }
                }
            }
        }
        // (a lane about to park keeps the loop going: the next pass parks it)
        if (!__any(phase == PH_NEED || phase == PH_MW || phase == PH_PARK)) break;

        // ---- one transition for lanes that need one ----
        if (phase == PH_NEED) {
            const GAS Segment& SG = gp(A.segs)[sg];
            auto& S = walk_struct<MULTI>(A, SG);
            bool park = false, done = false;
            int net = S.n_nets;
            float3 c;
            float R;
            float3 x;
            int cell;
            float dq;  // conductor-free half-size before the cube-size rule
            uint2 drange;
            {
                cell = grid_cell(S, pos);
                // the cell's dielectric candidate range, read with the
                // conductor candidates
                drange = make_uint2(gp(S.gd_off)[cell], gp(S.gd_off)[cell + 1]);
                R = query_dist(S, pos, cell, &net);
                dq = R;
                c = pos;
                if (R <= S.delta_abs) {
                    done = true;
                } else if (t > HOP_CAP) {
                    done = true;
                    net = S.n_nets;
                    ++c_cap;
                }
            }
            if (!done) {
                CubeInfo I = build_cube<CELL>(S, cell, c, R, n, L, false, lt, &drange);
                const bool halved = I.overflow;
                for (int it = 0; it < 40 && I.overflow; ++it) {
                    R *= 0.5f;  // capacity rule: halve while more than 16 boxes touch
                    I = build_cube<CELL>(S, cell, c, R, n, L, false, lt, &drange);
                }
                if (I.overflow) {
                    // more than 16 boxes overlap at this point: the call fails
                    err |= ERR_REGIONS;
                    I.cls = 0;
                    I.axis = 2;
                }
                const float h = 2.f * R / (float)n;
                {
                    ++c_hops;
                    ++c_cls[I.cls];
                    if (A.hybrid && I.cls <= 1) {
                        const int sax = I.axis;
                        // hop table key: (0, n, axis, 0, plane codes), or
                        // (2, n, axis, 0, plane permittivities) on the cell
                        // lattice; every uniform cube shares one table
                        uint32_t idx = A.uniform_index;
                        int res = LOOKUP_HIT;
                        const Rand4 r = philox10(0u, t, (uint32_t)walk, ctr_hi(walk, PURPOSE_TABLE), wk0, wk1);
                        uint32_t glo = 0, ghi = 0;
                        if (I.cls != 0) {
                            // plane codes written once over the background
                            // codes (the cube is not used after this hop),
                            // hashed as they are formed
                            uint32_t hsh = KEY_HASH_SEED;
                            hsh = key_hash_step(hsh, CELL ? 2u : 0u);
                            hsh = key_hash_step(hsh, (uint32_t)n);
                            hsh = key_hash_step(hsh, (uint32_t)sax);
                            hsh = key_hash_step(hsh, 0u);
                            const uint32_t b0 = L.bz[0];
                            if (!CELL && n == 16) {
                                // eight planes at a time: their mask words,
                                // background codes and box codes each in one
                                // LDS round trip
                                const LAS uint32_t* row = reinterpret_cast<const LAS uint32_t*>(L.mask) + sax * 8;
#pragma unroll
                                for (int p0 = 0; p0 < 16; p0 += 8) {
                                    uint32_t mw[4], bq[8], pc[8];
#pragma unroll
                                    for (int j = 0; j < 4; ++j) mw[j] = row[p0 / 2 + j];
#pragma unroll
                                    for (int j = 0; j < 8; ++j) bq[j] = sax == 2 ? L.bz[p0 + j] : b0;
#pragma unroll
                                    for (int j = 0; j < 8; ++j)
                                        pc[j] = cell_code(
                                            L, ((j & 1) ? mw[j / 2] >> 16 : mw[j / 2] & 0xffffu) & I.present, bq[j]);
#pragma unroll
                                    for (int j = 0; j < 8; ++j) {
                                        L.bz[p0 + j] = pc[j];
                                        hsh = key_hash_step(hsh, pc[j]);
                                    }
                                }
                            } else {
#pragma unroll 4
                                for (int p = 0; p < n; ++p) {
                                    const uint32_t pc =
                                        cell_code(L, L.mask[sax * ns + p] & I.present, sax == 2 ? L.bz[p] : b0);
                                    L.bz[p] = pc;
                                    hsh = key_hash_step(hsh, pc);
                                }
                            }
                            static_assert(KEY_HDR == 4, "hop-table key header is four words");
                            res = lookup_or_insert(
                                A.cache,
                                [&](uint32_t q) {
                                    if (CELL && q == 0) return 2u;
                                    return q == 1 ? (uint32_t)n
                                                  : (q == 2 ? (uint32_t)sax : (q < KEY_HDR ? 0u : L.bz[q - KEY_HDR]));
                                },
                                hsh, &idx, r.x, &glo, &ghi);
                        }
                        if (res != LOOKUP_HIT) {
                            if (res == LOOKUP_FULL) err |= ERR_TABLE_CAP;
                            park = true;
                            --c_hops;
                            --c_cls[I.cls];
                        } else {
                            c_halved += halved ? 1ull : 0ull;
                            const GAS uint32_t* tab = gp(A.cache.data) + (size_t)idx * A.cache.tab_words;
                            if (I.cls == 0) {
                                // the uniform table's guide pair (read with the key otherwise)
                                glo = tab[TAB_GUIDE + (r.x >> GUIDE_SHIFT)];
                                ghi = tab[TAB_GUIDE + (r.x >> GUIDE_SHIFT) + 1];
                            }
                            const int b = table_sample_guided(tab, A.cache.nb, r.x, glo, ghi);
                            if (CELL) {
                                int ci, cj, ck;
                                cell_panel_of_hit(n, b, &ci, &cj, &ck);
                                x = cell_exit_point(c, R, h, n, ci, cj, ck);
                            } else {
                                int nd[3];
                                node_of_hit(n, b, nd);
                                x = make_float3(c.x - R + (float)nd[0] * h, c.y - R + (float)nd[1] * h,
                                                c.z - R + (float)nd[2] * h);
                            }
                            pos = fold3(S, x);
                            ++t;
                            if (A.plain) phase = PH_PARK;
                        }
                    } else {
                        // MicroWalk from the centre node
                        mc = c;
                        mR = R;
                        phase = PH_MW;
                        if (EXP) {
                            // MicroWalk-E: the cube grows to n dq / (2 m)
                            // and may hold conductors; halved (not below
                            // dq) while it holds too many boxes or
                            // conductors, then by the ordinary rule
                            int it0;
                            bool marked;
                            unsigned long long mdiel, mcond;
                            const float Rx = expanded_size(S, c, dq, n, A.expand_m);
                            float Re = exp_fit(S, cell, c, Rx, dq, &it0, &marked, &mdiel, &mcond);
                            bool ok = false;
                            for (int it = it0;; ++it) {
                                // the marks describe the first size only
                                const bool mk = marked && it == it0;
                                const CubeInfo IE = build_cube(S, cell, c, Re, n, L, true, lt, nullptr, mk, mdiel);
                                ok = !IE.overflow && build_conductors(S, cell, c, Re, n, E, mk, mcond);
                                if (ok || it >= 110) break;
                                Re = Re > dq ? fmaxf(0.5f * Re, dq) : 0.5f * Re;
                            }
                            if (!ok) err |= ERR_REGIONS;
                            c_halved += Re < Rx ? 1ull : 0ull;
                            mR = Re;
                            env_net = S.n_nets;
                            if (N16)
                                mw_begin16(M, L, n);
                            else
                                mw_begin(M, L, n);
                            mw_begin_e(M, Q, E, n);
                        } else if (CELL) {
                            c_halved += halved ? 1ull : 0ull;
                            if (N16)
                                mw_begin_cell16(M, CR, L, n);
                            else
                                mw_begin_cell(M, CR, L, n);
                        } else if (N16) {
                            c_halved += halved ? 1ull : 0ull;
                            mw_begin16(M, L, n);
                        } else {
                            c_halved += halved ? 1ull : 0ull;
                            mw_begin(M, L, n);
                        }
                    }
                }
            }
            if (done) {
                const unsigned long long k = walk - SG.walk_begin;
                if (net == S.n_nets) ++c_env;
                gpw(SG.score_net)[k] = net;
                gpw(SG.score_w)[k] = omega;
                phase = PH_IDLE;
            } else if (park) {
                const uint32_t slot = atomicAdd(&K.park_count, 1u);
                if (slot < A.park_cap) {
                    Parked P;
                    P.walk = walk;
                    P.px = pos.x;
                    P.py = pos.y;
                    P.pz = pos.z;
                    P.omega = omega;
                    P.t = t;
                    P.seg = sg;
                    stpark(park_out + slot, P);
                } else {
                    err |= ERR_PARK_CAP;
                }
                phase = PH_IDLE;
            }
        }

        // ---- MicroWalk steps, four per Philox block, while enough lanes walk ----
        for (;;) {
            const uint64_t balmw = __ballot(phase == PH_MW);
            const uint64_t balact = __ballot(phase == PH_MW || phase == PH_NEED || phase == PH_IDLE);
            const int nmw = __popcll(balmw), nact = __popcll(balact);
            if (nmw == 0 || 2 * nmw < nact) break;
            if (phase == PH_MW) {
                const GAS Segment& SG = gp(A.segs)[sg];
                int anet = 0;
                int stt;
                if (EXP) {
                    const Rand4 r = philox10(M.s >> 2, t, (uint32_t)walk, ctr_hi(walk, PURPOSE_MICROWALK), wk0, wk1);
                    stt = N16 ? mw_block_e16(M, Q, L, E, n, r, env_net, &anet)
                              : mw_block_e(M, Q, L, E, n, r, env_net, &anet);
                } else {
                    // two Philox blocks per pass (eight steps); the second
                    // block's counter is the one it would have after four
                    // steps, so the words are those of one block at a time
                    const uint32_t b0 = M.s >> 2;
                    const Rand4 r0 = philox10(b0, t, (uint32_t)walk, ctr_hi(walk, PURPOSE_MICROWALK), wk0, wk1);
                    const Rand4 r1 = philox10(b0 + 1, t, (uint32_t)walk, ctr_hi(walk, PURPOSE_MICROWALK), wk0, wk1);
                    bool in;
                    if (CELL && N16) {
                        in = mw_block_cell16(M, CR, L, n, r0);
                        if (in) in = mw_block_cell16(M, CR, L, n, r1);
                    } else if (CELL) {
                        in = mw_block_cell(M, CR, L, n, r0);
                        if (in) in = mw_block_cell(M, CR, L, n, r1);
                    } else if (N16) {
                        in = mw_block16(M, L, n, r0);
                        if (in) in = mw_block16(M, L, n, r1);
                    } else {
                        in = mw_block(M, L, n, r0);
                        if (in) in = mw_block(M, L, n, r1);
                    }
                    stt = in ? 0 : 1;
                }
                bool alive = stt == 0;
                if (alive && M.s >= MW_STEP_CAP) {
                    // never reached for valid permittivities; keeps a logic
                    // error from spinning: the walk ends where it stands and
                    // the call reports MW_ELIMIT
                    err |= ERR_STEP_CAP;
                    alive = false;
                }
                if (EXP && stt == 2) {
                    // MicroWalk-E reached a conductor or the grounded enclosure
                    c_steps += M.s;
                    const unsigned long long k = walk - SG.walk_begin;
                    if (anet == env_net) ++c_env;
                    gpw(SG.score_net)[k] = anet;
                    gpw(SG.score_w)[k] = omega;
                    phase = PH_IDLE;
                } else if (!alive) {
                    c_steps += M.s;
                    const float h = 2.f * mR / (float)n;
                    const float3 xx = CELL ? cell_exit_point(mc, mR, h, n, M.ni, M.nj, M.nk)
                                           : make_float3(mc.x - mR + (float)M.ni * h, mc.y - mR + (float)M.nj * h,
                                                         mc.z - mR + (float)M.nk * h);
                    pos = fold3(walk_struct<MULTI>(A, SG), xx);
                    ++t;
                    phase = A.plain ? PH_PARK : PH_NEED;
                }
            }
        }
    }

    // ---- counters ----
    auto wsum = [&](unsigned long long v) {
        for (int off = 32; off > 0; off >>= 1) v += __shfl_down(v, off);
        return v;
    };
    c_hops = wsum(c_hops);
    c_steps = wsum(c_steps);
    for (int q = 0; q < 3; ++q) c_cls[q] = wsum(c_cls[q]);
    c_env = wsum(c_env);
    c_cap = wsum(c_cap);
    c_halved = wsum(c_halved);
    for (int off = 32; off > 0; off >>= 1) err |= __shfl_down(err, off);
    if (lane == 0) {
        if (c_hops) atomicAdd(&K.hops, c_hops);
        if (c_steps) atomicAdd(&K.micro_steps, c_steps);
        for (int q = 0; q < 3; ++q)
            if (c_cls[q]) atomicAdd(&K.hop_class[q], c_cls[q]);
        if (c_env) atomicAdd(&K.env, c_env);
        if (c_cap) atomicAdd(&K.hop_cap, c_cap);
        if (c_halved) atomicAdd(&K.halved, c_halved);
        if (err) atomicOr(&K.err, err);
    }
}

// -------------------------------------------------------------------------
// Exact SGF tables of stratified cubes (binary64).  In a cube stratified
// along w the vertex-lattice operator is separable: the in-plane part is the
// Dirichlet second difference scaled per plane, which the orthonormal sine
// transform diagonalises, leaving one tridiagonal system along w per pair of
// in-plane modes.  This is the discrete counterpart of the analytic SGF of
// stratified cubes (Table I: O(N^3)-class work on a cache miss).
// -------------------------------------------------------------------------
constexpr int TB_THREADS = 256;

struct BuildArgs {
    CacheDev cache;
    const uint32_t* list;  // table indices to build
    uint32_t count;
    double* work;          // per block: 3 M^3 + 3 nb doubles
    size_t work_stride;    // doubles per block
    // device-driven rounds: the list is the cache's queue and its length
    // is read here (blocks past it, and every block once the rounds handed
    // over to the host, do nothing)
    const uint32_t* dev_count;
    const Counters* ctr;
};

// Storage of one table build: the per-source mode columns (global work
// space), and in LDS the sine basis, eigenvalues, plane coefficients, a
// matrix product buffer and the CDF chunk sums.
struct BuildSpace {
    double* zh;    // [src][r][m][l] mode columns, then [src][nb] exit rows (3 M^3 + 4 nb doubles)
    double* Sm;    // 31 x 31
    double* lam;   // 32
    double* cr;    // 33
    double* ar;    // 33
    double* br;    // 33
    double* tmp;   // 31 x 31
    double* csum;  // TB_THREADS
    int* clast;    // TB_THREADS
    double* total;
    int* last;
};

// Exact SGF table idx of the cache, built by a group of NT threads (thread
// tid) that call sync() between phases.  Every value is computed by one
// thread in a fixed order and the CDF is cut into TB_THREADS chunks, so the
// table does not depend on how the work is spread over the threads.  The
// table's ready word receives ready_value.
template <int NT, class Sync>
__device__ void build_table_body(const CacheDev& C, uint32_t idx, int tid, const BuildSpace& W, Sync sync,
                                 uint32_t ready_value) {
    const uint32_t* key = C.keys + (size_t)idx * C.key_stride;
    const int kind = (int)key[0], n = (int)key[1], s = (int)key[2], anorm = (int)key[3];
    // kind: bit 0 first transition, bit 1 cell-centred lattice.  Vertex
    // lattice: M = n - 1 interior nodes per axis, Dirichlet sine basis.  Cell
    // lattice (n odd): M = n cells per axis; the boundary panel sits half a
    // cell away, which doubles the last in-plane link and makes the in-plane
    // operator the one the DST-II basis sin(pi (m + 1) (p + 1/2) / n)
    // diagonalises (eigenvalues 2 - 2 cos(pi (m + 1) / n)).
    const bool first = (kind & 1) != 0, cellk = (kind & 2) != 0;
    const int M = cellk ? n : n - 1, M2 = M * M, nb = 6 * M2;
    double* Sm = W.Sm;
    double* lam = W.lam;
    double* cr = W.cr;
    double* ar = W.ar;
    double* br = W.br;
    double* tmp = W.tmp;
    double* zh = W.zh;
    double* Pout = zh + (size_t)3 * M * M2;  // [src][nb]
    if (!cellk) {
        const double norm = sqrt(2.0 / (double)(M + 1));
        for (int q = tid; q < M2; q += NT) {
            const int m = q / M + 1, p = q % M + 1;
            Sm[q] = norm * sin(M_PI * (double)(m * p) / (double)(M + 1));
        }
        if (tid < M) lam[tid] = 2.0 - 2.0 * cos(M_PI * (double)(tid + 1) / (double)(M + 1));
        if (tid >= 1 && tid <= M) {
            const int r = tid;
            const double em = (double)key[KEY_HDR + r - 1], ep = (double)key[KEY_HDR + r];
            cr[r] = 2.0 * (em + ep);
            ar[r] = 4.0 * em;
            br[r] = 4.0 * ep;
        }
    } else {
        // Sm[mode * M + cell]; the last mode is normalised by sqrt(1 / n)
        for (int q = tid; q < M2; q += NT) {
            const int m = q / M, p = q % M;
            const double norm = sqrt((m == M - 1 ? 1.0 : 2.0) / (double)M);
            Sm[q] = norm * sin(M_PI * (double)(m + 1) * ((double)p + 0.5) / (double)M);
        }
        if (tid < M) lam[tid] = 2.0 - 2.0 * cos(M_PI * (double)(tid + 1) / (double)M);
        if (tid >= 1 && tid <= M) {
            // plane r (1-based): in-plane links 2^23 (equal permittivities),
            // Eq. (6) codes to the planes below and above, 2^24 to a panel
            const int r = tid;
            const double ev = (double)__uint_as_float(key[KEY_HDR + r - 1]);
            cr[r] = 8388608.0;
            if (r == 1) {
                ar[r] = 16777216.0;
            } else {
                const double e = (double)__uint_as_float(key[KEY_HDR + r - 2]);
                ar[r] = key[KEY_HDR + r - 2] == key[KEY_HDR + r - 1] ? 8388608.0 : rint(e / (e + ev) * 16777216.0);
            }
            if (r == M) {
                br[r] = 16777216.0;
            } else {
                const double e = (double)__uint_as_float(key[KEY_HDR + r]);
                br[r] = key[KEY_HDR + r] == key[KEY_HDR + r - 1] ? 8388608.0 : rint(e / (e + ev) * 16777216.0);
            }
        }
    }
    sync();
    // local frame: w = s, (u, v) the other two axes ascending
    const int ua = s == 0 ? 1 : 0, va = s == 2 ? 1 : 2;
    const int c0 = cellk ? (n - 1) / 2 + 1 : n / 2;  // centre node or cell, 1-based
    int src[3][3];
    int nsrc = first ? 3 : 1;
    for (int q = 0; q < 3; ++q) src[q][0] = src[q][1] = src[q][2] = c0;  // (p, q, r) local
    if (first) {
        const int lax = anorm == s ? 2 : (anorm == ua ? 0 : 1);
        src[1][lax] += 1;
        src[2][lax] -= 1;
    }
    // tridiagonal solves, one (m, l) mode pair per thread
    double cvals[32], dvals[32];
    for (int sidx = 0; sidx < nsrc; ++sidx) {
        const int p0 = src[sidx][0], q0 = src[sidx][1], r0 = src[sidx][2];
        for (int ml = tid; ml < M2; ml += NT) {
            const int m = ml / M, l = ml % M;  // 0-based modes
            const double lm = lam[m] + lam[l];
            const double rhs0 = Sm[m * M + (p0 - 1)] * Sm[l * M + (q0 - 1)];
            double* col = zh + (size_t)sidx * M * M2 + ml;  // stride M2 over r
            // Thomas algorithm: forward elimination, then back substitution.
            // The cell lattice's codes are not symmetric: its row of
            // (D - G)^-1 solves the transposed system, whose off-diagonals
            // are the neighbours' codes towards plane r.
            double cprev = 0.0, dprev = 0.0;
            #pragma unroll 1
            for (int r = 1; r <= M; ++r) {
                const double diag = cr[r] * lm + ar[r] + br[r];
                const double sub = r > 1 ? -(cellk ? br[r - 1] : ar[r]) : 0.0;
                const double sup = r < M ? -(cellk ? ar[r + 1] : br[r]) : 0.0;
                const double den = diag - sub * cprev;
                cvals[r] = sup / den;
                dvals[r] = ((r == r0 ? rhs0 : 0.0) - sub * dprev) / den;
                cprev = cvals[r];
                dprev = dvals[r];
            }
            double xnext = dvals[M];
            col[(size_t)(M - 1) * M2] = xnext;
            #pragma unroll 1
            for (int r = M - 1; r >= 1; --r) {
                const double xr = dvals[r] - cvals[r] * xnext;
                col[(size_t)(r - 1) * M2] = xr;
                xnext = xr;
            }
        }
    }
    sync();
    // exit probabilities on the six faces, in global hit-index order
    // (coordinates of boundary nodes 1..M on the vertex lattice, of the
    // cells next to a panel 0..M-1 on the cell lattice)
    const int o1 = cellk ? 0 : 1;
    for (int sidx = 0; sidx < nsrc; ++sidx) {
        const double* Z = zh + (size_t)sidx * M * M2;  // Z[(r-1)*M2 + m*M + l]
        double* P = Pout + (size_t)sidx * nb;
        // w faces: r = 1 (side 0, link ar[1]) and r = M (side 1, link br[M])
        for (int side = 0; side < 2; ++side) {
            const int r = side ? M : 1;
            const double link = side ? br[M] : ar[1];
            const double* Zr = Z + (size_t)(r - 1) * M2;
            // Y[m][q] = sum_l Z[m][l] S[l][q]
            for (int e = tid; e < M2; e += NT) {
                const int m = e / M, qq = e % M;
                double acc = 0.0;
                // unrolled so that the global loads of Z issue together (the
                // sum keeps its order)
                #pragma unroll 8
                for (int l = 0; l < M; ++l) acc += Zr[m * M + l] * Sm[l * M + qq];
                tmp[e] = acc;
            }
            sync();
            for (int e = tid; e < M2; e += NT) {
                const int p = e / M, qq = e % M;  // 0-based local coords p-1, q-1
                double acc = 0.0;
                #pragma unroll 1
                for (int m = 0; m < M; ++m) acc += Sm[m * M + p] * tmp[m * M + qq];
                int g[3];
                g[ua] = p + o1;
                g[va] = qq + o1;
                g[s] = side ? n : 0;
                const int f = 2 * s + side;
                const int oa = s == 0 ? 1 : 0, ob = s == 2 ? 1 : 2;
                P[f * M2 + (g[ob] - o1) * M + (g[oa] - o1)] = link * acc;
            }
            sync();
        }
        // u faces (p = 1 or M) and v faces (q = 1 or M)
        for (int which = 0; which < 4; ++which) {
            const bool ufaces = which < 2;
            const int side = which & 1;
            const int fixed = side ? M - 1 : 0;  // 0-based
            // X[l][r] = sum_m S[m][fixed] Z[r][m][l]  (u faces)
            // X[m][r] = sum_l S[l][fixed] Z[r][m][l]  (v faces)
            for (int e = tid; e < M2; e += NT) {
                const int j = e / M, r = e % M;
                const double* Zr = Z + (size_t)r * M2;
                double acc = 0.0;
                if (ufaces)
                    #pragma unroll 8
                    for (int m = 0; m < M; ++m) acc += Sm[m * M + fixed] * Zr[m * M + j];
                else
                    #pragma unroll 8
                    for (int l = 0; l < M; ++l) acc += Sm[l * M + fixed] * Zr[j * M + l];
                tmp[e] = acc;
            }
            sync();
            for (int e = tid; e < M2; e += NT) {
                const int other = e / M, r = e % M;  // other: q (u faces) or p (v faces), 0-based
                double acc = 0.0;
                #pragma unroll 1
                for (int j = 0; j < M; ++j) acc += Sm[j * M + other] * tmp[j * M + r];
                int g[3];
                const int fa = ufaces ? ua : va;
                g[s] = r + o1;
                if (ufaces) {
                    g[ua] = side ? n : 0;
                    g[va] = other + o1;
                } else {
                    g[va] = side ? n : 0;
                    g[ua] = other + o1;
                }
                const int f = 2 * fa + side;
                const int oa = fa == 0 ? 1 : 0, ob = fa == 2 ? 1 : 2;
                // the in-plane link into a panel: 2^24 on the cell lattice
                const double link = cellk ? 2.0 * cr[r + 1] : cr[r + 1];
                P[f * M2 + (g[ob] - o1) * M + (g[oa] - o1)] = link * acc;
            }
            sync();
        }
    }
    sync();
    // weights -> CDF (one thread: sequential prefix sum in hit-index order)
    uint32_t* tab = C.data + (size_t)idx * C.tab_words;
    if (first) {
        // flux kernel of the first transition along +anorm (Sec. II-A weight):
        // w_b = [G+ (P^c - P^+) + G- (P^- - P^c)] / 2, in units of 1/h, with
        // G+- the permittivity of the links from the centre along +-anorm
        // (cell lattice: the series combination of the two half cells)
        double Gp, Gm;
        if (cellk) {
            const int cc = c0 - 1;  // centre plane, 0-based
            const double ec = (double)__uint_as_float(key[KEY_HDR + cc]);
            if (anorm == s) {
                const double ep = (double)__uint_as_float(key[KEY_HDR + cc + 1]);
                const double em = (double)__uint_as_float(key[KEY_HDR + cc - 1]);
                Gp = 2.0 * ec * ep / (ec + ep);
                Gm = 2.0 * ec * em / (ec + em);
            } else {
                Gp = Gm = ec;
            }
        } else {
            const double e0 = (double)key[KEY_HDR + c0 - 1], e1 = (double)key[KEY_HDR + c0];
            if (anorm == s) {
                Gp = e1 / 65536.0;
                Gm = e0 / 65536.0;
            } else {
                Gp = Gm = (e0 + e1) / (2.0 * 65536.0);
            }
        }
        const double* Pc = Pout;
        const double* Pp = Pout + nb;
        const double* Pm = Pout + 2 * nb;
        for (int b = tid; b < nb; b += NT) {
            const double w = 0.5 * (Gp * (Pc[b] - Pp[b]) + Gm * (Pm[b] - Pc[b]));
            Pout[3 * nb + b] = w;  // stored after the three rows (workspace sized for it)
        }
        sync();
        for (int q = tid; q < (nb + 31) / 32; q += NT) {
            uint32_t bits = 0;
            for (int k = 0; k < 32 && q * 32 + k < nb; ++k)
                if (Pout[3 * nb + q * 32 + k] > 0.0) bits |= 1u << k;
            tab[TAB_CDF + nb + q] = bits;
        }
    }
    // weights -> CDF in hit-index order: each of TB_THREADS chunks is summed
    // by one thread, one thread scans the chunk sums, every chunk then
    // writes its thresholds ceil(cum / total * 2^32) (the last equals 2^32
    // exactly: the chunk sums are formed in the same order)
    const double* wv = first ? Pout + 3 * nb : Pout;
    const bool absw = first;
    const int chunk = (nb + TB_THREADS - 1) / TB_THREADS;
    for (int ch = tid; ch < TB_THREADS; ch += NT) {
        const int b0 = ch * chunk, b1 = min(nb, b0 + chunk);
        double sloc = 0.0;
        int last = -1;
        for (int b = b0; b < b1; ++b) {
            const double v = absw ? fabs(wv[b]) : wv[b];
            sloc += v;
            if (v > 0.0) last = b;
        }
        W.csum[ch] = sloc;
        W.clast[ch] = last;
    }
    sync();
    if (tid == 0) {
        double run = 0.0;
        int last = 0;
        for (int t = 0; t < TB_THREADS; ++t) {
            const double c = W.csum[t];
            W.csum[t] = run;  // exclusive prefix
            run += c;
            if (W.clast[t] >= 0) last = W.clast[t];
        }
        *W.total = run;
        *W.last = last;
    }
    sync();
    const double tot = *W.total;
    for (int ch = tid; ch < TB_THREADS; ch += NT) {
        const int b0 = ch * chunk, b1 = min(nb, b0 + chunk);
        const double off = W.csum[ch];
        double loc = 0.0;
        for (int b = b0; b < b1; ++b) {
            loc += absw ? fabs(wv[b]) : wv[b];
            const double cv = ceil((off + loc) / tot * 4294967296.0);
            tab[TAB_CDF + b] = cv >= 4294967295.0 ? 0xffffffffu : (uint32_t)cv;
        }
    }
    if (tid == 0) {
        tab[0] = (uint32_t)*W.last;
        tab[1] = first ? __float_as_uint((float)tot) : 0u;
    }
    sync();
    // guide[g] = first b with CDF[b] > g * 2^GUIDE_SHIFT (CDF nondecreasing):
    // entry b is the answer exactly for CDF[b-1] <= g 2^GUIDE_SHIFT < CDF[b]
    // (CDF[-1] = 0), and nb for g 2^GUIDE_SHIFT >= CDF[nb-1]; each entry
    // writes its own range of g (two loads per entry instead of a bisection
    // per g)
    const unsigned long long gstep = 1ull << GUIDE_SHIFT;
    for (int b = tid; b < nb; b += NT) {
        const unsigned long long lo = b ? tab[TAB_CDF + b - 1] : 0ull, hi = tab[TAB_CDF + b];
        const int g0 = (int)((lo + gstep - 1) >> GUIDE_SHIFT), g1 = (int)((hi + gstep - 1) >> GUIDE_SHIFT);
        for (int g = g0; g < g1; ++g) tab[TAB_GUIDE + g] = (uint32_t)b;
    }
    {
        const unsigned long long last = tab[TAB_CDF + nb - 1];
        for (int g = (int)((last + gstep - 1) >> GUIDE_SHIFT) + tid; g <= (1 << GUIDE_BITS); g += NT)
            tab[TAB_GUIDE + g] = (uint32_t)nb;
    }
    sync();
    if (tid == 0) {
        __threadfence();
        __hip_atomic_store(C.ready + idx, ready_value, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    }
}

__global__ void __launch_bounds__(TB_THREADS) build_tables_kernel(BuildArgs B) {
    if (B.dev_count && (B.ctr->dev_stop || blockIdx.x >= *B.dev_count)) return;
    const uint32_t idx = B.list[blockIdx.x];
    if (idx >= B.cache.capacity) return;  // a queue entry of a full cache
    __shared__ double Sm[31 * 31];
    __shared__ double lam[32];
    __shared__ double cr[33], ar[33], br[33];
    __shared__ double tmp[31 * 31];
    __shared__ double csum[TB_THREADS];
    __shared__ int clast[TB_THREADS];
    __shared__ double total_sh;
    __shared__ int last_sh;
    BuildSpace W;
    W.zh = B.work + (size_t)blockIdx.x * B.work_stride;
    W.Sm = Sm;
    W.lam = lam;
    W.cr = cr;
    W.ar = ar;
    W.br = br;
    W.tmp = tmp;
    W.csum = csum;
    W.clast = clast;
    W.total = &total_sh;
    W.last = &last_sh;
    build_table_body<TB_THREADS>(B.cache, idx, (int)threadIdx.x, W, [] { __syncthreads(); }, 1u);
}

// -------------------------------------------------------------------------
// Between walker launches.  The next launch resumes the walks the last one
// parked, from the queue it wrote, with the queue state reset.
// -------------------------------------------------------------------------
__device__ __forceinline__ void prep_resume(Counters& K, uint32_t park_cap, unsigned long long total) {
    K.resume_count = min(K.park_count, park_cap);
    K.launch_idle = K.resume_count == 0u && K.walk_next >= total ? 1u : 0u;
    K.resume_side ^= 1u;
    K.park_count = 0u;
    K.resume_next = 0ull;
}

__global__ void resume_prep_kernel(Counters* K, uint32_t park_cap, unsigned long long total) {
    prep_resume(*K, park_cap, total);
}

// A device-driven round (no host decision between launches): the tables
// queued by the earlier launches were built by the kernel before this one,
// first transitions that missed one are redone next, then the parked walks
// resume.  More queued tables than that build covers hand everything over
// to the host: the rest of the round does nothing and the parked walks stay
// where they are.
__global__ void device_round_prep_kernel(Counters* K, CacheDev C, uint32_t build_max, uint32_t park_cap,
                                         unsigned long long total) {
    if (K->dev_stop) return;
    const uint32_t np = *C.n_pending;
    if (np > build_max) {
        K->dev_stop = 1u;
        K->need_first = 0u;
        K->resume_count = 0u;
        K->launch_idle = 1u;
        return;
    }
    *C.n_pending = 0u;
    K->tables_built += np;
    K->need_first = K->first_missing;
    K->first_missing = 0u;
    prep_resume(*K, park_cap, total);
}

// -------------------------------------------------------------------------
// Score reduction: per block fp32 compensated sums per net, then binary64
// across blocks.
// -------------------------------------------------------------------------
constexpr int RED_THREADS = 256;
constexpr int RED_CHUNK = 4096;

__device__ __forceinline__ void neumaier(float& s, float& c, float x) {
    const float t = s + x;
    if (fabsf(s) >= fabsf(x))
        c += (s - t) + x;
    else
        c += (x - t) + s;
    s = t;
}

// Block-level compensated sums of one RED_CHUNK slice of walks, per net.
//
// Up to RED_FLAGS nets: a stable counting sort of the slice by net (counts,
// segment starts, then one wave places the scores in walk order, ranking
// equal nets with ballots), after which every net's segment is cut into
// RED_PARTS contiguous pieces summed by different threads and combined in
// piece order.  The work is O(len) and the order of every sum is fixed by
// the slice alone (deterministic).  More nets: each thread scans the slice
// for one net.
constexpr int RED_FLAGS = 4096;
constexpr int RED_PARTS = 16;

struct RedSorted {
    uint16_t snet[RED_CHUNK];
    float sw[RED_CHUNK];
    float sorted[RED_CHUNK];
    uint32_t pos[RED_FLAGS];  // counts, then segment starts, then segment ends
    float4 part[RED_THREADS];
};
struct RedScan {
    int32_t snet[RED_CHUNK];
    float sw[RED_CHUNK];
    float4 part[RED_THREADS];
};
union RedLds {
    RedSorted s;
    RedScan d;
};

__device__ __forceinline__ void reduce_chunk_sorted(const int32_t* __restrict__ net, const float* __restrict__ w, uint64_t base,
                                    int len, int K, float4* __restrict__ out, RedSorted& L) {
    const int t = threadIdx.x;
    for (int j = t; j < K; j += RED_THREADS) L.pos[j] = 0u;
    __syncthreads();
    for (int q0 = 0; q0 < len; q0 += 4 * RED_THREADS) {
        // four loads in flight per thread
        int32_t nq[4];
        float wq[4];
#pragma unroll
        for (int u = 0; u < 4; ++u) {
            const int q = q0 + u * RED_THREADS + t;
            if (q < len) {
                nq[u] = net[base + q];
                wq[u] = w[base + q];
            }
        }
#pragma unroll
        for (int u = 0; u < 4; ++u) {
            const int q = q0 + u * RED_THREADS + t;
            if (q < len) {
                L.snet[q] = (uint16_t)nq[u];
                L.sw[q] = wq[u];
                atomicAdd(&L.pos[nq[u]], 1u);
            }
        }
    }
    __syncthreads();
    {
        // exclusive scan of the counts: segment starts
        __shared__ uint32_t wsum[RED_THREADS / 64];
        constexpr int PER = RED_FLAGS / RED_THREADS;
        const int j0 = t * PER;
        uint32_t loc[PER];
        uint32_t run = 0;
#pragma unroll
        for (int i = 0; i < PER; ++i) {
            loc[i] = j0 + i < K ? L.pos[j0 + i] : 0u;
            run += loc[i];
        }
        uint32_t incl = run;
        const int lane = t & 63;
        for (int off = 1; off < 64; off <<= 1) {
            const uint32_t v = __shfl_up(incl, off);
            if (lane >= off) incl += v;
        }
        if (lane == 63) wsum[t >> 6] = incl;
        __syncthreads();
        uint32_t before = incl - run;
        for (int wv = 0; wv < (t >> 6); ++wv) before += wsum[wv];
#pragma unroll
        for (int i = 0; i < PER; ++i) {
            if (j0 + i < K) L.pos[j0 + i] = before;
            before += loc[i];
        }
    }
    __syncthreads();
    if (t < 64) {
        // stable placement, 64 scores at a time: the lanes holding the same
        // net find each other with one ballot per bit of the net index; a
        // lane's rank is the number of such lanes below it, and the group's
        // last lane moves the segment pointer
        const int nbits = K > 1 ? 32 - __clz(K - 1) : 0;
        const unsigned long long below = (1ull << t) - 1ull;
        // the next 64 keys and scores are read one pass ahead
        uint32_t key_n = t < len ? (uint32_t)L.snet[t] : 0u;
        float w_n = t < len ? L.sw[t] : 0.f;
        for (int i = 0; i < len; i += 64) {
            const int q = i + t;
            const bool ok = q < len;
            const uint32_t key = key_n;
            const float wq = w_n;
            if (q + 64 < len) {
                key_n = L.snet[q + 64];
                w_n = L.sw[q + 64];
            }
            unsigned long long match = __ballot(ok);
            for (int bt = 0; bt < nbits; ++bt) {
                const bool bit = (key >> bt) & 1u;
                const unsigned long long m = __ballot(bit);
                match &= bit ? m : ~m;
            }
            if (ok) {
                const uint32_t p0 = L.pos[key];
                L.sorted[p0 + (uint32_t)__popcll(match & below)] = wq;
                if ((match >> t) == 1ull) L.pos[key] = p0 + (uint32_t)__popcll(match);
            }
        }
    }
    __syncthreads();
    // pos[j] is now the end of net j's segment (and the start of j + 1's)
    for (int g0 = 0; g0 < K * RED_PARTS; g0 += RED_THREADS) {
        const int task = g0 + t, j = task / RED_PARTS, pi = task % RED_PARTS;
        float s1 = 0.f, c1 = 0.f, s2 = 0.f, c2 = 0.f;
        if (j < K) {
            const uint32_t e = L.pos[j], b = j ? L.pos[j - 1] : 0u, c = e - b;
            const uint32_t q0 = b + c * pi / RED_PARTS, q1 = b + c * (pi + 1) / RED_PARTS;
            uint32_t q = q0;
            for (; q + 4 <= q1; q += 4) {
                // four scores read ahead, added in order
                float xv[4];
#pragma unroll
                for (int u = 0; u < 4; ++u) xv[u] = L.sorted[q + u];
#pragma unroll
                for (int u = 0; u < 4; ++u) {
                    neumaier(s1, c1, xv[u]);
                    neumaier(s2, c2, xv[u] * xv[u]);
                }
            }
            for (; q < q1; ++q) {
                const float x = L.sorted[q];
                neumaier(s1, c1, x);
                neumaier(s2, c2, x * x);
            }
        }
        L.part[t] = make_float4(s1, c1, s2, c2);
        __syncthreads();
        if (t < RED_THREADS / RED_PARTS) {
            const int jj = g0 / RED_PARTS + t;
            if (jj < K) {
                float a1 = 0.f, e1 = 0.f, a2 = 0.f, e2 = 0.f;
                for (int k = 0; k < RED_PARTS; ++k) {
                    const float4 v = L.part[t * RED_PARTS + k];
                    neumaier(a1, e1, v.x);
                    neumaier(a1, e1, v.y);
                    neumaier(a2, e2, v.z);
                    neumaier(a2, e2, v.w);
                }
                out[jj] = make_float4(a1, e1, a2, e2);
            }
        }
        __syncthreads();
    }
}

__device__ __forceinline__ void reduce_chunk_scan(const int32_t* __restrict__ net, const float* __restrict__ w, uint64_t base,
                                  int len, int K, float4* __restrict__ out, RedScan& L) {
    const int t = threadIdx.x;
    for (int q = t; q < len; q += RED_THREADS) {
        L.snet[q] = net[base + q];
        L.sw[q] = w[base + q];
    }
    __syncthreads();
    for (int j = t; j < K; j += RED_THREADS) {
        float s1 = 0.f, c1 = 0.f, s2 = 0.f, c2 = 0.f;
        for (int q = 0; q < len; ++q) {
            if (L.snet[q] == j) {
                const float x = L.sw[q];
                neumaier(s1, c1, x);
                neumaier(s2, c2, x * x);
            }
        }
        out[j] = make_float4(s1, c1, s2, c2);
    }
}

__device__ __forceinline__ void reduce_chunk(const int32_t* __restrict__ net, const float* __restrict__ w,
                                             uint64_t base, int len, int K, float4* __restrict__ out, RedLds& L) {
    if (K <= RED_FLAGS)
        reduce_chunk_sorted(net, w, base, len, K, out, L.s);
    else
        reduce_chunk_scan(net, w, base, len, K, out, L.d);
}

// The gate of a reduction: the counters of the walker run that wrote the
// scores.  Closed when that run did not end every walk of its gate_total (a
// walk parked, a first transition missed its table): the scores are then
// incomplete, nothing is reduced, and the host completes the run first.
__device__ __forceinline__ bool gate_closed(const Counters* gate, unsigned long long gate_total) {
    return gate && (gate->park_count != 0u || gate->first_missing != 0u || gate->walk_next < gate_total);
}

__global__ void __launch_bounds__(RED_THREADS) reduce_scores_kernel(const int32_t* __restrict__ net,
                                                                   const float* __restrict__ w, uint64_t count,
                                                                   int K, float4* __restrict__ partial,
                                                                   const Counters* gate,
                                                                   unsigned long long gate_total) {
    __shared__ RedLds L;
    if (gate_closed(gate, gate_total)) return;
    const uint64_t base = (uint64_t)blockIdx.x * RED_CHUNK;
    const int len = (int)min((uint64_t)RED_CHUNK, count - base);
    reduce_chunk(net, w, base, len, K, partial + (size_t)blockIdx.x * K, L);
}

// Reduction of a round that served several requests: segment s owns blocks
// [first_block, first_block + ceil(count / RED_CHUNK)) of the launch.
struct RedSeg {
    const int32_t* net;
    const float* w;
    unsigned long long count;
    int32_t K, first_block;
    float4* partial;
    double* acc;
    double n_total;
    double* out;  // 2K results (row, se) for the host copy
};

__global__ void __launch_bounds__(RED_THREADS) reduce_multi_kernel(const RedSeg* __restrict__ segs, int n_segs) {
    __shared__ RedLds L;
    int lo = 0, hi = n_segs - 1;
    while (lo < hi) {
        const int mid = (lo + hi + 1) >> 1;
        if (segs[mid].first_block <= (int)blockIdx.x)
            lo = mid;
        else
            hi = mid - 1;
    }
    const RedSeg R = segs[lo];
    const int local = (int)blockIdx.x - R.first_block;
    const uint64_t base = (uint64_t)local * RED_CHUNK;
    if (base >= R.count) return;
    const int len = (int)min((uint64_t)RED_CHUNK, R.count - base);
    reduce_chunk(R.net, R.w, base, len, R.K, R.partial + (size_t)local * R.K, L);
}

__global__ void finish_multi_kernel(const RedSeg* __restrict__ segs) {
    const RedSeg R = segs[blockIdx.x];
    const int blocks = (int)((R.count + RED_CHUNK - 1) / RED_CHUNK);
    const int K = R.K;
    for (int j = threadIdx.x; j < K; j += blockDim.x) {
        double s1 = 0.0, s2 = 0.0;
        for (int b = 0; b < blocks; ++b) {
            const float4 p = R.partial[(size_t)b * K + j];
            s1 += (double)p.x + (double)p.y;
            s2 += (double)p.z + (double)p.w;
        }
        s1 += R.acc[j];
        s2 += R.acc[K + j];
        R.acc[j] = s1;
        R.acc[K + j] = s2;
        const double m = s1 / R.n_total;
        const double var = (s2 / R.n_total - m * m) / (R.n_total - 1.0);
        R.out[j] = m;
        R.out[K + j] = sqrt(var > 0.0 ? var : 0.0);
    }
}

// Binary64 sums of a launch's block partials and the stopping rule of
// Alg. 1 (walk until the estimate of C_mm is accurate enough).  The blocks
// of 4096 walks form groups of SUM_GROUP; a group's partials are added in
// block order from zero, and the group sums are added in order to acc[2*K],
// the running sums (S1, S2) per net of the walks before the launch.
// Launches start on a group boundary, so the sums do not depend on how the
// walks were split into launches.  Checkpoints fall every `per_ck` blocks
// (a multiple of SUM_GROUP); the first one where 3 SE(C_mm) / |C_mm| <=
// target ends the extraction, and the blocks after it are not added.
struct Choice {
    int32_t blocks;  // blocks added (-1: the gate was closed, nothing added)
    int32_t met;     // 1: the target was met at that checkpoint
    unsigned long long walks;
};

constexpr int SUM_GROUP = 16;            // blocks per group (65536 walks)
constexpr int DECIDE_MAX_GROUPS = 4096;  // groups per launch (group sums in LDS)

__device__ __forceinline__ void mean_se(double s1, double s2, double n, double* m, double* se) {
    const double mm = s1 / n;
    const double var = (s2 / n - mm * mm) / (n - 1.0);
    *m = mm;
    *se = sqrt(var > 0.0 ? var : 0.0);
}

// Group sums of net j over blocks [0, blocks): one lane per group, each
// group's partials loaded at once and added in block order.
__device__ __forceinline__ void group_sums(const float4* __restrict__ partial, int blocks, int K, int j, double* g1,
                                           double* g2) {
    const int ng = (blocks + SUM_GROUP - 1) / SUM_GROUP;
    for (int g = (int)threadIdx.x; g < ng; g += 64) {
        const int b0 = g * SUM_GROUP;
        float4 p[SUM_GROUP];
#pragma unroll
        for (int u = 0; u < SUM_GROUP; ++u)
            p[u] = b0 + u < blocks ? partial[(size_t)(b0 + u) * K + j] : make_float4(0.f, 0.f, 0.f, 0.f);
        double a1 = 0.0, a2 = 0.0;
#pragma unroll
        for (int u = 0; u < SUM_GROUP; ++u) {
            if (b0 + u < blocks) {
                a1 += (double)p[u].x + (double)p[u].y;
                a2 += (double)p[u].z + (double)p[u].w;
            }
        }
        g1[g] = a1;
        g2[g] = a2;
    }
    __syncthreads();
}

// One wave: the master's group sums, then lane 0 adds them in order and
// tests each checkpoint.  target <= 0: every block is added.
__global__ void __launch_bounds__(64) decide_kernel(const float4* __restrict__ partial, int blocks, int K, int master,
                                                    int per_ck, const double* __restrict__ acc, double n_before,
                                                    unsigned long long count, double target, const Counters* gate,
                                                    unsigned long long gate_total, Choice* out) {
    __shared__ double g1[DECIDE_MAX_GROUPS], g2[DECIDE_MAX_GROUPS];
    if (gate_closed(gate, gate_total)) {
        if (threadIdx.x == 0) {
            out->blocks = -1;
            out->met = 0;
            out->walks = 0ull;
        }
        return;
    }
    int chosen = blocks, met = 0;
    if (target > 0.0) {
        group_sums(partial, blocks, K, master, g1, g2);
        if (threadIdx.x != 0) return;
        const int ng = (blocks + SUM_GROUP - 1) / SUM_GROUP, ck_groups = per_ck / SUM_GROUP;
        double s1 = acc[master], s2 = acc[K + master];
        int to_ck = ck_groups;
        for (int g = 0; g < ng; ++g) {
            s1 += g1[g];
            s2 += g2[g];
            if (--to_ck == 0 || g + 1 == ng) {
                to_ck = ck_groups;
                const int nb = min((g + 1) * SUM_GROUP, blocks);
                const unsigned long long w = min((unsigned long long)nb * RED_CHUNK, count);
                double m, se;
                mean_se(s1, s2, n_before + (double)w, &m, &se);
                if (m != 0.0 && 3.0 * se / fabs(m) <= target) {
                    chosen = nb;
                    met = 1;
                    break;
                }
            }
        }
    } else if (threadIdx.x != 0) {
        return;
    }
    out->blocks = chosen;
    out->met = met;
    out->walks = min((unsigned long long)chosen * RED_CHUNK, count);
}

// One wave per net: the group sums of the chosen blocks added in order by
// lane 0, then the row entry and its standard error.
__global__ void __launch_bounds__(64) finish_seq_kernel(const float4* __restrict__ partial, int K, double* acc,
                                                        double n_before, const Choice* choice, double* result) {
    __shared__ double g1[DECIDE_MAX_GROUPS], g2[DECIDE_MAX_GROUPS];
    const int j = blockIdx.x;
    const int nb = choice->blocks;
    if (nb < 0) return;
    group_sums(partial, nb, K, j, g1, g2);
    if (threadIdx.x != 0) return;
    const int ng = (nb + SUM_GROUP - 1) / SUM_GROUP;
    double s1 = acc[j], s2 = acc[K + j];
    for (int g = 0; g < ng; ++g) {
        s1 += g1[g];
        s2 += g2[g];
    }
    acc[j] = s1;
    acc[K + j] = s2;
    double m, se;
    mean_se(s1, s2, n_before + (double)choice->walks, &m, &se);
    result[j] = m;
    result[K + j] = se;
}

// -------------------------------------------------------------------------
// Geometry store construction kernels.
// -------------------------------------------------------------------------
__device__ __forceinline__ void cell_box(const StructDev& S, int c, float lo[3], float hi[3]) {
    const int ix = c % S.gdim[0], iy = (c / S.gdim[0]) % S.gdim[1], iz = c / (S.gdim[0] * S.gdim[1]);
    const int ii[3] = {ix, iy, iz};
    for (int a = 0; a < 3; ++a) {
        lo[a] = S.gorg[a] + ii[a] * S.gcell[a];
        hi[a] = lo[a] + S.gcell[a];
    }
}

__device__ float cell_dfar(const StructDev& S, const float lo[3], const float hi[3]) {
    float dfar = INFINITY;
    for (int c = 0; c < S.n_cond; ++c) {
        const float4 bl = S.cond_lo[c], bh = S.cond_hi[c];
        const float l[3] = {bl.x, bl.y, bl.z}, h[3] = {bh.x, bh.y, bh.z};
        float d = 0.f;
        for (int a = 0; a < 3; ++a) d = fmaxf(d, fmaxf(fmaxf(l[a] - lo[a], hi[a] - h[a]), 0.f));
        dfar = fminf(dfar, d);
    }
    for (int a = 0; a < 3; ++a) {
        if (S.bc[2 * a] == MW_BC_DIRICHLET) dfar = fminf(dfar, hi[a] - S.wlo[a]);
        if (S.bc[2 * a + 1] == MW_BC_DIRICHLET) dfar = fminf(dfar, S.whi[a] - lo[a]);
    }
    return dfar * 1.0001f + 1e-6f;
}

// Candidate counts and lists per grid cell: conductors within factor x the
// cell's conductor-free distance (factor 1: the conductors that can be
// nearest) and dielectric boxes within the same range.
__global__ void grid_count_kernel(StructDev S, uint32_t* ccount, uint32_t* dcount, int ncells, float factor) {
    const int c = blockIdx.x * blockDim.x + threadIdx.x;
    if (c >= ncells) return;
    float lo[3], hi[3];
    cell_box(S, c, lo, hi);
    const float dfar = cell_dfar(S, lo, hi) * factor;
    uint32_t nc = 0, nd = 0;
    for (int q = 0; q < S.n_cond; ++q) {
        const float4 bl = S.cond_lo[q], bh = S.cond_hi[q];
        const float l[3] = {bl.x, bl.y, bl.z}, h[3] = {bh.x, bh.y, bh.z};
        float gap = 0.f;
        for (int a = 0; a < 3; ++a) gap = fmaxf(gap, fmaxf(l[a] - hi[a], lo[a] - h[a]));
        if (gap <= dfar) ++nc;
    }
    for (int q = 0; q < S.n_diel; ++q) {
        const float4 bl = S.diel_lo[q], bh = S.diel_hi[q];
        const float l[3] = {bl.x, bl.y, bl.z}, h[3] = {bh.x, bh.y, bh.z};
        bool hit = true;
        for (int a = 0; a < 3; ++a) hit &= l[a] <= hi[a] + dfar && h[a] >= lo[a] - dfar;
        if (hit) ++nd;
    }
    ccount[c] = nc;
    dcount[c] = nd;
}

__global__ void grid_fill_kernel(StructDev S, const uint32_t* coff, const uint32_t* doff, uint32_t* clist,
                                 uint32_t* dlist, int ncells, float factor) {
    const int c = blockIdx.x * blockDim.x + threadIdx.x;
    if (c >= ncells) return;
    float lo[3], hi[3];
    cell_box(S, c, lo, hi);
    const float dfar = cell_dfar(S, lo, hi) * factor;
    uint32_t pc = coff[c], pd = doff[c];
    for (int q = 0; q < S.n_cond; ++q) {
        const float4 bl = S.cond_lo[q], bh = S.cond_hi[q];
        const float l[3] = {bl.x, bl.y, bl.z}, h[3] = {bh.x, bh.y, bh.z};
        float gap = 0.f;
        for (int a = 0; a < 3; ++a) gap = fmaxf(gap, fmaxf(l[a] - hi[a], lo[a] - h[a]));
        if (gap <= dfar) clist[pc++] = (uint32_t)q;
    }
    for (int q = 0; q < S.n_diel; ++q) {
        const float4 bl = S.diel_lo[q], bh = S.diel_hi[q];
        const float l[3] = {bl.x, bl.y, bl.z}, h[3] = {bh.x, bh.y, bh.z};
        bool hit = true;
        for (int a = 0; a < 3; ++a) hit &= l[a] <= hi[a] + dfar && h[a] >= lo[a] - dfar;
        if (hit) dlist[pd++] = (uint32_t)q;
    }
}

// In-place candidate records: rec[2 i] = lo[list[i]], rec[2 i + 1] = hi[list[i]].
__global__ void grid_records_kernel(const uint32_t* list, uint32_t total, const float4* lo, const float4* hi,
                                    float4* rec) {
    const uint32_t i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= total) return;
    const uint32_t id = list[i];
    rec[2 * (size_t)i] = lo[id];
    rec[2 * (size_t)i + 1] = hi[id];
}

// Exclusive scan of counts (single block) into off[0..n].
__global__ void scan_kernel(const uint32_t* count, uint32_t* off, int n) {
    __shared__ uint32_t part[1024];
    const int per = (n + blockDim.x - 1) / blockDim.x;
    const int b = threadIdx.x * per, e = min(n, b + per);
    uint32_t s = 0;
    for (int q = b; q < e; ++q) s += count[q];
    part[threadIdx.x] = s;
    __syncthreads();
    if (threadIdx.x == 0) {
        uint32_t run = 0;
        for (int q = 0; q < (int)blockDim.x; ++q) {
            const uint32_t v = part[q];
            part[q] = run;
            run += v;
        }
        off[n] = run;
    }
    __syncthreads();
    uint32_t run = part[threadIdx.x];
    for (int q = b; q < e; ++q) {
        off[q] = run;
        run += count[q];
    }
}

// -------------------------------------------------------------------------
// Host side.
// -------------------------------------------------------------------------
struct Cache {
    CacheDev d{};
    void* mem = nullptr;
    std::mutex mu;
    uint32_t uniform_index = NO_INDEX;  // valid until the cache is emptied
    uint64_t flushes = 0;               // times the full cache was emptied
    // Empties the cache (with its lock held and no FRW work in flight).
    void clear() {
        MW_HIP(hipMemset(d.slot, 0, 8ull * ((size_t)d.slot_mask + 1)));
        MW_HIP(hipMemset(d.ready, 0, 4ull * d.capacity));
        MW_HIP(hipMemset(d.n_tables, 0, 4));
        MW_HIP(hipMemset(d.n_pending, 0, 4));
        MW_HIP(hipMemset(d.pending, 0xff, 4ull * d.capacity));
        MW_HIP(hipDeviceSynchronize());
        uniform_index = NO_INDEX;
    }
};

std::mutex g_cache_mu;
std::map<std::pair<int, int>, std::unique_ptr<Cache>> g_caches;

// Boundary entries per face side of a table: interior nodes per axis on the
// vertex lattice (n even), cells per axis on the cell lattice (n odd).
uint32_t table_m(int n) { return (n & 1) ? (uint32_t)n : (uint32_t)(n - 1); }

size_t env_size(const char* name, size_t dflt) {
    const char* v = getenv(name);
    return v ? (size_t)strtoull(v, nullptr, 10) : dflt;
}

Cache& get_cache(int n) {
    int dev = 0;
    MW_HIP(hipGetDevice(&dev));
    std::lock_guard<std::mutex> g(g_cache_mu);
    auto& slot = g_caches[{dev, n}];
    if (!slot) {
        auto c = std::make_unique<Cache>();
        const uint32_t M = table_m(n);
        const uint32_t nb = 6 * M * M;
        const uint32_t cap = (uint32_t)env_size("MWALK_TABLE_CAP", 65536);
        uint32_t nslots = 1;
        while (nslots < 2 * cap) nslots <<= 1;
        c->d.n = n;
        c->d.nb = nb;
        c->d.capacity = cap;
        c->d.slot_mask = nslots - 1;
        c->d.key_words = KEY_HDR + n;
        c->d.key_stride = (c->d.key_words + 3) & ~3u;
        c->d.tab_words = TAB_CDF + nb + (nb + 31) / 32;
        const size_t b_hash = (size_t)nslots * 8, b_ready = (size_t)cap * 4;
        const size_t b_keys = (size_t)cap * c->d.key_stride * 4, b_data = (size_t)cap * c->d.tab_words * 4;
        const size_t b_misc = 256, b_pend = (size_t)cap * 4;
        const size_t total = b_hash + b_ready + b_keys + b_data + b_misc + b_pend + 2048;
        char* m = (char*)dev_alloc(total);
        c->mem = m;
        size_t o = 0;
        auto take = [&](size_t b) {
            char* p = m + o;
            o += (b + 255) / 256 * 256;
            return p;
        };
        c->d.slot = (unsigned long long*)take(b_hash);
        c->d.ready = (uint32_t*)take(b_ready);
        c->d.keys = (uint32_t*)take(b_keys);
        c->d.data = (uint32_t*)take(b_data);
        uint32_t* misc = (uint32_t*)take(b_misc);
        c->d.n_tables = misc;
        c->d.n_pending = misc + 1;
        c->d.pending = (uint32_t*)take(b_pend);
        MW_HIP(hipMemset(c->d.slot, 0, b_hash));
        MW_HIP(hipMemset(c->d.ready, 0, b_ready));
        MW_HIP(hipMemset(misc, 0, b_misc));
        MW_HIP(hipMemset(c->d.pending, 0xff, b_pend));  // empty queue entries hold NO_INDEX
        MW_HIP(hipDeviceSynchronize());
        slot = std::move(c);
    }
    return *slot;
}

}  // namespace
}  // namespace mw

using namespace mw;

namespace {
struct ExtractCtx;
void delete_ctx(ExtractCtx* c);
}  // namespace

struct mw_structure {
    int device = 0;
    size_t bytes = 0;  // device memory held (arrays, grid index)
    StructDev h{};
    StructDev* d = nullptr;
    char* mem = nullptr;
    int32_t n_nets = 0;
    std::vector<mw_cond_box> cond;
    // walks the last target-mode extraction per (master, checkpoint, target)
    // needed: sizes the next one's first launch (results do not depend on it)
    std::mutex hint_mu;
    std::map<std::tuple<int, uint64_t, double>, uint64_t> hints;
    uint64_t walk_hint(int master, uint64_t ck, double target) {
        std::lock_guard<std::mutex> g(hint_mu);
        auto it = hints.find({master, ck, target});
        return it == hints.end() ? 0 : it->second;
    }
    void set_walk_hint(int master, uint64_t ck, double target, uint64_t walks) {
        std::lock_guard<std::mutex> g(hint_mu);
        hints[{master, ck, target}] = walks;
    }
    // frw_extract's buffers and launch graphs kept between calls, one per
    // (master, options) in use; guarded by ctx_mu
    std::mutex ctx_mu;
    std::vector<ExtractCtx*> ctxs;
    uint64_t ctx_clock = 0;
};

static void validate_desc(const mw_structure_desc* D) {
    MW_REQUIRE(D, MW_EINVAL, "null structure description");
    MW_REQUIRE(D->n_cond >= 1 && D->cond, MW_EINVAL, "at least one conductor box is required");
    MW_REQUIRE(D->n_nets >= 1 && D->n_nets <= (1 << 20), MW_EINVAL, "n_nets out of range");
    MW_REQUIRE(D->n_diel >= 0 && (D->n_diel == 0 || D->diel), MW_EINVAL, "bad dielectric list");
    MW_REQUIRE(D->n_layers >= 1 && D->layer_z0 && D->layer_eps, MW_EINVAL, "at least one background layer");
    for (int f = 0; f < 6; ++f) MW_REQUIRE(D->bc[f] <= 1, MW_EINVAL, "bc[%d] must be 0 or 1", f);
    for (int a = 0; a < 3; ++a) MW_REQUIRE(D->win_lo[a] < D->win_hi[a], MW_EGEOM, "empty window");
    std::vector<int> per_net(D->n_nets, 0);
    for (int i = 0; i < D->n_cond; ++i) {
        const mw_cond_box& b = D->cond[i];
        MW_REQUIRE(b.net >= 0 && b.net < D->n_nets, MW_EGEOM, "conductor %d: net %d out of range", i, b.net);
        per_net[b.net]++;
        for (int a = 0; a < 3; ++a) {
            MW_REQUIRE(b.lo[a] < b.hi[a], MW_EGEOM, "conductor %d is empty", i);
            MW_REQUIRE(b.lo[a] >= D->win_lo[a] && b.hi[a] <= D->win_hi[a], MW_EGEOM,
                       "conductor %d leaves the window", i);
        }
    }
    for (int j = 0; j < D->n_nets; ++j) MW_REQUIRE(per_net[j] >= 1, MW_EGEOM, "net %d has no box", j);
    // boxes of one net may touch or overlap; boxes of different nets may not
    for (int i = 0; i < D->n_cond; ++i)
        for (int k = i + 1; k < D->n_cond; ++k) {
            if (D->cond[i].net == D->cond[k].net) continue;
            bool overlap = true;
            for (int a = 0; a < 3; ++a)
                overlap &= D->cond[i].lo[a] < D->cond[k].hi[a] && D->cond[k].lo[a] < D->cond[i].hi[a];
            MW_REQUIRE(!overlap, MW_EGEOM, "conductors %d and %d overlap", i, k);
        }
    for (int i = 0; i < D->n_diel; ++i) {
        const float e = D->diel[i].eps;
        MW_REQUIRE(e >= 1e-3f && e <= 1e3f, MW_EINVAL, "dielectric %d: eps %g outside [1e-3, 1e3]", i, e);
        for (int a = 0; a < 3; ++a) MW_REQUIRE(D->diel[i].lo[a] < D->diel[i].hi[a], MW_EGEOM, "dielectric %d is empty", i);
    }
    for (int l = 0; l < D->n_layers; ++l) {
        const float e = D->layer_eps[l];
        MW_REQUIRE(e >= 1e-3f && e <= 1e3f, MW_EINVAL, "layer %d: eps %g outside [1e-3, 1e3]", l, e);
        if (l > 0) MW_REQUIRE(D->layer_z0[l] > D->layer_z0[l - 1], MW_EINVAL, "layer_z0 must ascend");
    }
}

// A non-blocking stream of the calling thread for structure creation and
// extraction set-up: their copies and kernels neither wait for nor hold up
// work on the legacy default stream (a server prepares the next requests
// while a round runs there).
hipStream_t setup_stream() {
    thread_local hipStream_t s = nullptr;
    thread_local int dev = -1;
    int cur = 0;
    MW_HIP(hipGetDevice(&cur));
    if (!s || dev != cur) {
        MW_HIP(hipStreamCreateWithFlags(&s, hipStreamNonBlocking));
        dev = cur;
    }
    return s;
}

extern "C" mw_status mw_structure_create(const mw_structure_desc* D, mw_structure** out) {
    return guarded([&] {
        MW_REQUIRE(out, MW_EINVAL, "null output handle");
        validate_desc(D);
        hipStream_t ss = setup_stream();
        auto st = std::make_unique<mw_structure>();
        MW_HIP(hipGetDevice(&st->device));
        st->n_nets = D->n_nets;
        st->cond.assign(D->cond, D->cond + D->n_cond);
        const int nc = D->n_cond, nd = D->n_diel, nl = D->n_layers;
        // uniform grid over the window
        float ext[3], vol = 1.f;
        for (int a = 0; a < 3; ++a) {
            ext[a] = D->win_hi[a] - D->win_lo[a];
            vol *= ext[a];
        }
        const double target = std::min(1048576.0, std::max(512.0, 256.0 * (nc + nd)));
        const double cs = std::cbrt(vol / target);
        int gd[3];
        int ncells = 1;
        for (int a = 0; a < 3; ++a) {
            gd[a] = std::max(1, std::min(512, (int)std::ceil(ext[a] / cs)));
            ncells *= gd[a];
        }
        std::vector<float4> clo(nc), chi(nc), dlo(std::max(nd, 1)), dhi(std::max(nd, 1));
        for (int i = 0; i < nc; ++i) {
            const mw_cond_box& b = D->cond[i];
            int net = b.net;
            float w;
            std::memcpy(&w, &net, 4);
            clo[i] = make_float4(b.lo[0], b.lo[1], b.lo[2], w);
            chi[i] = make_float4(b.hi[0], b.hi[1], b.hi[2], 0.f);
        }
        for (int i = 0; i < nd; ++i) {
            const mw_diel_box& b = D->diel[i];
            const uint32_t code = (uint32_t)std::nearbyint((double)b.eps * 65536.0);
            float cw;
            std::memcpy(&cw, &code, 4);
            dlo[i] = make_float4(b.lo[0], b.lo[1], b.lo[2], b.eps);
            dhi[i] = make_float4(b.hi[0], b.hi[1], b.hi[2], cw);
        }
        std::vector<float> z0(D->layer_z0, D->layer_z0 + nl);
        std::vector<uint32_t> lcode(nl), leps(nl);
        for (int l = 0; l < nl; ++l) {
            lcode[l] = (uint32_t)std::nearbyint((double)D->layer_eps[l] * 65536.0);
            std::memcpy(&leps[l], &D->layer_eps[l], 4);
        }
        // one allocation: arrays, then grid offsets/counts (lists sized after counting)
        size_t o = 0;
        auto sz = [&](size_t b) {
            size_t r = o;
            o += (b + 255) / 256 * 256;
            return r;
        };
        const size_t o_clo = sz(16 * nc), o_chi = sz(16 * nc), o_dlo = sz(16 * dlo.size()), o_dhi = sz(16 * dhi.size());
        const size_t o_z0 = sz(4 * nl), o_lc = sz(4 * nl), o_le = sz(4 * nl);
        const size_t o_cc = sz(4 * ncells), o_dc = sz(4 * ncells), o_coff = sz(4 * (ncells + 1)),
                     o_doff = sz(4 * (ncells + 1));
        const size_t o_ecc = sz(4 * ncells), o_edc = sz(4 * ncells), o_eoff = sz(4 * (ncells + 1)),
                     o_xoff = sz(4 * (ncells + 1));
        const size_t o_desc = sz(sizeof(StructDev));
        char* m = (char*)dev_alloc(o);
        struct Guard {
            char* p;
            bool keep = false;
            ~Guard() {
                if (!keep) dev_free(p);
            }
        } guard{m};
        MW_HIP(hipMemcpyAsync(m + o_clo, clo.data(), 16 * nc, hipMemcpyHostToDevice, ss));
        MW_HIP(hipMemcpyAsync(m + o_chi, chi.data(), 16 * nc, hipMemcpyHostToDevice, ss));
        MW_HIP(hipMemcpyAsync(m + o_dlo, dlo.data(), 16 * dlo.size(), hipMemcpyHostToDevice, ss));
        MW_HIP(hipMemcpyAsync(m + o_dhi, dhi.data(), 16 * dhi.size(), hipMemcpyHostToDevice, ss));
        MW_HIP(hipMemcpyAsync(m + o_z0, z0.data(), 4 * nl, hipMemcpyHostToDevice, ss));
        MW_HIP(hipMemcpyAsync(m + o_lc, lcode.data(), 4 * nl, hipMemcpyHostToDevice, ss));
        MW_HIP(hipMemcpyAsync(m + o_le, leps.data(), 4 * nl, hipMemcpyHostToDevice, ss));
        StructDev& S = st->h;
        S.n_cond = nc;
        S.n_nets = D->n_nets;
        S.n_diel = nd;
        S.n_layers = nl;
        S.cond_lo = (const float4*)(m + o_clo);
        S.cond_hi = (const float4*)(m + o_chi);
        S.diel_lo = (const float4*)(m + o_dlo);
        S.diel_hi = (const float4*)(m + o_dhi);
        S.layer_z0 = (const float*)(m + o_z0);
        S.layer_code = (const uint32_t*)(m + o_lc);
        S.layer_eps = (const uint32_t*)(m + o_le);
        double diag = 0;
        for (int a = 0; a < 3; ++a) {
            S.wlo[a] = D->win_lo[a];
            S.whi[a] = D->win_hi[a];
            S.gdim[a] = gd[a];
            S.gorg[a] = D->win_lo[a];
            S.gcell[a] = ext[a] / gd[a];
            S.ginv[a] = gd[a] / ext[a];
            diag += (double)ext[a] * ext[a];
        }
        for (int f = 0; f < 6; ++f) S.bc[f] = D->bc[f];
        S.delta_abs = (float)(1e-6 * std::sqrt(diag));
        uint32_t* ccount = (uint32_t*)(m + o_cc);
        uint32_t* dcount = (uint32_t*)(m + o_dc);
        uint32_t* coff = (uint32_t*)(m + o_coff);
        uint32_t* doff = (uint32_t*)(m + o_doff);
        uint32_t* ecount = (uint32_t*)(m + o_ecc);
        uint32_t* xcount = (uint32_t*)(m + o_edc);
        uint32_t* eoff = (uint32_t*)(m + o_eoff);
        uint32_t* xoff = (uint32_t*)(m + o_xoff);
        const int tb = 128, nbk = (ncells + tb - 1) / tb;
        grid_count_kernel<<<nbk, tb, 0, ss>>>(S, ccount, dcount, ncells, 1.f);
        grid_count_kernel<<<nbk, tb, 0, ss>>>(S, ecount, xcount, ncells, EXP_LIST_FACTOR);
        scan_kernel<<<1, 1024, 0, ss>>>(ccount, coff, ncells);
        scan_kernel<<<1, 1024, 0, ss>>>(dcount, doff, ncells);
        scan_kernel<<<1, 1024, 0, ss>>>(ecount, eoff, ncells);
        scan_kernel<<<1, 1024, 0, ss>>>(xcount, xoff, ncells);
        MW_HIP(hipGetLastError());
        uint32_t tot[4];
        MW_HIP(hipMemcpyAsync(&tot[0], coff + ncells, 4, hipMemcpyDeviceToHost, ss));
        MW_HIP(hipMemcpyAsync(&tot[1], doff + ncells, 4, hipMemcpyDeviceToHost, ss));
        MW_HIP(hipMemcpyAsync(&tot[2], eoff + ncells, 4, hipMemcpyDeviceToHost, ss));
        MW_HIP(hipMemcpyAsync(&tot[3], xoff + ncells, 4, hipMemcpyDeviceToHost, ss));
        MW_HIP(hipStreamSynchronize(ss));
        size_t lo4[4], lb = 0;
        for (int q = 0; q < 4; ++q) {
            lo4[q] = lb;
            lb += ((4ull * tot[q] + 255) / 256) * 256;
        }
        const size_t o_crec = lb;
        lb += ((32ull * tot[0] + 255) / 256) * 256;
        const size_t o_drec = lb;
        lb += ((32ull * tot[1] + 255) / 256) * 256;
        const size_t o_erec = lb;
        lb += ((32ull * tot[2] + 255) / 256) * 256;
        const size_t o_xrec = lb;
        lb += ((32ull * tot[3] + 255) / 256) * 256;
        const size_t list_bytes = lb + 512;
        char* lists = (char*)dev_alloc(list_bytes);
        st->bytes = o + list_bytes;
        uint32_t* clist = (uint32_t*)(lists + lo4[0]);
        uint32_t* dlist = (uint32_t*)(lists + lo4[1]);
        uint32_t* elist = (uint32_t*)(lists + lo4[2]);
        uint32_t* xlist = (uint32_t*)(lists + lo4[3]);
        grid_fill_kernel<<<nbk, tb, 0, ss>>>(S, coff, doff, clist, dlist, ncells, 1.f);
        grid_fill_kernel<<<nbk, tb, 0, ss>>>(S, eoff, xoff, elist, xlist, ncells, EXP_LIST_FACTOR);
        float4* crec = (float4*)(lists + o_crec);
        float4* drec = (float4*)(lists + o_drec);
        if (tot[0]) grid_records_kernel<<<(tot[0] + 255) / 256, 256, 0, ss>>>(clist, tot[0], S.cond_lo, S.cond_hi, crec);
        if (tot[1]) grid_records_kernel<<<(tot[1] + 255) / 256, 256, 0, ss>>>(dlist, tot[1], S.diel_lo, S.diel_hi, drec);
        float4* erec = (float4*)(lists + o_erec);
        float4* xrec = (float4*)(lists + o_xrec);
        if (tot[2]) grid_records_kernel<<<(tot[2] + 255) / 256, 256, 0, ss>>>(elist, tot[2], S.cond_lo, S.cond_hi, erec);
        if (tot[3]) grid_records_kernel<<<(tot[3] + 255) / 256, 256, 0, ss>>>(xlist, tot[3], S.diel_lo, S.diel_hi, xrec);
        MW_HIP(hipGetLastError());
        S.gc_off = coff;
        S.gc_list = clist;
        S.gd_off = doff;
        S.gd_list = dlist;
        S.ge_off = eoff;
        S.ge_list = elist;
        S.gx_off = xoff;
        S.gx_list = xlist;
        S.gc_rec = crec;
        S.gd_rec = drec;
        S.ge_rec = erec;
        S.gx_rec = xrec;
        st->d = (StructDev*)(m + o_desc);
        MW_HIP(hipMemcpyAsync(st->d, &S, sizeof S, hipMemcpyHostToDevice, ss));
        MW_HIP(hipStreamSynchronize(ss));
        st->mem = m;
        guard.keep = true;
        // the list block (starting with the conductor list) is owned
        // through the pointer kept in h.gc_list
        st->h.gc_list = clist;
        *out = st.release();
        (void)lists;
    });
}

extern "C" mw_status mw_structure_destroy(mw_structure* s) {
    return guarded([&] {
        if (!s) return;
        (void)hipDeviceSynchronize();
        for (ExtractCtx* c : s->ctxs) delete_ctx(c);
        s->ctxs.clear();
        dev_free((void*)s->h.gc_list);
        dev_free(s->mem);
        delete s;
    });
}

namespace {

// Launch geometry of the FRW kernels for lattice size n.
struct LaunchGeom {
    uint32_t lane_stride, first_stride, lane_stride_e;
    size_t lds, first_lds, lds_e;
    int blocks, first_blocks, blocks_e;
    int cus;
    uint64_t pool;
};

LaunchGeom launch_geom(int n) {
    int dev = 0, cus = 0;
    MW_HIP(hipGetDevice(&dev));
    MW_HIP(hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev));
    LaunchGeom g;
    g.cus = cus;
    // LDS per lane: axis masks + region codes (+ a key buffer for first
    // transitions); odd dword strides spread lanes over the banks
    // (cell lattice, odd n: mask rows n + 1 apart)
    const int ns = n + (n & 1);
    g.lane_stride = (uint32_t)((6 * ns + 4 * MAX_REGIONS + 4 * ns + 3) / 4) | 1u;
    g.first_stride = (uint32_t)((6 * ns + 4 * MAX_REGIONS + 4 * ns + 4 * (KEY_HDR + n) + 3) / 4) | 1u;
    // (+ the walker's LDS copy of the layer table)
    g.lds = (size_t)g.lane_stride * 4 * WALK_THREADS + 4 * 2 * LAYER_LDS;
    g.first_lds = (size_t)g.first_stride * 4 * FRW_THREADS + 4 * 2 * LAYER_LDS;
    // LDS is allocated in 512-byte granules; 16 waves per CU is the VGPR limit
    g.blocks = cus * std::max(1, std::min(16, (int)(163840 / ((g.lds + 511) / 512 * 512))));
    g.first_blocks = cus * std::max(1, std::min(8, (int)(163840 / (g.first_lds + 512))));
    // MicroWalk-E lanes also hold the expanded cube's node masks
    g.lane_stride_e = (uint32_t)(g.lane_stride + lane_exp_words(n)) | 1u;
    g.lds_e = (size_t)g.lane_stride_e * 4 * WALK_THREADS + 4 * 2 * LAYER_LDS;
    g.blocks_e = cus * std::max(1, std::min(16, (int)(163840 / ((g.lds_e + 511) / 512 * 512))));
    g.pool = (uint64_t)g.blocks * WALK_THREADS;
    return g;
}

// Runs the walks of a list of segments to completion: first transitions
// (retried after missing tables are built), then walker launches (parked
// walks resume after their tables are built).  Holds the table cache of one
// lattice size while it runs.
// Device-driven rounds enqueued after a run's first walker launch (table
// builds and resumes without a host decision in between), and the most
// queued tables one such round builds.
constexpr int DEVICE_ROUNDS = 3;
constexpr uint32_t DEV_BUILD_MAX = 128;


struct Runner {
    int n, hybrid;
    int expand_m = 0;  // MicroWalk-E when > 0 (expanded half-size n d / (2 m))
    int plain = 0;     // one walker launch per transition round
    Cache* cache;
    LaunchGeom g;
    uint32_t park_cap;
    int seg_cap;
    uint32_t uniform_index = NO_INDEX;
    char* mem = nullptr;
    Counters* ctr;
    uint32_t* status;
    Parked* park[2];
    Segment* dsegs;
    // HIP event pairs around the walker launches not yet counted in walker_ms
    // (recorded as external events, so that a captured graph records them)
    std::vector<std::pair<hipEvent_t, hipEvent_t>> evs;
    size_t ev_used = 0;
    uint64_t misses = 0, launches = 0;
    uint32_t built_seen = 0;  // device-round table builds already counted in misses
    double walker_ms = 0.0;
    double* dev_work = nullptr;  // workspace of the device-round table builds

    // stream of this runner's launches and copies (nullptr: the legacy
    // default stream); table builds and cache flushes always run on the
    // default stream with the device otherwise idle
    hipStream_t stream = nullptr;
    int waves_per_cu = 0;  // resident walker waves per CU (0: as many as LDS allows)
    // the run in progress (start .. finish)
    std::vector<Segment> cur_segs;
    StructDev cur_s0{};
    bool cur_single = false;
    unsigned long long cur_total = 0;

    template <class F>
    void set_lds(F* f, size_t bytes) {
        MW_HIP(hipFuncSetAttribute((const void*)f, hipFuncAttributeMaxDynamicSharedMemorySize, (int)bytes));
    }

    Runner(int n_, int hybrid_, uint64_t max_walks, int seg_cap_) : n(n_), hybrid(hybrid_), seg_cap(seg_cap_) {
        cache = &get_cache(n);
        g = launch_geom(n);
        park_cap = (uint32_t)std::min<uint64_t>(std::max<uint64_t>(max_walks, 1024), 1u << 24);
        size_t o = 0;
        auto sz = [&](size_t b) {
            size_t r = o;
            o += (b + 255) / 256 * 256;
            return r;
        };
        // counters and segment list adjacent: one copy sets both per run
        const size_t o_ctr = sz(sizeof(Counters)), o_sg = sz(sizeof(Segment) * (size_t)seg_cap), o_st = sz(16);
        const size_t o_p0 = sz(sizeof(Parked) * (size_t)park_cap), o_p1 = sz(sizeof(Parked) * (size_t)park_cap);
        mem = (char*)dev_alloc(o);
        ctr = (Counters*)(mem + o_ctr);
        status = (uint32_t*)(mem + o_st);
        park[0] = (Parked*)(mem + o_p0);
        park[1] = (Parked*)(mem + o_p1);
        dsegs = (Segment*)(mem + o_sg);
        set_lds(frw_walk_kernel<false, false>, g.lds);
        set_lds(frw_walk_kernel<true, false>, g.lds);
        set_lds(frw_walk_kernel<false, false, true>, g.lds);
        set_lds(frw_walk_kernel<true, false, true>, g.lds);
        set_lds(frw_walk_kernel<false, true>, g.lds_e);
        set_lds(frw_walk_kernel<true, true>, g.lds_e);
        set_lds(frw_walk_kernel<false, true, true>, g.lds_e);
        set_lds(frw_walk_kernel<true, true, true>, g.lds_e);
        set_lds(first_kernel<false>, g.first_lds);
        set_lds(first_kernel<true>, g.first_lds);
        set_lds(frw_walk_kernel<false, false, false, true>, g.lds);
        set_lds(frw_walk_kernel<true, false, false, true>, g.lds);
        set_lds(frw_walk_kernel<false, false, true, true>, g.lds);
        set_lds(frw_walk_kernel<true, false, true, true>, g.lds);
        set_lds(first_kernel<false, true>, g.first_lds);
        set_lds(first_kernel<true, true>, g.first_lds);
    }
    ~Runner() {
        for (auto& e : evs) {
            (void)hipEventDestroy(e.first);
            (void)hipEventDestroy(e.second);
        }
        dev_free(dev_work);
        dev_free(mem);
    }

    // builds every table queued since the last call (binary64 solves);
    // returns how many
    size_t build_pending() {
        uint32_t npend = 0;
        MW_HIP(hipMemcpy(&npend, cache->d.n_pending, 4, hipMemcpyDeviceToHost));
        if (!npend) return 0;
        std::vector<uint32_t> list(npend);
        MW_HIP(hipMemcpy(list.data(), cache->d.pending, 4ull * npend, hipMemcpyDeviceToHost));
        std::vector<uint32_t> valid;
        for (uint32_t v : list)
            if (v < cache->d.capacity) valid.push_back(v);
        const uint32_t M = table_m(n);
        const size_t stride = (size_t)3 * M * M * M + (size_t)4 * 6 * M * M + 64;
        const uint32_t chunk = 512;
        double* work = (double*)dev_alloc(sizeof(double) * stride * std::min<size_t>(chunk, valid.size()));
        uint32_t* dlist = nullptr;
        try {
            dlist = (uint32_t*)dev_alloc(4ull * valid.size());
        } catch (...) {
            dev_free(work);
            throw;
        }
        struct G2 {
            void *a, *b;
            ~G2() {
                dev_free(a);
                dev_free(b);
            }
        } g2{work, dlist};
        MW_HIP(hipMemcpy(dlist, valid.data(), 4ull * valid.size(), hipMemcpyHostToDevice));
        for (size_t c0 = 0; c0 < valid.size(); c0 += chunk) {
            BuildArgs Ba{cache->d, dlist + c0, (uint32_t)std::min<size_t>(chunk, valid.size() - c0), work, stride};
            build_tables_kernel<<<Ba.count, TB_THREADS>>>(Ba);
            MW_HIP(hipGetLastError());
        }
        MW_HIP(hipDeviceSynchronize());
        MW_HIP(hipMemset(cache->d.n_pending, 0, 4));
        misses += valid.size();
        return valid.size();
    }

    // The cache-wide index of the uniform cube's table (another runner may
    // have emptied the cache since this one last ran).
    void ensure_uniform_table() {
        uniform_index = cache->uniform_index;
        for (int it = 0; it < 3 && uniform_index == NO_INDEX; ++it) {
            uniform_table_kernel<<<1, 1>>>(cache->d, n, status);
            MW_HIP(hipGetLastError());
            uint32_t res[2];
            MW_HIP(hipMemcpy(res, status, 8, hipMemcpyDeviceToHost));
            if (res[0] == LOOKUP_HIT)
                uniform_index = res[1];
            else if (res[0] == LOOKUP_FULL)
                flush_cache();
            else
                build_pending();
        }
        MW_REQUIRE(uniform_index != NO_INDEX, MW_EDEVICE, "uniform SGF table could not be built");
        cache->uniform_index = uniform_index;
    }

    // Empties the table cache when it is full.  Tables are pure functions of
    // their keys and a walk that finds the cache full parks as on a miss, so
    // the walks resume after the flush, rebuild what they need and keep
    // their results.  Called between launches, with the cache lock held.
    uint32_t flushes = 0;
    void flush_cache() {
        MW_REQUIRE(++flushes <= 4096, MW_ELIMIT,
                   "SGF table cache emptied 4096 times in one call (raise MWALK_TABLE_CAP)");
        cache->clear();
        uniform_index = NO_INDEX;
        ++cache->flushes;
        ensure_uniform_table();
    }

    // Handles a full cache reported by the last launch (the walks that met
    // it are parked or marked missing): the tables queued before it filled
    // are built first, so that the walks waiting for them move on; a cache
    // that is full with nothing queued is emptied.
    void after_launch(Counters& h) {
        if (h.err & ERR_TABLE_CAP) {
            if (build_pending() == 0) flush_cache();
            MW_HIP(hipMemset(&ctr->err, 0, 4));
            h.err &= ~(uint32_t)ERR_TABLE_CAP;
        }
        check_errors(h);
    }

    // The cached table of a key (built if missing), copied to the host.
    void fetch_table(const std::vector<uint32_t>& key, std::vector<uint32_t>& tab) {
        std::lock_guard<std::mutex> lock(cache->mu);
        flushes = 0;
        MW_REQUIRE(key.size() == cache->d.key_words, MW_EINVAL, "bad table key length");
        // the key goes to the status buffer's neighbour: the first parked
        // queue, unused outside walker runs
        uint32_t* dkey = reinterpret_cast<uint32_t*>(park[0]);
        MW_HIP(hipMemcpy(dkey, key.data(), 4 * key.size(), hipMemcpyHostToDevice));
        uint32_t res[2] = {LOOKUP_PARK, NO_INDEX};
        for (int it = 0; it < 4; ++it) {
            key_table_kernel<<<1, 1>>>(cache->d, dkey, status);
            MW_HIP(hipGetLastError());
            MW_HIP(hipMemcpy(res, status, 8, hipMemcpyDeviceToHost));
            if (res[0] == LOOKUP_HIT) break;
            if (res[0] == LOOKUP_FULL)
                flush_cache();
            else
                build_pending();
        }
        MW_REQUIRE(res[0] == LOOKUP_HIT, MW_EDEVICE, "SGF table could not be built");
        tab.resize(cache->d.tab_words);
        MW_HIP(hipMemcpy(tab.data(), cache->d.data + (size_t)res[1] * cache->d.tab_words, 4ull * tab.size(),
                         hipMemcpyDeviceToHost));
    }

    static void check_errors(const Counters& h) {
        MW_REQUIRE(!(h.err & ERR_REGIONS), MW_ELIMIT, "more than %d dielectric boxes overlap at one point",
                   MAX_REGIONS);
        MW_REQUIRE(!(h.err & ERR_PARK_CAP), MW_ELIMIT, "parked-walk queue overflow");
        MW_REQUIRE(!(h.err & ERR_STEP_CAP), MW_ELIMIT, "a micro-walk exceeded %u steps", MW_STEP_CAP);
    }

    // Zeroed counters and the segment list in one copy; returns the number
    // of walks (or points) of the list.
    unsigned long long upload(const std::vector<Segment>& segs, const StructDev* s0) {
        MW_REQUIRE((int)segs.size() <= seg_cap && !segs.empty(), MW_EINVAL, "bad segment list");
        MW_REQUIRE(segs.size() > 1 || s0, MW_EINVAL, "single-segment run without its structure");
        unsigned long long total = 0;
        for (const Segment& sgm : segs) total += sgm.count;
        MW_REQUIRE(total <= park_cap || total <= (1ull << 40), MW_ELIMIT, "round too large");
        const size_t off = (char*)dsegs - (char*)ctr;
        std::vector<char> staging(off + sizeof(Segment) * segs.size(), 0);
        memcpy(staging.data() + off, segs.data(), sizeof(Segment) * segs.size());
        MW_HIP(hipMemcpyAsync(ctr, staging.data(), staging.size(), hipMemcpyHostToDevice, stream));
        MW_HIP(hipStreamSynchronize(stream));  // the staging buffer goes out of scope
        built_seen = 0;                        // the counters restart at zero
        return total;
    }

    // The upload of a single-segment run (zeroed counters, then the segment)
    // as host bytes, for a copy that a graph replays.
    size_t staging_bytes(size_t nseg) const { return (size_t)((char*)dsegs - (char*)ctr) + sizeof(Segment) * nseg; }
    void fill_staging(const Segment& sg, char* buf) const {
        const size_t off = (char*)dsegs - (char*)ctr;
        memset(buf, 0, off);
        memcpy(buf + off, &sg, sizeof sg);
    }

    // start() of a single-segment run whose upload is already in pinned host
    // memory: nothing waits, so the calls can be captured in a graph.
    void start_from(const Segment& sg, const StructDev* s0, const char* pinned) {
        cur_segs = {sg};
        cur_single = true;
        cur_s0 = *s0;
        cur_total = sg.count;
        MW_HIP(hipMemcpyAsync(ctr, pinned, staging_bytes(1), hipMemcpyHostToDevice, stream));
        built_seen = 0;
        launch_first(cur_segs, &cur_s0, cur_total, 0, nullptr);
        launch_walker();
        for (int r = 0; r < DEVICE_ROUNDS; ++r) device_round();
    }

    // Per-call statistics start from zero (a runner kept between calls).
    void reset_stats() {
        misses = launches = 0;
        walker_ms = 0.0;
        flushes = 0;
    }

    // Adds the durations of the walker launches recorded since the last look.
    void account_events() {
        for (size_t i = 0; i < ev_used; ++i) {
            float ms = 0.f;
            MW_HIP(hipEventElapsedTime(&ms, evs[i].first, evs[i].second));
            walker_ms += ms;
        }
        ev_used = 0;
    }

    Counters read_counters() {
        Counters h{};
        MW_HIP(hipMemcpyAsync(&h, ctr, sizeof h, hipMemcpyDeviceToHost, stream));
        MW_HIP(hipStreamSynchronize(stream));
        account_events();
        misses += h.tables_built - built_seen;
        built_seen = h.tables_built;

        return h;
    }

    // One first-transition launch (round 0: every walk, writing its done
    // flag; later rounds: the walks still missing), without waiting.
    void launch_first(const std::vector<Segment>& segs, const StructDev* s0, unsigned long long total, int round,
                      const float4* eval, bool dev_round = false) {
        FirstArgs F{};
        F.eval = eval;
        F.segs = dsegs;
        F.n_segs = (int)segs.size();
        F.total = total;
        F.cache = cache->d;
        F.n = n;
        F.ctr = ctr;
        F.lane_stride = g.first_stride;
        if (segs.size() == 1) F.S0 = *s0;
        F.round = round;
        F.dev_round = dev_round ? 1 : 0;
        if (round > 0 && !dev_round) MW_HIP(hipMemsetAsync(&ctr->first_missing, 0, 4, stream));
        const int fblocks = (int)std::min<uint64_t>((total + FRW_THREADS - 1) / FRW_THREADS, (uint64_t)g.first_blocks);
        // odd n: the cell-centred lattice
        if (n & 1) {
            if (segs.size() == 1)
                first_kernel<false, true><<<fblocks, FRW_THREADS, g.first_lds, stream>>>(F);
            else
                first_kernel<true, true><<<fblocks, FRW_THREADS, g.first_lds, stream>>>(F);
        } else if (segs.size() == 1) {
            first_kernel<false><<<fblocks, FRW_THREADS, g.first_lds, stream>>>(F);
        } else {
            first_kernel<true><<<fblocks, FRW_THREADS, g.first_lds, stream>>>(F);
        }
        MW_HIP(hipGetLastError());
    }

    // One walker launch over the current run (fresh walks not yet taken and
    // the parked walks the counters name), without waiting.
    void launch_walker() {
        const bool multi = !cur_single;
        WalkArgs W{};
        W.segs = dsegs;
        W.n_segs = (int)cur_segs.size();
        W.total = cur_total;
        W.cache = cache->d;
        W.n = n;
        W.hybrid = hybrid;
        W.park[0] = park[0];
        W.park[1] = park[1];
        W.park_cap = park_cap;
        W.ctr = ctr;
        W.lane_stride = g.lane_stride;
        W.uniform_index = uniform_index;
        W.plain = plain;
        if (!multi) W.S0 = cur_s0;
        // one-wave blocks: the grid sets the resident waves per CU
        const int blocks = waves_per_cu > 0 ? std::min(g.blocks, g.cus * waves_per_cu) : g.blocks;
        const int blocks_e = waves_per_cu > 0 ? std::min(g.blocks_e, g.cus * waves_per_cu) : g.blocks_e;
        if (ev_used == evs.size()) {
            hipEvent_t a = nullptr, b = nullptr;
            MW_HIP(hipEventCreate(&a));
            if (hipEventCreate(&b) != hipSuccess) {
                (void)hipEventDestroy(a);
                MW_REQUIRE(false, MW_EDEVICE, "hipEventCreate failed");
            }
            evs.push_back({a, b});
        }
        const std::pair<hipEvent_t, hipEvent_t> ev = evs[ev_used++];
        MW_HIP(hipEventRecordWithFlags(ev.first, stream, hipEventRecordExternal));
        if (expand_m > 0) {
            W.lane_stride = g.lane_stride_e;
            W.expand_m = expand_m;
            if (multi && n <= 16)
                frw_walk_kernel<true, true, true><<<blocks_e, WALK_THREADS, g.lds_e, stream>>>(W);
            else if (multi)
                frw_walk_kernel<true, true><<<blocks_e, WALK_THREADS, g.lds_e, stream>>>(W);
            else if (n <= 16)
                frw_walk_kernel<false, true, true><<<blocks_e, WALK_THREADS, g.lds_e, stream>>>(W);
            else
                frw_walk_kernel<false, true><<<blocks_e, WALK_THREADS, g.lds_e, stream>>>(W);
        } else if (n & 1) {
            // the cell-centred lattice (register row masks up to 15 cells)
            if (multi && n <= 15)
                frw_walk_kernel<true, false, true, true><<<blocks, WALK_THREADS, g.lds, stream>>>(W);
            else if (multi)
                frw_walk_kernel<true, false, false, true><<<blocks, WALK_THREADS, g.lds, stream>>>(W);
            else if (n <= 15)
                frw_walk_kernel<false, false, true, true><<<blocks, WALK_THREADS, g.lds, stream>>>(W);
            else
                frw_walk_kernel<false, false, false, true><<<blocks, WALK_THREADS, g.lds, stream>>>(W);
        } else if (multi) {
            if (n <= 16)
                frw_walk_kernel<true, false, true><<<blocks, WALK_THREADS, g.lds, stream>>>(W);
            else
                frw_walk_kernel<true, false><<<blocks, WALK_THREADS, g.lds, stream>>>(W);
        } else {
            if (n <= 16)
                frw_walk_kernel<false, false, true><<<blocks, WALK_THREADS, g.lds, stream>>>(W);
            else
                frw_walk_kernel<false, false><<<blocks, WALK_THREADS, g.lds, stream>>>(W);
        }
        MW_HIP(hipGetLastError());
        MW_HIP(hipEventRecordWithFlags(ev.second, stream, hipEventRecordExternal));
        ++launches;
    }

    // One device-driven round, enqueued without waiting: build the queued
    // tables, redo first transitions that missed one, resume the parked
    // walks.  A round with nothing to do costs a few empty launches.
    size_t dev_work_stride() const {
        const uint32_t M = table_m(n);
        return (size_t)3 * M * M * M + (size_t)4 * 6 * M * M + 64;
    }
    void prepare_device_rounds() {
        if (!dev_work) dev_work = (double*)dev_alloc(sizeof(double) * dev_work_stride() * DEV_BUILD_MAX);
    }
    void device_round() {
        const size_t stride = dev_work_stride();
        prepare_device_rounds();
        BuildArgs Ba{cache->d, cache->d.pending, 0u, dev_work, stride, cache->d.n_pending, ctr};
        build_tables_kernel<<<DEV_BUILD_MAX, TB_THREADS, 0, stream>>>(Ba);
        device_round_prep_kernel<<<1, 1, 0, stream>>>(ctr, cache->d, DEV_BUILD_MAX, park_cap, cur_total);
        MW_HIP(hipGetLastError());
        launch_first(cur_segs, &cur_s0, cur_total, 1, nullptr, true);
        launch_walker();
    }

    // Enqueues a run without waiting: counters and segments, the first
    // transitions of every walk and one walker launch (walks whose first
    // transition missed its table park until finish()).  The caller holds the
    // cache lock and has called ensure_uniform_table().
    void start(const std::vector<Segment>& segs, const StructDev* s0) {
        cur_segs = segs;
        cur_single = segs.size() == 1;
        if (cur_single) cur_s0 = *s0;
        cur_total = upload(segs, s0);
        launch_first(cur_segs, &cur_s0, cur_total, 0, nullptr);
        launch_walker();
        for (int r = 0; r < DEVICE_ROUNDS; ++r) device_round();
    }

    // Waits for the started run and completes it: missing tables are built,
    // first transitions that missed them are redone and parked walks resume,
    // until every walk has ended.  Builds run with no other FRW work in
    // flight on the device (the caller's guarantee).
    Counters finish() { return finish_from(read_counters()); }

    // finish() after the caller has read the counters of the first launch
    Counters finish_from(Counters h) {
        for (uint64_t local = 1;; ++local) {
            after_launch(h);
            if (h.first_missing > 0) {
                build_pending();
                first_rounds(cur_segs, &cur_s0, cur_total, nullptr, 1);
                h = read_counters();
            }
            // a lane that queued a table parked its walk
            if (h.park_count > 0) build_pending();
            if (h.park_count == 0 && h.walk_next >= cur_total) return h;
            MW_REQUIRE(local < 100000, MW_ELIMIT, "walker relaunch limit reached");
            // the parked walks resume; the walk counter is kept
            resume_prep_kernel<<<1, 1, 0, stream>>>(ctr, park_cap, cur_total);
            launch_walker();
            h = read_counters();
        }
    }

    // First-kernel rounds until no walk misses a table (eval: the kernel
    // sums K / h at given points instead of sampling first transitions).
    void first_rounds(const std::vector<Segment>& segs, const StructDev* s0, unsigned long long total,
                      const float4* eval, int first_round = 0) {
        for (int round = first_round;; ++round) {
            launch_first(segs, s0, total, round, eval);
            Counters h = read_counters();
            after_launch(h);
            MW_REQUIRE(round < 1000, MW_ELIMIT, "first-transition retry limit reached");
            if (h.first_missing == 0) break;  // no walk missed a table, so none was queued
            build_pending();
        }
    }

    // K / h of the first-transition kernel at each point of eval (device,
    // count entries, w = axis | side << 2 bits) on Gaussian surface G of
    // structure s0; written to out[k].x (device).
    void evaluate(const StructDev& s0, StructDev* dS, GaussDev* G, const float4* eval, uint64_t count, float4* out,
                  uint32_t* done) {
        std::lock_guard<std::mutex> lock(cache->mu);
        flushes = 0;
        ensure_uniform_table();
        Segment sgm{};
        sgm.S = dS;
        sgm.G = G;
        sgm.count = count;
        sgm.first_state = out;
        sgm.first_done = done;
        const std::vector<Segment> segs{sgm};
        first_rounds(segs, &s0, upload(segs, &s0), eval);
    }

    // Runs every walk of segs to its end (synchronous).  s0: host copy of
    // the structure header of a single segment.
    Counters run(const std::vector<Segment>& segs, const StructDev* s0) {
        std::lock_guard<std::mutex> lock(cache->mu);
        flushes = 0;
        ensure_uniform_table();
        start(segs, s0);
        return finish();
    }
};

}  // namespace

extern "C" mw_status mw_table_cache_clear(int32_t n_cells) {
    return guarded([&] {
        MW_REQUIRE(n_cells >= 3 && n_cells <= 32, MW_EINVAL,
                   "table lattice size must be 4..32 (even, vertex lattice) or 3..31 (odd, cell lattice)");
        Cache& c = get_cache(n_cells);
        std::lock_guard<std::mutex> lock(c.mu);
        c.clear();
    });
}

extern "C" mw_status mw_sgf_table(int32_t n_cells, int32_t kind, int32_t axis, int32_t normal_axis,
                                  const uint32_t* plane_codes, uint32_t* cdf, uint32_t* sign_bits, float* kh) {
    return guarded([&] {
        MW_REQUIRE(n_cells >= 3 && n_cells <= 32, MW_EINVAL,
                   "table lattice size must be 4..32 (even, vertex lattice) or 3..31 (odd, cell lattice)");
        MW_REQUIRE(kind == 0 || kind == 1, MW_EINVAL, "kind must be 0 (hop) or 1 (first transition)");
        const bool cell = (n_cells & 1) != 0;
        MW_REQUIRE(axis >= 0 && axis < 3, MW_EINVAL, "axis must be 0, 1 or 2");
        MW_REQUIRE(kind == 0 || (normal_axis >= 0 && normal_axis < 3), MW_EINVAL, "normal axis must be 0, 1 or 2");
        MW_REQUIRE(plane_codes && cdf, MW_EINVAL, "null plane codes or CDF buffer");
        const int n = n_cells;
        for (int p = 0; p < n; ++p) {
            if (cell) {
                float e;
                std::memcpy(&e, &plane_codes[p], 4);
                MW_REQUIRE(e >= 1e-3f && e <= 1e3f, MW_EINVAL, "plane permittivity outside [1e-3, 1e3]");
            } else {
                MW_REQUIRE(plane_codes[p] >= 66u && plane_codes[p] <= 65536000u, MW_EINVAL,
                           "plane code outside rint(eps * 2^16) for eps in [1e-3, 1e3]");
            }
        }
        std::vector<uint32_t> key(KEY_HDR + n);
        key[0] = (uint32_t)kind + (cell ? 2u : 0u);
        key[1] = (uint32_t)n;
        key[2] = (uint32_t)axis;
        key[3] = kind == 1 ? (uint32_t)normal_axis : 0u;
        for (int p = 0; p < n; ++p) key[KEY_HDR + p] = plane_codes[p];
        Runner R(n, 1, 0, 1);
        std::vector<uint32_t> tab;
        R.fetch_table(key, tab);
        const uint32_t nb = 6u * table_m(n) * table_m(n);
        memcpy(cdf, tab.data() + TAB_CDF, 4ull * nb);
        if (sign_bits) memcpy(sign_bits, tab.data() + TAB_CDF + nb, 4ull * ((nb + 31) / 32));
        if (kh) memcpy(kh, tab.data() + 1, 4);
    });
}

namespace {

// Gaussian surface of a net (Alg. 1 input G) as a list of axis-aligned
// rectangles.  G is the boundary of the union of the net's boxes, each grown by
// g on every side, where g is half the smallest L-infinity gap between a box of
// the net and a box of another net or a grounded window face; a net of one box
// gets the six faces of its grown box.  Pieces on planes outside the open
// window are dropped (a symmetry wall closes the surface there and carries no
// flux) and the rest are clipped to the window.  Each grown face is cut along
// the extents of the grown boxes that reach its plane; a piece is kept when
// the space just outside it belongs to no other grown box and no earlier box
// of the net has a coplanar face with the same outward normal over it.
// Returns 0, or 1 (no box), 2 (no positive gap), 3 (empty surface),
// 4 (too many pieces).
constexpr size_t GAUSS_MAX_FACES = 1 << 16;
constexpr size_t GAUSS_MAX_PATCHES = 1 << 22;

// frw_extract: walks between two checks of the stopping rule (default), most
// walks per launch, and the first launch of an extraction with no size hint
constexpr uint64_t FRW_CHECKPOINT = 1u << 16;
constexpr uint64_t FRW_LAUNCH_CAP = 1ull << 26;         // fixed budget
constexpr uint64_t FRW_TARGET_LAUNCH_CAP = 1ull << 23;  // with a target (buffers sized for it)
constexpr uint64_t FRW_FIRST_LAUNCH = 1u << 20;

struct GaussHost {
    double g = 0, area = 0;
    std::vector<GaussFace> faces;
    std::vector<double> rect;  // per rectangle: plane, lo, hi (lower tangent axis), lo, hi (higher), binary64
};

int gauss_surface(const mw_structure& st, int master, GaussHost& out) {
    struct Grown {
        double lo[3], hi[3];
    };
    std::vector<Grown> B;
    for (const mw_cond_box& b : st.cond)
        if (b.net == master) B.push_back({{b.lo[0], b.lo[1], b.lo[2]}, {b.hi[0], b.hi[1], b.hi[2]}});
    if (B.empty()) return 1;
    const StructDev& S = st.h;
    double g0 = INFINITY;
    for (const mw_cond_box& o : st.cond) {
        if (o.net == master) continue;
        for (const Grown& m : B) {
            double gap = 0;
            for (int a = 0; a < 3; ++a) gap = std::max(gap, std::max((double)o.lo[a] - m.hi[a], m.lo[a] - (double)o.hi[a]));
            g0 = std::min(g0, gap);
        }
    }
    for (const Grown& m : B)
        for (int a = 0; a < 3; ++a) {
            if (S.bc[2 * a] == MW_BC_DIRICHLET) g0 = std::min(g0, m.lo[a] - (double)S.wlo[a]);
            if (S.bc[2 * a + 1] == MW_BC_DIRICHLET) g0 = std::min(g0, (double)S.whi[a] - m.hi[a]);
        }
    if (!(g0 > 0) || !std::isfinite(g0)) return 2;
    const double g = 0.5 * g0;
    for (Grown& m : B)
        for (int a = 0; a < 3; ++a) {
            m.lo[a] -= g;
            m.hi[a] += g;
        }
    out.g = g;
    out.area = 0;
    out.faces.clear();
    const int nb = (int)B.size();
    std::vector<int> near;
    std::vector<double> cu, cv;
    for (int i = 0; i < nb; ++i)
        for (int a = 0; a < 3; ++a)
            for (int side = 0; side < 2; ++side) {
                const double p = side ? B[i].hi[a] : B[i].lo[a];
                if (!(p > S.wlo[a] && p < S.whi[a])) continue;
                const int ta = a == 0 ? 1 : 0, tb = a == 2 ? 1 : 2;
                const double u0 = std::max(B[i].lo[ta], (double)S.wlo[ta]), u1 = std::min(B[i].hi[ta], (double)S.whi[ta]);
                const double v0 = std::max(B[i].lo[tb], (double)S.wlo[tb]), v1 = std::min(B[i].hi[tb], (double)S.whi[tb]);
                if (!(u0 < u1 && v0 < v1)) continue;
                // grown boxes that reach the plane over the face
                near.clear();
                for (int j = 0; j < nb; ++j)
                    if (j != i && B[j].lo[a] <= p && p <= B[j].hi[a] && B[j].lo[ta] < u1 && B[j].hi[ta] > u0 &&
                        B[j].lo[tb] < v1 && B[j].hi[tb] > v0)
                        near.push_back(j);
                cu.assign({u0, u1});
                cv.assign({v0, v1});
                for (int j : near) {
                    for (double x : {B[j].lo[ta], B[j].hi[ta]})
                        if (x > u0 && x < u1) cu.push_back(x);
                    for (double x : {B[j].lo[tb], B[j].hi[tb]})
                        if (x > v0 && x < v1) cv.push_back(x);
                }
                std::sort(cu.begin(), cu.end());
                cu.erase(std::unique(cu.begin(), cu.end()), cu.end());
                std::sort(cv.begin(), cv.end());
                cv.erase(std::unique(cv.begin(), cv.end()), cv.end());
                for (size_t iu = 0; iu + 1 < cu.size(); ++iu)
                    for (size_t iv = 0; iv + 1 < cv.size(); ++iv) {
                        const double qu = 0.5 * (cu[iu] + cu[iu + 1]), qv = 0.5 * (cv[iv] + cv[iv + 1]);
                        bool keep = true;
                        for (int j : near) {
                            if (!(B[j].lo[ta] < qu && qu < B[j].hi[ta] && B[j].lo[tb] < qv && qv < B[j].hi[tb]))
                                continue;
                            // another grown box just outside the piece
                            const bool outside = side ? (B[j].lo[a] <= p && p < B[j].hi[a])
                                                      : (B[j].lo[a] < p && p <= B[j].hi[a]);
                            // an earlier coplanar face with the same normal
                            const bool earlier = j < i && (side ? B[j].hi[a] == p : B[j].lo[a] == p);
                            if (outside || earlier) {
                                keep = false;
                                break;
                            }
                        }
                        if (!keep) continue;
                        const double ar = (cu[iu + 1] - cu[iu]) * (cv[iv + 1] - cv[iv]);
                        if (!(ar > 0)) continue;
                        if (out.faces.size() >= GAUSS_MAX_FACES) return 4;
                        out.area += ar;
                        GaussFace F;
                        const uint32_t bits = (uint32_t)a | (uint32_t)side << 2;
                        float fbits;
                        memcpy(&fbits, &bits, 4);
                        F.p = make_float4((float)p, (float)out.area, fbits, 0.f);
                        F.t = make_float4((float)cu[iu], (float)cu[iu + 1], (float)cv[iv], (float)cv[iv + 1]);
                        out.faces.push_back(F);
                        out.rect.insert(out.rect.end(), {p, cu[iu], cu[iu + 1], cv[iv], cv[iv + 1]});
                    }
            }
    if (out.faces.empty()) return 3;
    return 0;
}

// Device state of one extraction: structure copy with the call's absorption
// tolerance, Gaussian surface, per-walk buffers of one chunk and the fp64
// accumulators.
struct Extraction {
    int K = 0, master = 0;
    uint64_t chunk_cap = 0;
    char* mem = nullptr;
    StructDev* dS;
    GaussDev* G;
    float4* partial;
    double* acc;
    double* result;
    Choice* choice;
    int32_t* score_net;
    float* score_w;
    float4* first_state;
    uint32_t* first_done;
    uint64_t done = 0;      // walks in the sums
    uint64_t launched = 0;  // walks walked, including those after the stopping checkpoint
    std::vector<double> res;

    static size_t bytes(int K, uint64_t chunk_cap, bool chunk_buffers = true, size_t n_faces = 6) {
        const uint64_t red_blocks = (chunk_cap + RED_CHUNK - 1) / RED_CHUNK;
        return 256 * 12 + sizeof(StructDev) + sizeof(GaussDev) + sizeof(GaussFace) * n_faces +
               sizeof(float4) * red_blocks * K + sizeof(double) * 4 * K +
               (chunk_buffers ? chunk_cap * (4 + 4 + 16 + 4) : 0);
    }
    size_t n_faces = 0;
    double gauss_g = 0, gauss_area = 0;
    StructDev hS{};  // host copy of the device structure header
    std::vector<GaussFace> faces_h;  // the surface's rectangles (uniform sampling)
    std::vector<double> rect_h;      // their binary64 bounds
    char* patch_mem = nullptr;       // importance-sampling patches (device)
    size_t n_patches = 0;

    Extraction(const mw_structure& st, int master_, double abs_tol_rel, uint64_t chunk_cap_, bool own_scores,
               bool own_first = true)
        : K(st.n_nets + 1), master(master_), chunk_cap(chunk_cap_) {
        GaussHost GH;
        const int gst = gauss_surface(st, master, GH);
        MW_REQUIRE(gst != 4, MW_ELIMIT, "Gaussian surface of net %d needs more than %zu rectangles", master,
                   GAUSS_MAX_FACES);
        MW_REQUIRE(gst == 0, MW_EGEOM, "no valid Gaussian surface for net %d (status %d)", master, gst);
        n_faces = GH.faces.size();
        gauss_g = GH.g;
        gauss_area = GH.area;
        // uniform sampling: every rectangle's weight factor is |G|
        for (GaussFace& F : GH.faces) F.p.w = (float)GH.area;
        faces_h = GH.faces;
        rect_h = GH.rect;
        size_t o = 0;
        auto sz = [&](size_t b) {
            size_t r = o;
            o += (b + 255) / 256 * 256;
            return r;
        };
        const uint64_t red_blocks = (chunk_cap + RED_CHUNK - 1) / RED_CHUNK;
        const size_t o_sd = sz(sizeof(StructDev)), o_G = sz(sizeof(GaussDev)), o_gf = sz(sizeof(GaussFace) * n_faces);
        const size_t o_acc = sz(sizeof(double) * 2 * K);  // zeroed by the same copy
        const size_t o_part = sz(sizeof(float4) * red_blocks * K);
        const size_t o_res = sz(sizeof(double) * 2 * K + sizeof(Choice));  // the choice follows the row
        const size_t o_fs = own_first ? sz(sizeof(float4) * chunk_cap) : 0;
        const size_t o_fd = own_first ? sz(sizeof(uint32_t) * chunk_cap) : 0;
        const size_t o_sn = own_scores ? sz(4 * chunk_cap) : 0, o_sw = own_scores ? sz(4 * chunk_cap) : 0;
        mem = (char*)dev_alloc(o);
        dS = (StructDev*)(mem + o_sd);
        G = (GaussDev*)(mem + o_G);
        partial = (float4*)(mem + o_part);
        acc = (double*)(mem + o_acc);
        result = (double*)(mem + o_res);
        choice = (Choice*)(result + 2 * K);
        first_state = own_first ? (float4*)(mem + o_fs) : nullptr;
        first_done = own_first ? (uint32_t*)(mem + o_fd) : nullptr;
        score_net = own_scores ? (int32_t*)(mem + o_sn) : nullptr;
        score_w = own_scores ? (float*)(mem + o_sw) : nullptr;
        StructDev S = st.h;
        double diag = 0;
        for (int a = 0; a < 3; ++a) diag += (double)(S.whi[a] - S.wlo[a]) * (S.whi[a] - S.wlo[a]);
        S.delta_abs = (float)(abs_tol_rel * std::sqrt(diag));
        hS = S;
        GaussDev Gh{};
        Gh.g = (float)GH.g;
        Gh.area = (float)GH.area;
        Gh.n_faces = (int32_t)n_faces;
        Gh.faces = (const GaussFace*)(mem + o_gf);
        // one host-to-device copy of the structure header, the surface header,
        // its rectangles and the zeroed fp64 sums (laid out as on the device)
        std::vector<char> staging(o_acc + sizeof(double) * 2 * K - o_sd, 0);
        memcpy(staging.data(), &S, sizeof S);
        memcpy(staging.data() + (o_G - o_sd), &Gh, sizeof Gh);
        memcpy(staging.data() + (o_gf - o_sd), GH.faces.data(), sizeof(GaussFace) * n_faces);
        hipStream_t cs = setup_stream();
        MW_HIP(hipMemcpyAsync(mem + o_sd, staging.data(), staging.size(), hipMemcpyHostToDevice, cs));
        MW_HIP(hipStreamSynchronize(cs));
        res.assign(2 * K, 0.0);
    }
    ~Extraction() {
        dev_free(patch_mem);
        dev_free(mem);
    }

    // Importance sampling of the Gaussian-surface point (the first
    // transition of Alg. 1 is importance sampling with its weight): each
    // rectangle is cut into nu x nv equal patches, nu = ceil(length / edge),
    // and patch p is drawn with probability q_p / Q, q_p = area_p K(c_p) / h
    // (the first-transition kernel sum at the patch centre, evaluated by the
    // first-transition kernel itself), then a uniform point on it; the
    // walk's weight uses Q area_p / q_p in place of |G|, so the estimator is
    // unchanged in expectation.
    void importance(Runner& R, double edge) {
        std::vector<double> pb;  // plane, u0, u1, v0, v1 per patch
        std::vector<uint32_t> bits;
        for (size_t f = 0; f < faces_h.size(); ++f) {
            const double* r = &rect_h[5 * f];
            const double la = r[2] - r[1], lb = r[4] - r[3];
            const int nu = std::max(1, (int)std::ceil(la / edge)), nv = std::max(1, (int)std::ceil(lb / edge));
            MW_REQUIRE((double)nu * nv + (double)bits.size() <= (double)GAUSS_MAX_PATCHES, MW_ELIMIT,
                       "importance sampling needs more than %zu patches", GAUSS_MAX_PATCHES);
            uint32_t fb;
            memcpy(&fb, &faces_h[f].p.z, 4);
            for (int j = 0; j < nv; ++j)
                for (int i = 0; i < nu; ++i) {
                    pb.insert(pb.end(), {r[0], r[1] + la * i / nu, r[1] + la * (i + 1) / nu, r[3] + lb * j / nv,
                                         r[3] + lb * (j + 1) / nv});
                    bits.push_back(fb);
                }
        }
        const size_t np = bits.size();
        dev_free(patch_mem);
        patch_mem = nullptr;
        const size_t o_eval = 0, o_out = o_eval + 16 * np, o_done = o_out + 16 * np;
        const size_t o_faces = (o_done + 4 * np + 255) / 256 * 256;
        patch_mem = (char*)dev_alloc(o_faces + sizeof(GaussFace) * np);
        std::vector<float4> ev(np);
        for (size_t k = 0; k < np; ++k) {
            const double* q = &pb[5 * k];
            const int a = (int)(bits[k] & 3u);
            const int ta = a == 0 ? 1 : 0, tb = a == 2 ? 1 : 2;
            double c[3];
            c[a] = q[0];
            c[ta] = 0.5 * (q[1] + q[2]);
            c[tb] = 0.5 * (q[3] + q[4]);
            float fb;
            memcpy(&fb, &bits[k], 4);
            ev[k] = make_float4((float)c[0], (float)c[1], (float)c[2], fb);
        }
        MW_HIP(hipMemcpy(patch_mem + o_eval, ev.data(), 16 * np, hipMemcpyHostToDevice));
        R.evaluate(hS, dS, G, (const float4*)(patch_mem + o_eval), np, (float4*)(patch_mem + o_out),
                   (uint32_t*)(patch_mem + o_done));
        std::vector<float4> kv(np);
        MW_HIP(hipMemcpy(kv.data(), patch_mem + o_out, 16 * np, hipMemcpyDeviceToHost));
        std::vector<double> q(np);
        double Q = 0;
        for (size_t k = 0; k < np; ++k) {
            const double* b = &pb[5 * k];
            const double area = (b[2] - b[1]) * (b[4] - b[3]);
            q[k] = area * (double)kv[k].x;
            MW_REQUIRE(q[k] > 0, MW_EDEVICE, "importance-sampling patch %zu has no weight", k);
            Q += q[k];
        }
        std::vector<GaussFace> F(np);
        double cum = 0;
        for (size_t k = 0; k < np; ++k) {
            const double* b = &pb[5 * k];
            const double area = (b[2] - b[1]) * (b[4] - b[3]);
            cum += q[k];
            float fb;
            memcpy(&fb, &bits[k], 4);
            F[k].p = make_float4((float)b[0], (float)cum, fb, (float)(Q * area / q[k]));
            F[k].t = make_float4((float)b[1], (float)b[2], (float)b[3], (float)b[4]);
        }
        MW_HIP(hipMemcpy(patch_mem + o_faces, F.data(), sizeof(GaussFace) * np, hipMemcpyHostToDevice));
        GaussDev Gh{};
        Gh.g = (float)gauss_g;
        Gh.area = (float)Q;
        Gh.n_faces = (int32_t)np;
        Gh.faces = (const GaussFace*)(patch_mem + o_faces);
        MW_HIP(hipMemcpy(G, &Gh, sizeof Gh, hipMemcpyHostToDevice));
        n_patches = np;
    }

    // Segment for walks [first, first + count) writing scores to net/w (or
    // the extraction's own buffers from entry `at` on).
    Segment segment(uint64_t first, uint64_t count, uint64_t seed, int32_t* net, float* w, uint64_t at = 0) {
        MW_REQUIRE(at + count <= chunk_cap, MW_EINVAL, "chunk larger than its buffers");
        Segment s{};
        s.S = dS;
        s.G = G;
        s.walk_begin = first;
        s.count = count;
        s.score_net = net ? net : score_net + at;
        s.score_w = w ? w : score_w + at;
        s.first_state = first_state + at;
        s.first_done = first_done + at;
        s.k0 = (uint32_t)seed;
        s.k1 = (uint32_t)(seed >> 32);
        return s;
    }

    // bytes of a launch's result copy: the row and its standard errors, then
    // the choice of the stopping rule
    size_t out_bytes() const { return sizeof(double) * 2 * K + sizeof(Choice); }

    // The reduction, the stopping rule and the binary64 sums of a launch's
    // scores (gated on the walker's counters, or not when gate is null), and
    // the copy of the result to out (host).  Nothing waits.
    void enqueue_tail(Runner& R, const Segment& sg, int per_ck, double target, const Counters* gate, char* out) {
        const int rb = (int)((sg.count + RED_CHUNK - 1) / RED_CHUNK);
        reduce_scores_kernel<<<rb, RED_THREADS, 0, R.stream>>>(sg.score_net, sg.score_w, sg.count, K, partial, gate,
                                                                sg.count);
        decide_kernel<<<1, 64, 0, R.stream>>>(partial, rb, K, master, per_ck, acc, (double)done, sg.count, target,
                                              gate, sg.count, choice);
        finish_seq_kernel<<<K, 64, 0, R.stream>>>(partial, K, acc, (double)done, choice, result);
        MW_HIP(hipGetLastError());
        MW_HIP(hipMemcpyAsync(out, result, out_bytes(), hipMemcpyDeviceToHost, R.stream));
    }

    // After the gated tail of a launch has run (counters h, result copy in
    // out): when the gate was closed the launch's walks are completed and the
    // tail runs again ungated; then the sums move on.
    Counters complete(Runner& R, const Segment& sg, int per_ck, double target, Counters h, char* out, bool* met) {
        Choice c;
        memcpy(&c, out + sizeof(double) * 2 * K, sizeof c);
        if (c.blocks < 0) {
            h = R.finish_from(h);
            enqueue_tail(R, sg, per_ck, target, nullptr, out);
            MW_HIP(hipStreamSynchronize(R.stream));
            memcpy(&c, out + sizeof(double) * 2 * K, sizeof c);
        } else {
            R.check_errors(h);
        }
        MW_REQUIRE(c.blocks >= 0 && c.walks <= sg.count, MW_EDEVICE, "stopping rule returned no choice");
        done += c.walks;
        launched += sg.count;
        memcpy(res.data(), out, sizeof(double) * 2 * K);
        *met = c.met != 0;
        return h;
    }

    // One launch of walks [done, done + sg.count) (done is a checkpoint)
    // with a single wait in the usual case: the walks, then the gated
    // reduction, stopping rule and binary64 sums, and one copy of the row and
    // the choice.  Returns the walker counters; *met tells whether the
    // target was met.
    Counters run_launch(Runner& R, const Segment& sg, int per_ck, double target, bool* met) {
        std::vector<char> out(out_bytes());
        R.start({sg}, &hS);
        enqueue_tail(R, sg, per_ck, target, R.ctr, out.data());
        const Counters h = R.read_counters();  // waits for the stream
        return complete(R, sg, per_ck, target, h, out.data(), met);
    }

    // A kept extraction starts again from zero walks.
    void reset(hipStream_t stream) {
        done = launched = 0;
        res.assign(2 * K, 0.0);
        MW_HIP(hipMemsetAsync(acc, 0, sizeof(double) * 2 * K, stream));
    }

    bool converged(double target) const {
        return target > 0 && res[master] != 0.0 && 3.0 * res[K + master] / std::fabs(res[master]) <= target;
    }
};

// frw_extract's buffers kept with the structure between calls: the
// extraction's device arrays, the runner's queues and events, a stream of
// their own, and HIP graphs of the usual launch (upload, first transitions,
// walker, device-driven rounds, gated reduction, stopping rule, sums and the
// copies back), replayed when a call's launch has the same shape.  Replays
// run the same kernels with the same arguments as the eager launch, so
// results do not depend on which ran.  A graph holds no memset node.
struct ExtractCtx {
    // what the buffers depend on
    int master = 0, n = 0, hybrid = 0, expand_m = 0, plain = 0;
    double abs_tol_rel = 0.0, gauss_is = 0.0;
    uint64_t chunk = 0;
    bool own_scores = true;
    bool busy = false;
    uint64_t last_use = 0;
    std::unique_ptr<Extraction> X;
    std::unique_ptr<Runner> R;
    hipStream_t stream = nullptr;
    char* host_in = nullptr;   // pinned: the upload of a launch
    char* host_out = nullptr;  // pinned: the result copy, then the counters
    bool graphs_ok = true;
    struct Graph {
        uint64_t done, count;
        int per_ck;
        double target;
        uint32_t uniform_index;
        int waves_per_cu;
        hipGraphExec_t exec;
        uint64_t launches;
        std::vector<std::pair<hipEvent_t, hipEvent_t>> events;  // around its walker launches
    };
    std::vector<Graph> graphs;

    ~ExtractCtx() {
        for (Graph& g : graphs) {
            (void)hipGraphExecDestroy(g.exec);
            destroy_events(g.events);
        }
        if (host_in) (void)hipHostFree(host_in);
        if (host_out) (void)hipHostFree(host_out);
        R.reset();
        X.reset();
        if (stream) (void)hipStreamDestroy(stream);
    }

    static void destroy_events(std::vector<std::pair<hipEvent_t, hipEvent_t>>& ev) {
        for (auto& e : ev) {
            (void)hipEventDestroy(e.first);
            (void)hipEventDestroy(e.second);
        }
        ev.clear();
    }

    size_t out_counters_offset() const { return (X->out_bytes() + 255) / 256 * 256; }

    // A graph of the launch of sg, captured on first use of its shape.
    Graph* graph_for(const Segment& sg, int per_ck, double target) {
        for (Graph& g : graphs)
            if (g.done == X->done && g.count == sg.count && g.per_ck == per_ck && g.target == target &&
                g.uniform_index == R->uniform_index && g.waves_per_cu == R->waves_per_cu)
                return &g;
        if (graphs.size() >= 8) return nullptr;
        Graph g{X->done, sg.count, per_ck, target, R->uniform_index, R->waves_per_cu, nullptr, 0, {}};
        R->account_events();  // the pool's pairs are free again
        const uint64_t l0 = R->launches;
        hipGraph_t graph = nullptr;
        R->prepare_device_rounds();  // no allocation inside the capture
        MW_HIP(hipStreamBeginCapture(stream, hipStreamCaptureModeRelaxed));
        bool captured = true;
        try {
            R->start_from(sg, &X->hS, host_in);
            X->enqueue_tail(*R, sg, per_ck, target, R->ctr, host_out);
            MW_HIP(hipMemcpyAsync(host_out + out_counters_offset(), R->ctr, sizeof(Counters), hipMemcpyDeviceToHost,
                                  stream));
        } catch (...) {
            captured = false;
        }
        const hipError_t ee = hipStreamEndCapture(stream, &graph);
        g.launches = R->launches - l0;
        // the event pairs recorded in the graph belong to it from now on
        g.events.assign(R->evs.begin(), R->evs.begin() + R->ev_used);
        R->evs.erase(R->evs.begin(), R->evs.begin() + R->ev_used);
        R->ev_used = 0;
        R->launches = l0;
        hipGraphExec_t exec = nullptr;
        if (captured && ee == hipSuccess && graph && hipGraphInstantiate(&exec, graph, nullptr, nullptr, 0) == hipSuccess) {
            (void)hipGraphDestroy(graph);
            (void)hipGetLastError();
            g.exec = exec;
            graphs.push_back(std::move(g));
            return &graphs.back();
        }
        // capture not possible here: eager launches from now on
        if (graph) (void)hipGraphDestroy(graph);
        destroy_events(g.events);
        (void)hipGetLastError();
        graphs_ok = false;
        return nullptr;
    }

    // One launch as Extraction::run_launch, replayed from a graph when the
    // segment uses the extraction's own buffers.
    Counters run_launch(const Segment& sg, int per_ck, double target, bool* met) {
        if (!graphs_ok || !own_scores || !env_size("MWALK_FRW_GRAPHS", 1))
            return X->run_launch(*R, sg, per_ck, target, met);
        R->fill_staging(sg, host_in);
        Graph* g = graph_for(sg, per_ck, target);
        if (!g) return X->run_launch(*R, sg, per_ck, target, met);
        MW_HIP(hipGraphLaunch(g->exec, stream));
        MW_HIP(hipStreamSynchronize(stream));
        R->launches += g->launches;
        for (auto& e : g->events) {
            float ms = 0.f;
            MW_HIP(hipEventElapsedTime(&ms, e.first, e.second));
            R->walker_ms += ms;
        }
        // the runner's view of the run, as start() leaves it
        R->cur_segs = {sg};
        R->cur_single = true;
        R->cur_s0 = X->hS;
        R->cur_total = sg.count;
        Counters h;
        memcpy(&h, host_out + out_counters_offset(), sizeof h);
        R->misses += h.tables_built;
        R->built_seen = h.tables_built;
        return X->complete(*R, sg, per_ck, target, h, host_out, met);
    }
};

void delete_ctx(ExtractCtx* c) { delete c; }

// The context of a call (created when no idle one matches; at most four
// are kept per structure, the least recently used idle one making room).
struct CtxLease {
    mw_structure* st;
    ExtractCtx* c = nullptr;
    bool kept = true;
    CtxLease(mw_structure* st_, int master, const frw_options& opt, int expand_m, uint64_t chunk, bool own)
        : st(st_) {
        {
            std::lock_guard<std::mutex> g(st->ctx_mu);
            for (ExtractCtx* x : st->ctxs)
                if (!x->busy && x->master == master && x->n == opt.n_cells && x->hybrid == opt.hybrid &&
                    x->expand_m == expand_m && x->plain == opt.plain && x->abs_tol_rel == opt.abs_tol_rel &&
                    x->gauss_is == opt.gauss_is && x->chunk == chunk && x->own_scores == own) {
                    c = x;
                    break;
                }
            if (c) {
                c->busy = true;
                c->last_use = ++st->ctx_clock;
                return;
            }
        }
        auto x = std::make_unique<ExtractCtx>();
        x->master = master;
        x->n = opt.n_cells;
        x->hybrid = opt.hybrid;
        x->expand_m = expand_m;
        x->plain = opt.plain;
        x->abs_tol_rel = opt.abs_tol_rel;
        x->gauss_is = opt.gauss_is;
        x->chunk = chunk;
        x->own_scores = own;
        MW_HIP(hipStreamCreateWithFlags(&x->stream, hipStreamNonBlocking));
        x->X = std::make_unique<Extraction>(*st, master, opt.abs_tol_rel, chunk, own);
        x->R = std::make_unique<Runner>(opt.n_cells, opt.hybrid, chunk, 1);
        x->R->stream = x->stream;
        x->R->expand_m = expand_m;
        x->R->plain = opt.plain;
        MW_HIP(hipHostMalloc((void**)&x->host_in, x->R->staging_bytes(1), 0));
        MW_HIP(hipHostMalloc((void**)&x->host_out, x->out_counters_offset() + sizeof(Counters), 0));
        if (opt.gauss_is > 0) x->X->importance(*x->R, opt.gauss_is * x->X->gauss_g);
        x->busy = true;
        std::lock_guard<std::mutex> g(st->ctx_mu);
        x->last_use = ++st->ctx_clock;
        if (st->ctxs.size() >= 4) {
            size_t victim = st->ctxs.size();
            for (size_t i = 0; i < st->ctxs.size(); ++i)
                if (!st->ctxs[i]->busy && (victim == st->ctxs.size() || st->ctxs[i]->last_use < st->ctxs[victim]->last_use))
                    victim = i;
            if (victim < st->ctxs.size()) {
                delete st->ctxs[victim];
                st->ctxs.erase(st->ctxs.begin() + victim);
            }
        }
        if (st->ctxs.size() < 4)
            st->ctxs.push_back(x.get());
        else
            kept = false;  // every kept context is in use: this one lives for the call
        c = x.release();
    }
    ~CtxLease() {
        if (!c) return;
        if (!kept) {
            delete c;
            return;
        }
        std::lock_guard<std::mutex> g(st->ctx_mu);
        c->busy = false;
    }
};

frw_options normalised_options(const frw_options* options) {
    frw_options opt{};
    opt.n_cells = 16;
    opt.hybrid = 1;
    opt.abs_tol_rel = 1e-6;
    if (options) opt = *options;
    MW_REQUIRE(opt.lattice == MW_LATTICE_VERTEX || opt.lattice == MW_LATTICE_CELL, MW_EINVAL,
               "unknown lattice %d", opt.lattice);
    if (opt.n_cells == 0) opt.n_cells = opt.lattice == MW_LATTICE_CELL ? 15 : 16;
    // the kernels tell the lattices apart by the parity of n
    if (opt.lattice == MW_LATTICE_VERTEX)
        MW_REQUIRE(opt.n_cells >= 4 && opt.n_cells <= 32 && opt.n_cells % 2 == 0, MW_EINVAL,
                   "vertex lattice: n_cells must be even in [4, 32]");
    else
        MW_REQUIRE(opt.n_cells >= 3 && opt.n_cells <= 31 && opt.n_cells % 2 == 1, MW_EINVAL,
                   "cell lattice: n_cells must be odd in [3, 31]");
    MW_REQUIRE(opt.lattice == MW_LATTICE_VERTEX || opt.expand <= 1, MW_EINVAL,
               "MicroWalk-E (expand > 1) runs on the vertex lattice only");
    if (opt.abs_tol_rel <= 0) opt.abs_tol_rel = 1e-6;
    MW_REQUIRE(opt.plain == 0 || opt.plain == 1, MW_EINVAL, "plain must be 0 or 1");
    MW_REQUIRE(opt.gauss_is == 0 || (opt.gauss_is >= 0.05 && opt.gauss_is <= 64), MW_EINVAL,
               "gauss_is must be 0 or in [0.05, 64]");
    MW_REQUIRE(opt.expand >= 0 && opt.expand <= 64, MW_EINVAL, "expand must be in [0, 64]");
    if (opt.expand > 1) {
        const int m = std::max(1, (int)std::lround(opt.n_cells / (2.0 * opt.expand)));
        MW_REQUIRE(opt.n_cells <= EXP_LIST_FACTOR * 2 * m, MW_EINVAL,
                   "expand %d with n_cells %d gives cubes %.1fx the conductor-free size; the structure index "
                   "covers %.0fx",
                   opt.expand, opt.n_cells, opt.n_cells / (2.0 * m), (double)EXP_LIST_FACTOR);
    }
    return opt;
}

// MicroWalk-E lattice factor m (expanded half-size n d / (2 m)); 0 = off.
int expand_m_of(const frw_options& opt) {
    return opt.expand > 1 ? std::max(1, (int)std::lround(opt.n_cells / (2.0 * opt.expand))) : 0;
}

void add_counters(frw_stats& st, const Counters& h) {
    st.hops += h.hops;
    st.micro_steps += h.micro_steps;
    for (int q = 0; q < 3; ++q) st.hop_class[q] += h.hop_class[q];
    for (int q = 0; q < 4; ++q) st.first_branch[q] += h.first_branch[q];
    st.env_absorbed += h.env;
    st.hop_cap += h.hop_cap;
    st.cube_halved += h.halved;
}

// One round over several extractions (server requests, or the masters of a
// matrix extraction): their shares of walks run in one set of walker
// launches, then one reduction launch and one copy of all results.  The
// per-walk buffers of a round are shared; each share's buffers start on a
// reduction block.
struct SharedRound {
    uint64_t cap = 0;
    int max_segs = 0;
    char* mem = nullptr;
    int32_t* net = nullptr;
    float* w = nullptr;
    float4* fs = nullptr;
    uint32_t* fd = nullptr;
    RedSeg* dred = nullptr;
    double* out = nullptr;
    size_t out_cap = 0;

    static size_t layout(uint64_t c, int segs, size_t* o_n, size_t* o_w, size_t* o_fs, size_t* o_fd,
                         size_t* o_sg) {
        size_t o = 0;
        auto sz = [&](size_t b) {
            size_t r = o;
            o += (b + 255) / 256 * 256;
            return r;
        };
        *o_n = sz(4 * c);
        *o_w = sz(4 * c);
        *o_fs = sz(16 * c);
        *o_fd = sz(4 * c);
        *o_sg = sz(sizeof(RedSeg) * (size_t)segs);
        return o;
    }
    static size_t bytes(uint64_t round_walks, int segs) {
        size_t a, b, c, d, e;
        return layout(round_walks + (uint64_t)segs * RED_CHUNK, segs, &a, &b, &c, &d, &e);
    }

    SharedRound(uint64_t round_walks, int segs) : cap(round_walks + (uint64_t)segs * RED_CHUNK), max_segs(segs) {
        size_t o_n, o_w, o_fs, o_fd, o_sg;
        const size_t total = layout(cap, segs, &o_n, &o_w, &o_fs, &o_fd, &o_sg);
        mem = (char*)dev_alloc(total);
        net = (int32_t*)(mem + o_n);
        w = (float*)(mem + o_w);
        fs = (float4*)(mem + o_fs);
        fd = (uint32_t*)(mem + o_fd);
        dred = (RedSeg*)(mem + o_sg);
    }
    ~SharedRound() {
        dev_free(out);
        dev_free(mem);
    }

    // Runs share[i] walks of X[i] (walk ids first_walk + X[i]->done on,
    // Philox key seeds[i]); shares of zero are skipped.  Updates done and res
    // of every extraction that ran.  Returns the run's counters.
    Counters run(Runner& R, const std::vector<Extraction*>& X, const std::vector<uint64_t>& share,
                 const std::vector<uint64_t>& seeds, uint64_t first_walk) {
        std::vector<Segment> segs;
        std::vector<RedSeg> red;
        std::vector<size_t> part;
        uint64_t offset = 0;
        int blocks = 0;
        size_t outn = 0;
        for (size_t i = 0; i < X.size(); ++i)
            if (share[i]) outn += 2 * (size_t)X[i]->K;
        if (outn > out_cap) {
            dev_free(out);
            out = nullptr;
            out = (double*)dev_alloc(sizeof(double) * outn);
            out_cap = outn;
        }
        size_t out_off = 0;
        for (size_t i = 0; i < X.size(); ++i) {
            if (!share[i]) continue;
            Extraction& E = *X[i];
            const int nblk = (int)((share[i] + RED_CHUNK - 1) / RED_CHUNK);
            MW_REQUIRE(offset + (uint64_t)nblk * RED_CHUNK <= cap && (int)segs.size() < max_segs, MW_ELIMIT,
                       "round larger than its buffers");
            Segment sg{};
            sg.S = E.dS;
            sg.G = E.G;
            sg.walk_begin = first_walk + E.done;
            sg.count = share[i];
            sg.score_net = net + offset;
            sg.score_w = w + offset;
            sg.first_state = fs + offset;
            sg.first_done = fd + offset;
            sg.k0 = (uint32_t)seeds[i];
            sg.k1 = (uint32_t)(seeds[i] >> 32);
            RedSeg rs{};
            rs.net = sg.score_net;
            rs.w = sg.score_w;
            rs.count = share[i];
            rs.K = E.K;
            rs.first_block = blocks;
            rs.partial = E.partial;
            rs.acc = E.acc;
            rs.n_total = (double)(E.done + share[i]);
            rs.out = out + out_off;
            out_off += 2 * (size_t)E.K;
            blocks += nblk;
            offset += (uint64_t)nblk * RED_CHUNK;
            segs.push_back(sg);
            red.push_back(rs);
            part.push_back(i);
        }
        if (segs.empty()) return Counters{};
        // list indices are dense; buffers start on reduction blocks
        uint64_t dense = 0;
        for (Segment& sg : segs) {
            sg.offset = dense;
            dense += sg.count;
        }
        MW_HIP(hipMemsetAsync(fd, 0, sizeof(uint32_t) * offset, 0));
        const Counters h = R.run(segs, segs.size() == 1 ? &X[part[0]]->hS : nullptr);
        MW_HIP(hipMemcpy(dred, red.data(), sizeof(RedSeg) * red.size(), hipMemcpyHostToDevice));
        reduce_multi_kernel<<<blocks, RED_THREADS>>>(dred, (int)red.size());
        finish_multi_kernel<<<(int)red.size(), 256>>>(dred);
        MW_HIP(hipGetLastError());
        std::vector<double> host(outn);
        MW_HIP(hipMemcpy(host.data(), out, sizeof(double) * outn, hipMemcpyDeviceToHost));
        size_t o2 = 0;
        for (size_t q = 0; q < part.size(); ++q) {
            Extraction& E = *X[part[q]];
            E.done += share[part[q]];
            std::copy(host.begin() + o2, host.begin() + o2 + 2 * E.K, E.res.begin());
            o2 += 2 * (size_t)E.K;
        }
        return h;
    }
};

}  // namespace

extern "C" mw_status frw_extract(mw_structure* st, int32_t master, uint64_t walk_budget, uint64_t seed,
                                 const frw_options* options, double* cap_row, double* stderr_row,
                                 frw_stats* stats, int32_t* score_net, float* score_w) {
    return guarded([&] {
        const auto t_start = std::chrono::steady_clock::now();
        MW_REQUIRE(st, MW_EINVAL, "null structure");
        MW_REQUIRE(cap_row && stderr_row, MW_EINVAL, "cap_row and stderr_row are required");
        MW_REQUIRE(master >= 0 && master < st->n_nets, MW_EINVAL, "master %d out of range", master);
        MW_REQUIRE(walk_budget >= 2, MW_EINVAL, "walk_budget must be at least 2");
        const frw_options opt = normalised_options(options);
        int dev = 0;
        MW_HIP(hipGetDevice(&dev));
        MW_REQUIRE(dev == st->device, MW_EINVAL, "structure belongs to device %d, current device is %d",
                   st->device, dev);
        const int n = opt.n_cells;
        const bool target_mode = opt.target_rel_3sigma > 0;
        // the stopping rule's checkpoints: every ck walks, a whole number of
        // 65536-walk groups of the binary64 sums; a launch walks a whole
        // number of checkpoints (or groups without a target), so the result
        // does not depend on the launch sizes
        const uint64_t group = (uint64_t)SUM_GROUP * RED_CHUNK;
        uint64_t ck = group;
        if (target_mode) {
            ck = opt.batch_walks ? opt.batch_walks : FRW_CHECKPOINT;
            ck = (ck + group - 1) / group * group;
            MW_REQUIRE(ck <= ((uint64_t)DECIDE_MAX_GROUPS * group) / 2, MW_EINVAL, "batch_walks above 2^27");
        }
        const uint64_t cap_mode = target_mode ? FRW_TARGET_LAUNCH_CAP : FRW_LAUNCH_CAP;
        const uint64_t launch_cap = std::min<uint64_t>(walk_budget, std::max<uint64_t>(ck, cap_mode / ck * ck));
        // first launch: the walks the last extraction of this structure,
        // master and rule needed, plus one checkpoint (1/64 of them when that
        // is more) for the spread between seeds; a shortfall costs one more
        // launch, never a different result
        uint64_t next = launch_cap;
        if (target_mode) {
            const uint64_t hint = st->walk_hint(master, ck, opt.target_rel_3sigma);
            next = hint ? (hint + std::max<uint64_t>(hint / 64, ck) + ck - 1) / ck * ck
                        : std::max<uint64_t>(ck, FRW_FIRST_LAUNCH / ck * ck);
        }
        const bool own_scores = !(score_net && score_w);
        // buffers kept with the structure for this master and these options
        CtxLease lease(st, master, opt, expand_m_of(opt), launch_cap, own_scores);
        ExtractCtx& ctx = *lease.c;
        Extraction& X = *ctx.X;
        Runner& R = *ctx.R;
        X.reset(R.stream);
        R.reset_stats();
        (void)frw_tuned_waves(n, R.expand_m, &R.waves_per_cu);
        frw_stats acc{};
        bool met = false;
        while (X.done < walk_budget && !met) {
            const uint64_t nb = std::min(std::min(next, launch_cap), walk_budget - X.done);
            const Segment sgm = X.segment(opt.first_walk + X.done, nb, seed, own_scores ? nullptr : score_net + X.done,
                                          own_scores ? nullptr : score_w + X.done);
            {
                std::lock_guard<std::mutex> lock(R.cache->mu);
                R.flushes = 0;
                R.ensure_uniform_table();
                add_counters(acc, ctx.run_launch(sgm, (int)(ck / RED_CHUNK), opt.target_rel_3sigma, &met));
            }
            if (!met && target_mode) {
                // the walks still needed, predicted from the estimate so far
                // (performance only: the checkpoints decide)
                const double m = X.res[X.master], se = X.res[X.K + X.master];
                double want = 0.0;
                if (m != 0.0 && se > 0.0) {
                    const double rel = 3.0 * se / std::fabs(m) / opt.target_rel_3sigma;
                    want = 1.05 * (double)X.done * rel * rel - (double)X.done;
                }
                next = want > (double)ck ? (uint64_t)std::ceil(want / (double)ck) * ck : ck;
            }
        }
        if (met) st->set_walk_hint(master, ck, opt.target_rel_3sigma, X.done);
        const int K = X.K;
        for (int j = 0; j < K; ++j) {
            cap_row[j] = X.res[j];
            stderr_row[j] = X.res[K + j];
        }
        if (stats) {
            *stats = acc;
            stats->walks = X.done;
            stats->walks_launched = X.launched;
            stats->cache_miss = R.misses;
            stats->launches = R.launches;
            stats->seconds = std::chrono::duration<double>(std::chrono::steady_clock::now() - t_start).count();
            stats->walker_seconds = R.walker_ms * 1e-3;
            stats->gauss_g = X.gauss_g;
            stats->gauss_area = X.gauss_area;
            stats->gauss_faces = X.n_faces;
        }
    });
}

// Walker launch geometry: times the walker on `walks` walks of this
// extraction at several resident-wave counts per CU and keeps the fastest for
// the lattice size and MicroWalk-E setting of the options.
extern "C" mw_status frw_autotune(mw_structure* st, int32_t master, uint64_t walks, uint64_t seed,
                                  const frw_options* options, int32_t* waves_per_cu) {
    return guarded([&] {
        MW_REQUIRE(st && waves_per_cu, MW_EINVAL, "null argument");
        MW_REQUIRE(master >= 0 && master < st->n_nets, MW_EINVAL, "master %d out of range", master);
        MW_REQUIRE(walks >= 1024, MW_EINVAL, "autotune needs at least 1024 walks");
        frw_options opt = normalised_options(options);
        const int n = opt.n_cells;
        const int em = expand_m_of(opt);
        const LaunchGeom g = launch_geom(n);
        const int most = (em > 0 ? g.blocks_e : g.blocks) / g.cus;
        std::vector<int> cand;
        for (int w : {4, 6, 8, 10, 12, 16})
            if (w < most) cand.push_back(w);
        cand.push_back(most);
        Extraction X(*st, master, opt.abs_tol_rel, walks, true);
        double best_ms = 1e30;
        int best = most;
        for (int w : cand) {
            Runner R(n, opt.hybrid, walks, 1);
            R.expand_m = em;
            R.waves_per_cu = w;
            double t = 1e30;
            for (int rep = 0; rep < 3; ++rep) {
                // the first pass also builds the tables the walks need
                const Segment sgm = X.segment(opt.first_walk, walks, seed, nullptr, nullptr);
                const double before = R.walker_ms;
                (void)R.run({sgm}, &X.hS);
                if (rep > 0) t = std::min(t, R.walker_ms - before);
            }
            if (t < best_ms) {
                best_ms = t;
                best = w;
            }
        }
        frw_store_waves(n, em, best);
        *waves_per_cu = best;
    });
}

// Capacitance matrix: Alg. 1 for several masters in shared rounds.
extern "C" mw_status frw_extract_matrix(mw_structure* st, int32_t n_masters, const int32_t* masters,
                                        uint64_t walks_per_master, uint64_t seed, const frw_options* options,
                                        double* cap, double* stderr_out, double* cap_sym, frw_stats* stats) {
    return guarded([&] {
        const auto t_start = std::chrono::steady_clock::now();
        MW_REQUIRE(st, MW_EINVAL, "null structure");
        MW_REQUIRE(n_masters >= 1 && masters, MW_EINVAL, "at least one master is required");
        MW_REQUIRE(cap && stderr_out, MW_EINVAL, "cap and stderr are required");
        MW_REQUIRE(walks_per_master >= 2, MW_EINVAL, "walks_per_master must be at least 2");
        for (int i = 0; i < n_masters; ++i) {
            MW_REQUIRE(masters[i] >= 0 && masters[i] < st->n_nets, MW_EINVAL, "master %d out of range", masters[i]);
            for (int j = 0; j < i; ++j) MW_REQUIRE(masters[j] != masters[i], MW_EINVAL, "master %d listed twice", masters[i]);
        }
        const frw_options opt = normalised_options(options);
        int dev = 0;
        MW_HIP(hipGetDevice(&dev));
        MW_REQUIRE(dev == st->device, MW_EINVAL, "structure belongs to device %d, current device is %d",
                   st->device, dev);
        const int n = opt.n_cells;
        const LaunchGeom g = launch_geom(n);
        // one round holds up to round_walks walks over all active masters
        const uint64_t round_walks = std::max<uint64_t>(8 * g.pool, 1 << 22);
        const uint64_t per_round = opt.target_rel_3sigma > 0 && opt.batch_walks ? opt.batch_walks : walks_per_master;
        std::vector<std::unique_ptr<Extraction>> own;
        std::vector<Extraction*> X;
        std::vector<uint64_t> seeds;
        for (int i = 0; i < n_masters; ++i) {
            own.push_back(std::make_unique<Extraction>(*st, masters[i], opt.abs_tol_rel, round_walks, false, false));
            X.push_back(own.back().get());
            seeds.push_back(seed + (uint64_t)i);  // master i: Philox key seed + i
        }
        Runner R(n, opt.hybrid, round_walks, n_masters);
        R.expand_m = expand_m_of(opt);
        R.plain = opt.plain;
        (void)frw_tuned_waves(n, R.expand_m, &R.waves_per_cu);
        if (opt.gauss_is > 0)
            for (Extraction* x : X) x->importance(R, opt.gauss_is * x->gauss_g);
        SharedRound round(round_walks, n_masters);
        frw_stats acc{};
        std::vector<bool> active(n_masters, true);
        for (;;) {
            // shares: each active master's next batch, as many masters as fit
            std::vector<uint64_t> sh(n_masters, 0);
            uint64_t used = 0;
            bool any = false;
            for (int i = 0; i < n_masters; ++i) {
                if (!active[i]) continue;
                any = true;
                const uint64_t want = std::min<uint64_t>(per_round, walks_per_master - X[i]->done);
                const uint64_t padded = (want + RED_CHUNK - 1) / RED_CHUNK * RED_CHUNK;
                if (used > 0 && used + padded > round_walks) continue;  // next round
                sh[i] = std::min<uint64_t>(want, round_walks);
                used += (sh[i] + RED_CHUNK - 1) / RED_CHUNK * RED_CHUNK;
            }
            if (!any) break;
            add_counters(acc, round.run(R, X, sh, seeds, opt.first_walk));
            for (int i = 0; i < n_masters; ++i)
                if (active[i] && (X[i]->done >= walks_per_master || (sh[i] && X[i]->converged(opt.target_rel_3sigma))))
                    active[i] = false;
        }
        const int K = X[0]->K;
        for (int i = 0; i < n_masters; ++i)
            for (int j = 0; j < K; ++j) {
                cap[(size_t)i * K + j] = X[i]->res[j];
                stderr_out[(size_t)i * K + j] = X[i]->res[K + j];
            }
        if (cap_sym) {
            // symmetrised block over the listed masters: mean of C_ab and C_ba
            for (int a = 0; a < n_masters; ++a)
                for (int b = 0; b < n_masters; ++b)
                    cap_sym[(size_t)a * n_masters + b] =
                        a == b ? X[a]->res[masters[a]] : 0.5 * (X[a]->res[masters[b]] + X[b]->res[masters[a]]);
        }
        if (stats) {
            *stats = acc;
            stats->walks = 0;
            for (auto* e : X) stats->walks += e->done;
            stats->walks_launched = stats->walks;
            stats->cache_miss = R.misses;
            stats->launches = R.launches;
            stats->seconds = std::chrono::duration<double>(std::chrono::steady_clock::now() - t_start).count();
            stats->walker_seconds = R.walker_ms * 1e-3;
        }
    });
}

// -------------------------------------------------------------------------
// Serving: continuous batching of extraction requests on one device.
// -------------------------------------------------------------------------
#include <condition_variable>
#include <deque>
#include <thread>

namespace {

struct ServerRequest {
    uint64_t ticket = 0;
    // copied description
    std::vector<mw_cond_box> cond;
    std::vector<mw_diel_box> diel;
    std::vector<float> z0, eps;
    mw_structure_desc desc{};
    int32_t master = 0;
    uint64_t budget = 0, seed = 0;
    size_t footprint = 0;
    // device state (worker thread only)
    mw_structure* st = nullptr;
    std::unique_ptr<Extraction> X;
    uint64_t chunk = 0;
    frw_stats stats{};
    // result
    enum State { QUEUED, RUNNING, DONE, FAILED } state = QUEUED;
    mw_status code = MW_OK;
    std::string message;
    std::vector<double> row, se;
    std::chrono::steady_clock::time_point t_submit, t_done;

    void release() {
        X.reset();
        if (st) {
            mw_structure_destroy(st);
            st = nullptr;
        }
    }
};

}  // namespace

constexpr uint64_t MIN_SHARE = 4096;  // walks per request and round, at least

struct mw_server {
    int device = 0;
    size_t budget = 0;
    frw_options opt{};
    size_t max_queue = 100000;
    int max_slots = 256;
    int max_ready = 8;  // requests prepared ahead of the rounds
    uint64_t round_walks = 0;
    std::mutex mu;
    std::condition_variable cv;
    bool stop = false;
    std::deque<std::shared_ptr<ServerRequest>> queue;  // submitted, not yet on the device
    std::deque<std::shared_ptr<ServerRequest>> ready;  // structure and buffers on the device
    std::map<uint64_t, std::shared_ptr<ServerRequest>> tickets;
    uint64_t next_ticket = 1;
    mw_server_stats st{};
    std::thread worker, preparer;
    bool preparing = false;  // the preparation thread holds a request

    void fail(const std::shared_ptr<ServerRequest>& r, mw_status code, const std::string& msg) {
        r->state = ServerRequest::FAILED;
        r->code = code;
        r->message = msg;
        r->t_done = std::chrono::steady_clock::now();
        st.failed++;
    }

    std::unique_ptr<SharedRound> round;  // buffers of one round (first round on)

    // Walk shares of one round (capacity round_walks): the longest-admitted
    // request gets up to three quarters, the rest goes to the requests with
    // the fewest remaining walks first, and capacity they leave goes back to
    // the longest-admitted one (which alone gets the whole round).
    std::vector<uint64_t> shares(const std::vector<std::shared_ptr<ServerRequest>>& running) const {
        const size_t m = running.size();
        std::vector<uint64_t> sh(m, 0), rem(m);
        for (size_t i = 0; i < m; ++i) rem[i] = running[i]->budget - running[i]->X->done;
        uint64_t used = std::min<uint64_t>(rem[0], round_walks / 4 * 3);
        sh[0] = used;
        std::vector<size_t> order(m);
        for (size_t i = 0; i < m; ++i) order[i] = i;
        std::stable_sort(order.begin(), order.end(), [&](size_t a, size_t b) { return rem[a] < rem[b]; });
        for (size_t i : order) {
            if (used >= round_walks) break;
            if (i == 0) continue;
            const uint64_t take = std::min<uint64_t>(rem[i] - sh[i], round_walks - used);
            sh[i] += take;
            used += take;
        }
        sh[0] += std::min<uint64_t>(rem[0] - sh[0], round_walks - used);
        return sh;
    }

    // Preparation thread: in arrival order, while the memory budget allows,
    // copies each request's structure to the device and builds its grid
    // index and extraction buffers (on a non-blocking stream, overlapping
    // the rounds), then hands it to the round worker.
    void prepare_loop() {
        (void)hipSetDevice(device);
        for (;;) {
            std::shared_ptr<ServerRequest> r;
            {
                std::unique_lock<std::mutex> lk(mu);
                for (;;) {
                    if (stop) {
                        for (auto& q : queue) fail(q, MW_EBUSY, "server destroyed before the request ran");
                        queue.clear();
                        cv.notify_all();
                        return;
                    }
                    if (!queue.empty()) {
                        auto& f = queue.front();
                        if (f->footprint > budget) {
                            fail(f, MW_ELIMIT, "request footprint exceeds the server's memory budget");
                            queue.pop_front();
                            cv.notify_all();
                            continue;
                        }
                        if ((int)ready.size() < max_ready && st.resident_bytes + f->footprint <= budget) break;
                    }
                    cv.wait(lk);
                }
                r = queue.front();
                queue.pop_front();
                preparing = true;
                st.resident_bytes += r->footprint;
                st.max_resident_bytes = std::max(st.max_resident_bytes, st.resident_bytes);
            }
            mw_status rc = mw_structure_create(&r->desc, &r->st);
            std::string msg = rc ? mw_last_error() : "";
            if (rc == MW_OK) {
                rc = guarded([&] {
                    r->X = std::make_unique<Extraction>(*r->st, r->master, opt.abs_tol_rel, round_walks, false,
                                                        false);
                });
                if (rc) msg = mw_last_error();
            }
            std::lock_guard<std::mutex> lk(mu);
            preparing = false;
            if (rc != MW_OK) {
                r->release();
                st.resident_bytes -= r->footprint;
                fail(r, rc, msg);
                cv.notify_all();
                continue;
            }
            // reconcile the reservation with the memory actually held; a
            // request that no longer fits waits at the queue's head
            const size_t actual = r->st->bytes + Extraction::bytes(r->X->K, round_walks, false, r->X->n_faces);
            if (actual > r->footprint && st.resident_bytes - r->footprint + actual > budget) {
                r->release();
                st.resident_bytes -= r->footprint;
                r->footprint = actual;
                if (actual > budget)
                    fail(r, MW_ELIMIT, "request footprint exceeds the server's memory budget");
                else
                    queue.push_front(r);
                cv.notify_all();
                continue;
            }
            st.resident_bytes += actual - r->footprint;
            r->footprint = actual;
            st.max_resident_bytes = std::max(st.max_resident_bytes, st.resident_bytes);
            ready.push_back(r);
            cv.notify_all();
        }
    }

    void loop() {
        (void)hipSetDevice(device);
        std::unique_ptr<Runner> R;
        std::vector<std::shared_ptr<ServerRequest>> running;
        for (;;) {
            {
                std::unique_lock<std::mutex> lk(mu);
                // an idle device waits for the request being prepared, so
                // that requests submitted together share their first round
                while (!stop && running.empty() && (ready.empty() || (preparing && (int)ready.size() < max_ready)))
                    cv.wait(lk);
                if (stop && running.empty()) {
                    // prepared requests that never ran give their memory back
                    for (auto& r : ready) {
                        r->release();
                        st.resident_bytes -= r->footprint;
                        fail(r, MW_EBUSY, "server destroyed before the request ran");
                    }
                    ready.clear();
                    cv.notify_all();
                    return;
                }
                // continuous admission: every prepared request joins the next round
                while (!stop && !ready.empty() && (int)running.size() < max_slots) {
                    auto r = ready.front();
                    ready.pop_front();
                    r->state = ServerRequest::RUNNING;
                    running.push_back(r);
                }
                cv.notify_all();
            }
            if (running.empty()) continue;
            // one round over the shares of the running requests
            const std::vector<uint64_t> sh = shares(running);
            uint64_t walks = 0;
            size_t n_run = 0;
            std::vector<Extraction*> X;
            std::vector<uint64_t> seeds;
            for (size_t i = 0; i < running.size(); ++i) {
                X.push_back(running[i]->X.get());
                seeds.push_back(running[i]->seed);
                walks += sh[i];
                n_run += sh[i] ? 1 : 0;
            }
            mw_status rc = guarded([&] {
                if (!round) round = std::make_unique<SharedRound>(round_walks, max_slots);
                if (!R) {
                    R = std::make_unique<Runner>(opt.n_cells, opt.hybrid, round_walks, max_slots);
                    R->expand_m = expand_m_of(opt);
                    R->plain = opt.plain;
                    (void)frw_tuned_waves(opt.n_cells, R->expand_m, &R->waves_per_cu);
                }
                if (opt.gauss_is > 0)
                    for (auto& r : running)
                        if (!r->X->n_patches) r->X->importance(*R, opt.gauss_is * r->X->gauss_g);
                (void)round->run(*R, X, sh, seeds, opt.first_walk);
                for (auto& r : running) {
                    r->stats.walks = r->X->done;
                    r->stats.walks_launched = r->X->done;
                    r->stats.gauss_g = r->X->gauss_g;
                    r->stats.gauss_area = r->X->gauss_area;
                    r->stats.gauss_faces = r->X->n_faces;
                }
            });
            std::string msg = rc ? mw_last_error() : "";
            std::vector<std::shared_ptr<ServerRequest>> still, finished;
            {
                std::lock_guard<std::mutex> lk(mu);
                st.rounds++;
                st.walks += walks;
                st.max_concurrent = std::max<uint64_t>(st.max_concurrent, n_run);
                for (size_t i = 0; i < running.size(); ++i) {
                    auto& r = running[i];
                    if (rc != MW_OK) {
                        fail(r, rc, msg);
                    } else if (r->X->done >= r->budget || (sh[i] && r->X->converged(opt.target_rel_3sigma))) {
                        const int K = r->X->K;
                        r->row.assign(r->X->res.begin(), r->X->res.begin() + K);
                        r->se.assign(r->X->res.begin() + K, r->X->res.end());
                        r->state = ServerRequest::DONE;
                        r->t_done = std::chrono::steady_clock::now();
                        st.completed++;
                    } else {
                        still.push_back(r);
                        continue;
                    }
                    finished.push_back(r);
                }
                cv.notify_all();
            }
            // device memory of finished requests is freed outside the lock
            for (auto& r : finished) r->release();
            {
                std::lock_guard<std::mutex> lk(mu);
                for (auto& r : finished) st.resident_bytes -= r->footprint;
                cv.notify_all();
            }
            running.swap(still);
        }
    }
};

extern "C" mw_status mw_server_create(size_t hbm_budget_bytes, const frw_options* options, mw_server** out) {
    return guarded([&] {
        MW_REQUIRE(out, MW_EINVAL, "null output handle");
        MW_REQUIRE(hbm_budget_bytes > 0, MW_EINVAL, "zero memory budget");
        auto s = std::make_unique<mw_server>();
        MW_HIP(hipGetDevice(&s->device));
        s->budget = hbm_budget_bytes;
        s->opt = normalised_options(options);
        const LaunchGeom g = launch_geom(s->opt.n_cells);
        s->round_walks = std::max<uint64_t>(32 * g.pool, 1 << 23);
        mw_server* raw = s.get();
        s->worker = std::thread([raw] { raw->loop(); });
        s->preparer = std::thread([raw] { raw->prepare_loop(); });
        *out = s.release();
    });
}

extern "C" mw_status mw_server_submit(mw_server* srv, const mw_structure_desc* D, int32_t master,
                                      uint64_t walk_budget, uint64_t seed, uint64_t* ticket) {
    return guarded([&] {
        MW_REQUIRE(srv && ticket, MW_EINVAL, "null argument");
        validate_desc(D);
        MW_REQUIRE(master >= 0 && master < D->n_nets, MW_EINVAL, "master %d out of range", master);
        MW_REQUIRE(walk_budget >= 2, MW_EINVAL, "walk_budget must be at least 2");
        auto r = std::make_shared<ServerRequest>();
        r->cond.assign(D->cond, D->cond + D->n_cond);
        r->diel.assign(D->diel, D->diel + D->n_diel);
        r->z0.assign(D->layer_z0, D->layer_z0 + D->n_layers);
        r->eps.assign(D->layer_eps, D->layer_eps + D->n_layers);
        r->desc = *D;
        r->desc.cond = r->cond.data();
        r->desc.diel = r->diel.empty() ? nullptr : r->diel.data();
        r->desc.layer_z0 = r->z0.data();
        r->desc.layer_eps = r->eps.data();
        r->master = master;
        r->budget = walk_budget;
        r->seed = seed;
        // footprint estimate: structure and grid index (the grid-size rule of
        // mw_structure_create; candidate lists guessed at a few boxes per
        // cell) plus the per-round extraction buffers.  Admission corrects it
        // to the memory actually held once the structure exists.
        const size_t boxes = (size_t)D->n_cond + D->n_diel;
        const size_t cells = (size_t)std::min(1048576.0, std::max(512.0, 256.0 * boxes)) * 2;  // rounding slack
        r->footprint = boxes * 64 + cells * 32 + cells * 36 * std::min<size_t>(boxes, 32) +
                       Extraction::bytes(D->n_nets + 1, srv->round_walks, false) + 64 * 1024;
        r->t_submit = std::chrono::steady_clock::now();
        std::lock_guard<std::mutex> lk(srv->mu);
        MW_REQUIRE(!srv->stop, MW_EINVAL, "server is shutting down");
        MW_REQUIRE(srv->queue.size() < srv->max_queue, MW_EBUSY, "server queue full");
        r->ticket = srv->next_ticket++;
        srv->tickets[r->ticket] = r;
        srv->queue.push_back(r);
        srv->st.submitted++;
        *ticket = r->ticket;
        srv->cv.notify_all();
    });
}

extern "C" mw_status mw_server_poll(mw_server* srv, uint64_t ticket, double* cap_row, double* stderr_row,
                                    frw_stats* stats, double* latency_s) {
    mw_status code = MW_OK;
    const mw_status rc = guarded([&] {
        MW_REQUIRE(srv, MW_EINVAL, "null server");
        std::lock_guard<std::mutex> lk(srv->mu);
        auto it = srv->tickets.find(ticket);
        MW_REQUIRE(it != srv->tickets.end(), MW_EINVAL, "unknown ticket %llu", (unsigned long long)ticket);
        auto& r = it->second;
        if (r->state == ServerRequest::QUEUED || r->state == ServerRequest::RUNNING) {
            code = MW_ENOTREADY;
            return;
        }
        if (r->state == ServerRequest::FAILED) {
            set_error("%s", r->message.c_str());
            code = r->code;
            return;
        }
        MW_REQUIRE(cap_row && stderr_row, MW_EINVAL, "cap_row and stderr_row are required");
        for (size_t j = 0; j < r->row.size(); ++j) {
            cap_row[j] = r->row[j];
            stderr_row[j] = r->se[j];
        }
        if (stats) *stats = r->stats;
        if (latency_s) *latency_s = std::chrono::duration<double>(r->t_done - r->t_submit).count();
    });
    return rc != MW_OK ? rc : code;
}

extern "C" mw_status mw_server_get_stats(mw_server* srv, mw_server_stats* out) {
    return guarded([&] {
        MW_REQUIRE(srv && out, MW_EINVAL, "null argument");
        std::lock_guard<std::mutex> lk(srv->mu);
        *out = srv->st;
    });
}

extern "C" mw_status mw_server_destroy(mw_server* srv) {
    return guarded([&] {
        if (!srv) return;
        {
            std::lock_guard<std::mutex> lk(srv->mu);
            srv->stop = true;
        }
        srv->cv.notify_all();
        if (srv->preparer.joinable()) srv->preparer.join();
        if (srv->worker.joinable()) srv->worker.join();
        delete srv;
    });
}
