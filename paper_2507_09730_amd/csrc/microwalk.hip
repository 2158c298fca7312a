// microwalk.hip — Alg. 3 (MicroWalk) on explicit voxelised transition cubes:
// mw_transition (one cube) and mw_transition_batch (many cubes of uneven
// size in one persistent launch).
//
// Per cube a prep kernel turns the eps grid into one of three tables; the
// walk kernel stages it in LDS and runs walks lane-parallel.  Every step is
// integer work: one Philox word, five compares against the node's
// thresholds (or against prefix sums with mulhi(u, S5), which selects the
// same direction), one index update and one LDS load.  Walks are refilled
// wave-wide (ballot + one LDS atomic) at group boundaries, so each walk's
// Philox words are word-aligned (group g uses counter c0 = g).
//
// Tile forms (all use a padded node grid so that reaching the cube boundary
// is detected by a sentinel in the loaded data, not by coordinate tests):
//   1 thresholds in LDS: T4[P^3] then T0..T3[P^3] as uint4; boundary nodes
//     have T4 = 0 (an interior node always has T4 >= 1).
//   2 cell codes in LDS (vertex lattice, large n): (n+2)^3 codes with a
//     border of sentinel cells 2^29; the six link codes of a node are sums of
//     its eight surrounding cells, recomputed per step.
//   3 thresholds as form 1, read from global memory (cubes too large for
//     LDS).
#include <algorithm>
#include <cmath>
#include <map>
#include <memory>
#include <mutex>
#include <vector>

#include "common.h"

namespace mw {
namespace {

constexpr int FORM_TLDS = 1, FORM_CODES = 2, FORM_TGLOBAL = 3;
constexpr uint32_t SENTINEL_CELL = 1u << 29;
constexpr uint32_t LDS_TABLE_WORDS = 40704;  // 159 KiB of the 160 KiB LDS

struct CubeDev {
    const float* eps;
    uint32_t* table;
    int32_t* hits;
    int32_t* steps;
    uint64_t walk0;
    uint64_t n_walks;
    int32_t n, lattice, form, P;
    uint32_t table_words;  // multiple of 4
    uint32_t t4_words;     // forms 1/3: words before the uint4 block
    uint32_t c1;
    int32_t start;
};

struct Item {
    int32_t cube;
    int32_t pad;
    uint64_t w_begin, w_end;
};

// -------------------------------------------------------------------------
// Table preparation.
// -------------------------------------------------------------------------
__device__ __forceinline__ uint32_t vcode(const float* eps, int n, int i, int j, int k) {
    return (uint32_t)rintf(eps[((size_t)k * n + j) * n + i] * 65536.0f);
}

// Five thresholds from six link codes.
__device__ __forceinline__ void thresholds6(const uint32_t g[6], uint32_t T[5]) {
    uint64_t S = 0, S5 = 0;
#pragma unroll
    for (int d = 0; d < 6; ++d) S5 += g[d];
#pragma unroll
    for (int k = 0; k < 5; ++k) {
        S += g[k];
        T[k] = ceil_threshold(S, S5);
    }
}

__global__ void prep_kernel(const CubeDev* __restrict__ cubes, int* bad) {
    const CubeDev C = cubes[blockIdx.y];
    const int P = C.P, n = C.n;
    const uint32_t nodes = (uint32_t)P * P * P;
    const uint32_t cells = (uint32_t)n * n * n;
    for (uint32_t v = blockIdx.x * blockDim.x + threadIdx.x; v < cells; v += gridDim.x * blockDim.x) {
        const float e = C.eps[v];
        if (!(e >= 1e-3f && e <= 1e3f)) atomicOr(bad, 1);
    }
    for (uint32_t v = blockIdx.x * blockDim.x + threadIdx.x; v < nodes; v += gridDim.x * blockDim.x) {
        const int i = v % P, j = (v / P) % P, k = v / (P * P);
        if (C.form == FORM_CODES) {
            // padded cell (i,j,k) = real cell (i-1, j-1, k-1)
            const bool real = i >= 1 && i <= n && j >= 1 && j <= n && k >= 1 && k <= n;
            C.table[v] = real ? vcode(C.eps, n, i - 1, j - 1, k - 1) : SENTINEL_CELL;
            continue;
        }
        uint32_t T[5] = {0, 0, 0, 0, 0};
        if (C.lattice == MW_LATTICE_VERTEX) {
            if (i >= 1 && i < n && j >= 1 && j < n && k >= 1 && k < n) {
                uint32_t c[2][2][2];
#pragma unroll
                for (int dz = 0; dz < 2; ++dz)
#pragma unroll
                    for (int dy = 0; dy < 2; ++dy)
#pragma unroll
                        for (int dx = 0; dx < 2; ++dx) c[dz][dy][dx] = vcode(C.eps, n, i - 1 + dx, j - 1 + dy, k - 1 + dz);
                uint32_t g[6];
                g[0] = c[0][0][0] + c[0][1][0] + c[1][0][0] + c[1][1][0];
                g[1] = c[0][0][1] + c[0][1][1] + c[1][0][1] + c[1][1][1];
                g[2] = c[0][0][0] + c[0][0][1] + c[1][0][0] + c[1][0][1];
                g[3] = c[0][1][0] + c[0][1][1] + c[1][1][0] + c[1][1][1];
                g[4] = c[0][0][0] + c[0][0][1] + c[0][1][0] + c[0][1][1];
                g[5] = c[1][0][0] + c[1][0][1] + c[1][1][0] + c[1][1][1];
                thresholds6(g, T);
            }
        } else {
            // cell lattice: padded index (x+1) for node coordinate x in [-1, N]
            const int x = i - 1, y = j - 1, z = k - 1;
            if (x >= 0 && x < n && y >= 0 && y < n && z >= 0 && z < n) {
                const double ev = (double)C.eps[((size_t)z * n + y) * n + x];
                const int q[6][3] = {{x - 1, y, z}, {x + 1, y, z}, {x, y - 1, z},
                                     {x, y + 1, z}, {x, y, z - 1}, {x, y, z + 1}};
                uint32_t g[6];
#pragma unroll
                for (int d = 0; d < 6; ++d) {
                    const int a = q[d][0], b = q[d][1], cc = q[d][2];
                    if (a >= 0 && a < n && b >= 0 && b < n && cc >= 0 && cc < n) {
                        const double ei = (double)C.eps[((size_t)cc * n + b) * n + a];
                        g[d] = (uint32_t)rint(ei / (ei + ev) * 16777216.0);
                    } else {
                        g[d] = 1u << 24;
                    }
                }
                thresholds6(g, T);
            }
        }
        C.table[v] = T[4];
        uint4* q4 = reinterpret_cast<uint4*>(C.table + C.t4_words);
        q4[v] = make_uint4(T[0], T[1], T[2], T[3]);
    }
}

// -------------------------------------------------------------------------
// Boundary hit index of the final (padded) node.
// -------------------------------------------------------------------------
__device__ __forceinline__ int32_t hit_index(const CubeDev& C, int node) {
    const int P = C.P;
    int c[3] = {node % P, (node / P) % P, node / (P * P)};
    if (C.lattice == MW_LATTICE_VERTEX) {
        const int n = C.n, M = n - 1;
#pragma unroll
        for (int ax = 0; ax < 3; ++ax) {
            if (c[ax] == 0 || c[ax] == n) {
                const int side = c[ax] == n;
                const int a = ax == 0 ? c[1] : c[0];
                const int b = ax == 2 ? c[1] : c[2];
                return (2 * ax + side) * M * M + (b - 1) * M + (a - 1);
            }
        }
        return -1;
    }
    const int N = C.n;
#pragma unroll
    for (int ax = 0; ax < 3; ++ax) c[ax] -= 1;
#pragma unroll
    for (int ax = 0; ax < 3; ++ax) {
        if (c[ax] < 0 || c[ax] >= N) {
            const int side = c[ax] >= N;
            const int a = ax == 0 ? c[1] : c[0];
            const int b = ax == 2 ? c[1] : c[2];
            return (2 * ax + side) * N * N + b * N + a;
        }
    }
    return -1;
}

constexpr uint32_t STEP_CAP = 1u << 30;

// Node data cached in registers between steps.
struct NodeT {
    uint32_t t0, t1, t2, t3, t4;
};

template <int FORM>
__device__ __forceinline__ NodeT load_t(const uint32_t* base, uint32_t t4_words, int node) {
    NodeT r;
    guvec4 q;
    if (FORM == FORM_TGLOBAL) {
        r.t4 = gp(base)[node];
        q = ((const GAS guvec4*)(base + t4_words))[node];
    } else {
        r.t4 = base[node];
        q = reinterpret_cast<const guvec4*>(base + t4_words)[node];
    }
    r.t0 = q.x;
    r.t1 = q.y;
    r.t2 = q.z;
    r.t3 = q.w;
    return r;
}

// Form 2: prefix sums S0..S4 and S5 of the node's links from its 8 cells;
// returns false at a boundary node (a sentinel cell among the eight).
struct NodeS {
    uint32_t s0, s1, s2, s3, s4, s5;
};

__device__ __forceinline__ bool load_s(const uint32_t* lds, int P, int node, NodeS& r) {
    const uint32_t* b0 = lds + node;
    const uint32_t* b1 = b0 + P * P;
    const uint32_t c000 = b0[0], c001 = b0[1], c010 = b0[P], c011 = b0[P + 1];
    const uint32_t c100 = b1[0], c101 = b1[1], c110 = b1[P], c111 = b1[P + 1];
    // c[dz][dy][dx] named c<dz><dy><dx>
    const uint32_t a0 = c000 + c100, a1 = c010 + c110;  // dx = 0, dy = 0/1, summed over dz
    const uint32_t b0s = c001 + c101, b1s = c011 + c111;  // dx = 1
    const uint32_t gmx = a0 + a1, gpx = b0s + b1s;
    const uint32_t total = gmx + gpx;
    const uint32_t gmy = a0 + b0s;
    const uint32_t gmz = c000 + c001 + c010 + c011;
    r.s0 = gmx;
    r.s1 = total;
    r.s2 = total + gmy;
    r.s3 = total + total;
    r.s4 = r.s3 + gmz;
    r.s5 = r.s3 + total;
    return total < SENTINEL_CELL;
}

__device__ __forceinline__ int select_delta(uint32_t u, uint32_t t0, uint32_t t1, uint32_t t2, uint32_t t3,
                                            uint32_t t4, int P, int P2) {
    int delta = -1;
    delta = u >= t0 ? 1 : delta;
    delta = u >= t1 ? -P : delta;
    delta = u >= t2 ? P : delta;
    delta = u >= t3 ? -P2 : delta;
    delta = u >= t4 ? P2 : delta;
    return delta;
}

// Walks of one work item [wb, we) of cube C, WPL interleaved walks per lane:
// each lane holds WPL walk slots and steps every live one per Philox block,
// so the slots' dependent chains (table load, compare, move) overlap.  Free
// slots are refilled wave-wide every groups_per_refill blocks; a walk's
// result depends only on its index, not on the lane or slot that runs it.
template <int FORM, int WPL>
__device__ void run_item(const CubeDev& C, const uint32_t* tab, uint64_t wb, uint64_t we, uint32_t* s_next,
                         uint32_t k0, uint32_t k1, int groups_per_refill, unsigned long long& my_steps) {
    const int lane = threadIdx.x & 63;
    const int P = C.P, P2 = C.P * C.P;
    const uint64_t cnt = we - wb;
    bool active[WPL];
    int node[WPL];
    uint32_t s[WPL];
    uint64_t rel[WPL];
    NodeT T[WPL];
    NodeS S[WPL];
#pragma unroll
    for (int w = 0; w < WPL; ++w) {
        active[w] = false;
        node[w] = 0;
        s[w] = 0;
        rel[w] = 0;
        T[w] = NodeT{};
        S[w] = NodeS{};
    }
    for (;;) {
        bool any = false;
#pragma unroll
        for (int w = 0; w < WPL; ++w) {
            const bool want = !active[w];
            const uint64_t bal = __ballot(want);
            if (bal) {
                const int leader = __ffsll((unsigned long long)bal) - 1;
                uint32_t base = 0;
                if (lane == leader) base = atomicAdd(s_next, (uint32_t)__popcll(bal));
                base = __shfl(base, leader);
                const uint32_t rank = __popcll(bal & ((1ull << lane) - 1ull));
                if (want && (uint64_t)base + rank < cnt) {
                    active[w] = true;
                    rel[w] = wb + base + rank;
                    s[w] = 0;
                    node[w] = C.start;
                    if (FORM == FORM_CODES)
                        load_s(tab, P, node[w], S[w]);
                    else
                        T[w] = load_t<FORM>(tab, C.t4_words, node[w]);
                }
            }
            any |= active[w];
        }
        if (!__any(any)) break;
        for (int g = 0; g < groups_per_refill; ++g) {
#pragma unroll
            for (int w = 0; w < WPL; ++w) {
                if (active[w]) {
                    const uint64_t walk = C.walk0 + rel[w];
                    const Rand4 r = philox10(s[w] >> 2, C.c1, (uint32_t)walk, ctr_hi(walk, PURPOSE_MICROWALK), k0, k1);
                    const uint32_t us[4] = {r.x, r.y, r.z, r.w};
                    bool alive = true;
#pragma unroll
                    for (int q = 0; q < 4; ++q) {
                        if (alive) {
                            int delta;
                            if (FORM == FORM_CODES) {
                                const uint32_t x = __umulhi(us[q], S[w].s5);
                                delta = select_delta(x, S[w].s0, S[w].s1, S[w].s2, S[w].s3, S[w].s4, P, P2);
                            } else {
                                delta = select_delta(us[q], T[w].t0, T[w].t1, T[w].t2, T[w].t3, T[w].t4, P, P2);
                            }
                            node[w] += delta;
                            ++s[w];
                            if (FORM == FORM_CODES) {
                                alive = load_s(tab, P, node[w], S[w]);
                            } else {
                                T[w] = load_t<FORM>(tab, C.t4_words, node[w]);
                                alive = T[w].t4 != 0;
                            }
                        }
                    }
                    if (!alive || s[w] >= STEP_CAP) {
                        gpw(C.hits)[rel[w]] = alive ? -1 : hit_index(C, node[w]);
                        if (C.steps) gpw(C.steps)[rel[w]] = (int32_t)s[w];
                        my_steps += s[w];
                        active[w] = false;
                    }
                }
            }
        }
    }
}

template <int FORM>
__device__ __forceinline__ void run_item_wpl(int wpl, const CubeDev& C, const uint32_t* tab, uint64_t wb,
                                             uint64_t we, uint32_t* s_next, uint32_t k0, uint32_t k1,
                                             int groups_per_refill, unsigned long long& my_steps) {
    if (wpl >= 4)
        run_item<FORM, 4>(C, tab, wb, we, s_next, k0, k1, groups_per_refill, my_steps);
    else if (wpl == 2)
        run_item<FORM, 2>(C, tab, wb, we, s_next, k0, k1, groups_per_refill, my_steps);
    else
        run_item<FORM, 1>(C, tab, wb, we, s_next, k0, k1, groups_per_refill, my_steps);
}

__global__ void __launch_bounds__(1024) walk_kernel(const CubeDev* __restrict__ cubes, const Item* __restrict__ items,
                                                    int32_t n_items, uint64_t item_walks, int32_t* item_counter,
                                                    const unsigned long long* __restrict__ seed_dev,
                                                    int32_t groups_per_refill, unsigned long long* step_total,
                                                    int32_t wpl) {
    extern __shared__ __attribute__((aligned(16))) uint32_t lds[];
    const unsigned long long seed = *seed_dev;
    const uint32_t k0 = (uint32_t)seed, k1 = (uint32_t)(seed >> 32);
    __shared__ int32_t s_item;
    __shared__ uint32_t s_next;
    int cur_cube = -1;
    unsigned long long my_steps = 0;
    for (;;) {
        if (threadIdx.x == 0) {
            s_item = atomicAdd(item_counter, 1);
            s_next = 0;
        }
        __syncthreads();
        const int it = s_item;
        if (it >= n_items) break;
        Item I;
        if (items) {
            I = items[it];
        } else {
            I.cube = 0;
            I.w_begin = (uint64_t)it * item_walks;
            const uint64_t e = I.w_begin + item_walks, nw = cubes[0].n_walks;
            I.w_end = e < nw ? e : nw;
        }
        const CubeDev C = cubes[I.cube];
        if (C.form != FORM_TGLOBAL && I.cube != cur_cube) {
            const GAS guvec4* src = (const GAS guvec4*)C.table;
            guvec4* dst = reinterpret_cast<guvec4*>(lds);
            for (uint32_t q = threadIdx.x; q < C.table_words / 4; q += blockDim.x) dst[q] = src[q];
            cur_cube = I.cube;
            __syncthreads();
        }
        // separate call sites keep the LDS table in the LDS address space
        if (C.form == FORM_CODES)
            run_item_wpl<FORM_CODES>(wpl, C, lds, I.w_begin, I.w_end, &s_next, k0, k1, groups_per_refill, my_steps);
        else if (C.form == FORM_TLDS)
            run_item_wpl<FORM_TLDS>(wpl, C, lds, I.w_begin, I.w_end, &s_next, k0, k1, groups_per_refill, my_steps);
        else
            run_item_wpl<FORM_TGLOBAL>(wpl, C, C.table, I.w_begin, I.w_end, &s_next, k0, k1, groups_per_refill,
                                       my_steps);
        __syncthreads();
    }
    // device-counted micro-steps
    for (int off = 32; off > 0; off >>= 1) my_steps += __shfl_down(my_steps, off);
    if ((threadIdx.x & 63) == 0 && my_steps) atomicAdd(step_total, my_steps);
}

// Clears the per-launch counters (a kernel, so that launches captured in a
// graph need no memset nodes).
__global__ void reset_kernel(int* bad, unsigned long long* step_total, int32_t* item_counter) {
    if (threadIdx.x == 0 && blockIdx.x == 0) {
        *bad = 0;
        *step_total = 0ull;
        *item_counter = 0;
    }
}

// Writes the seed into device memory (single-cube path).
__global__ void seed_kernel(unsigned long long* seed_dev, unsigned long long seed) {
    if (threadIdx.x == 0 && blockIdx.x == 0) *seed_dev = seed;
}

// -------------------------------------------------------------------------
// Host planning.
// -------------------------------------------------------------------------
struct Plan {
    int form;
    int P;
    uint32_t t4_words, table_words;
};

Plan plan_cube(int n, int lattice, int want_form) {
    Plan p{};
    auto tplan = [&](int P) {
        p.P = P;
        uint32_t nodes = (uint32_t)P * P * P;
        p.t4_words = (nodes + 3) / 4 * 4;
        p.table_words = p.t4_words + 4 * nodes;
    };
    if (lattice == MW_LATTICE_VERTEX) {
        const int Pc = n + 2;
        const uint32_t code_words = ((uint32_t)Pc * Pc * Pc + 3) / 4 * 4;
        tplan(n + 1);
        const bool t_fits = p.table_words <= LDS_TABLE_WORDS;
        const bool c_fits = code_words <= LDS_TABLE_WORDS;
        int form = want_form;
        if (form < 0 || form > FORM_TGLOBAL) form = 0;
        if (form == FORM_TLDS && !t_fits) form = 0;
        if (form == FORM_CODES && !c_fits) form = 0;
        if (form == 0) form = t_fits && n <= 16 ? FORM_TLDS : (c_fits ? FORM_CODES : (t_fits ? FORM_TLDS : FORM_TGLOBAL));
        p.form = form;
        if (form == FORM_CODES) {
            p.P = Pc;
            p.t4_words = 0;
            p.table_words = code_words;
        }
    } else {
        tplan(n + 2);
        p.form = p.table_words <= LDS_TABLE_WORDS && want_form != FORM_TGLOBAL ? FORM_TLDS : FORM_TGLOBAL;
    }
    return p;
}

void validate_cube(int n, int lattice) {
    MW_REQUIRE(lattice == MW_LATTICE_VERTEX || lattice == MW_LATTICE_CELL, MW_EINVAL, "unknown lattice %d", lattice);
    MW_REQUIRE(n >= 2 && n <= 64, MW_EINVAL, "n_cells %d outside [2, 64]", n);
    if (lattice == MW_LATTICE_VERTEX)
        MW_REQUIRE(n % 2 == 0, MW_EINVAL, "vertex lattice needs an even n_cells (got %d)", n);
    else
        MW_REQUIRE(n % 2 == 1, MW_EINVAL, "cell lattice needs an odd n_cells (got %d)", n);
}

void allow_large_lds() {
    static bool done = false;
    if (!done) {
        MW_HIP(hipFuncSetAttribute((const void*)walk_kernel, hipFuncAttributeMaxDynamicSharedMemorySize,
                                   (int)(LDS_TABLE_WORDS * 4)));
        done = true;
    }
}

int blocks_per_cu(size_t lds_bytes) {
    return std::max(1, std::min(2, (int)(163840 / (lds_bytes + 1024))));
}

int num_cus() {
    int dev = 0, cus = 0;
    MW_HIP(hipGetDevice(&dev));
    MW_HIP(hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev));
    return cus;
}

struct Launch {
    int waves;
    int groups;
    uint64_t item_walks;
    int wpl;  // interleaved walks per lane
};

Launch default_launch(const mw_tune* t, uint64_t total_walks) {
    Launch L{16, 2, 0, 1};
    if (t) {
        if (t->waves_per_wg > 0) L.waves = std::min(16, std::max(1, (int)t->waves_per_wg));
        if (t->refill_every > 0) L.groups = std::max(1, (int)t->refill_every / 4);
        if (t->item_walks > 0) L.item_walks = (uint64_t)t->item_walks;
        if (t->walks_per_lane > 0) L.wpl = t->walks_per_lane >= 4 ? 4 : (t->walks_per_lane >= 2 ? 2 : 1);
    }
    (void)total_walks;
    return L;
}

}  // namespace
}  // namespace mw

using namespace mw;

namespace mw {
namespace {

// Scratch of one single-cube call: [bad flag | step counter | item counter |
// seed | cube descriptor | prepared table].
constexpr size_t CALL_HDR = 256;

size_t transition_scratch_bytes(const Plan& p) { return CALL_HDR + (size_t)p.table_words * 4; }

// Enqueues one cube's preparation and walks on st with the given device
// scratch (at least transition_scratch_bytes(p)).  Returns false, with
// nothing but the preparation enqueued, when a permittivity is outside
// [1e-3, 1e3]; the range check waits for the preparation kernel.
bool transition_enqueue(const Plan& p, const float* eps, int32_t n_cells, int32_t lattice, uint64_t n_walks,
                        uint64_t first_walk, uint64_t seed, uint32_t cube_index, int32_t* hit_idx,
                        int32_t* steps, hipStream_t st, char* scratch) {
    int* bad = (int*)scratch;
    unsigned long long* step_total = (unsigned long long*)(scratch + 8);
    int32_t* item_counter = (int32_t*)(scratch + 16);
    unsigned long long* seed_dev = (unsigned long long*)(scratch + 24);
    CubeDev* dcube = (CubeDev*)(scratch + 64);
    CubeDev C{};
    C.eps = eps;
    C.table = (uint32_t*)(scratch + CALL_HDR);
    C.hits = hit_idx;
    C.steps = steps;
    C.walk0 = first_walk;
    C.n_walks = n_walks;
    C.n = n_cells;
    C.lattice = lattice;
    C.form = p.form;
    C.P = p.P;
    C.table_words = p.table_words;
    C.t4_words = p.t4_words;
    C.c1 = cube_index;
    const int cen = lattice == MW_LATTICE_VERTEX ? n_cells / 2 : (n_cells - 1) / 2 + 1;
    C.start = cen * (p.P * p.P + p.P + 1);
    // counters cleared by a kernel (no memset node if a caller captures it)
    reset_kernel<<<1, 1, 0, st>>>(bad, step_total, item_counter);
    MW_HIP(hipMemcpyAsync(dcube, &C, sizeof C, hipMemcpyHostToDevice, st));
    const uint32_t nodes = (uint32_t)p.P * p.P * p.P;
    prep_kernel<<<dim3(std::min<uint32_t>((nodes + 255) / 256, 1024), 1), 256, 0, st>>>(dcube, bad);
    MW_HIP(hipGetLastError());
    // eps is device memory: its range check needs one device round trip
    int h_bad = 0;
    MW_HIP(hipMemcpyAsync(&h_bad, bad, sizeof h_bad, hipMemcpyDeviceToHost, st));
    MW_HIP(hipStreamSynchronize(st));
    if (h_bad) return false;
    const Launch L = default_launch(nullptr, n_walks);
    const int threads = 64 * L.waves;
    uint64_t iw = L.item_walks ? L.item_walks : std::max<uint64_t>(threads * 4, 4096);
    const int cus = num_cus();
    // enough items to keep every CU busy
    while (iw > (uint64_t)threads && (n_walks + iw - 1) / iw < (uint64_t)cus * 2) iw /= 2;
    const int64_t n_items = (int64_t)((n_walks + iw - 1) / iw);
    MW_REQUIRE(n_items < (1ll << 31), MW_ELIMIT, "too many walks for one launch");
    const size_t lds = p.form == FORM_TGLOBAL ? 16 : (size_t)p.table_words * 4;
    const int blocks = (int)std::min<int64_t>(n_items, (int64_t)cus * blocks_per_cu(lds));
    allow_large_lds();
    seed_kernel<<<1, 1, 0, st>>>(seed_dev, seed);
    walk_kernel<<<blocks, threads, lds, st>>>(dcube, nullptr, (int32_t)n_items, iw, item_counter, seed_dev,
                                               L.groups, step_total, L.wpl);
    MW_HIP(hipGetLastError());
    return true;
}

constexpr size_t NOALLOC_SCRATCH_BYTES = MW_NOALLOC_SCRATCH_BYTES;
constexpr int MAX_DEVICES = 64;
std::mutex g_scratch_mu;
char* g_scratch_ptr[MAX_DEVICES] = {};

}  // namespace

// Static scratch of mw_transition_noalloc: each device holds its own copy
// until the process ends.  Host code reaches it only through the address
// hipGetSymbolAddress returns for the current device; the array's name is a
// host-side stand-in, not a device address.
__device__ __align__(256) char scratch[NOALLOC_SCRATCH_BYTES];

// Device address of the current device's static scratch (looked up once per
// device, with that device current).
char* noalloc_scratch() {
    int dev = 0;
    MW_HIP(hipGetDevice(&dev));
    MW_REQUIRE(dev >= 0 && dev < MAX_DEVICES, MW_ELIMIT, "device %d beyond the %d supported", dev, MAX_DEVICES);
    std::lock_guard<std::mutex> g(g_scratch_mu);
    if (!g_scratch_ptr[dev]) {
        void* ptr = nullptr;
        MW_HIP(hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch)));
        MW_REQUIRE(ptr, MW_EDEVICE, "no device address for the static scratch");
        g_scratch_ptr[dev] = (char*)ptr;
    }
    return g_scratch_ptr[dev];
}

}  // namespace mw

using namespace mw;

extern "C" mw_status mw_transition(const float* eps, int32_t n_cells, int32_t lattice, uint64_t n_walks,
                                   uint64_t first_walk, uint64_t seed, uint32_t cube_index, int32_t* hit_idx,
                                   int32_t* steps, void* stream) {
    return guarded([&] {
        validate_cube(n_cells, lattice);
        if (n_walks == 0) return;
        MW_REQUIRE(eps && hit_idx, MW_EINVAL, "eps and hit_idx are required");
        hipStream_t st = (hipStream_t)stream;
        const Plan p = plan_cube(n_cells, lattice, 0);
        char* scr = nullptr;
        MW_REQUIRE(!inject_alloc_failure(), MW_ENOMEM, "injected device allocation failure");
        MW_HIP(hipMallocAsync((void**)&scr, transition_scratch_bytes(p), st));
        bool ok = false;
        try {
            ok = transition_enqueue(p, eps, n_cells, lattice, n_walks, first_walk, seed, cube_index, hit_idx, steps,
                                    st, scr);
        } catch (...) {
            (void)hipFreeAsync(scr, st);
            throw;
        }
        MW_HIP(hipFreeAsync(scr, st));
        MW_REQUIRE(ok, MW_EINVAL, "permittivity outside [1e-3, 1e3]");
    });
}

extern "C" mw_status mw_transition_noalloc(const float* eps, int32_t n_cells, int32_t lattice, uint64_t n_walks,
                                           uint64_t first_walk, uint64_t seed, uint32_t cube_index,
                                           int32_t* hit_idx, int32_t* steps, void* stream) {
    return guarded([&] {
        validate_cube(n_cells, lattice);
        if (n_walks == 0) return;
        MW_REQUIRE(eps && hit_idx, MW_EINVAL, "eps and hit_idx are required");
        const Plan p = plan_cube(n_cells, lattice, 0);
        const size_t need = transition_scratch_bytes(p);
        MW_REQUIRE(need <= NOALLOC_SCRATCH_BYTES, MW_ELIMIT,
                   "cube of %d cells needs %zu bytes of scratch; the static scratch holds %zu", n_cells, need,
                   NOALLOC_SCRATCH_BYTES);
        char* scr = noalloc_scratch();
        const bool ok = transition_enqueue(p, eps, n_cells, lattice, n_walks, first_walk, seed, cube_index, hit_idx,
                                           steps, (hipStream_t)stream, scr);
        MW_REQUIRE(ok, MW_EINVAL, "permittivity outside [1e-3, 1e3]");
    });
}

namespace mw {
namespace {

// Device state of one batch: cube descriptors, work items (cubes in
// decreasing cost n^2 * walks, each cube's walk ranges contiguous), prepared
// tables and counters.  enqueue() issues reset + prep + walk kernels only, so
// the sequence can be captured in a graph and replayed.
struct BatchState {
    int n_cubes = 0;
    Launch L{};
    int threads = 0, blocks = 0;
    size_t lds = 0;
    uint32_t n_items = 0;
    uint64_t total_walks = 0;
    char* scratch = nullptr;
    int* bad = nullptr;
    unsigned long long* step_total = nullptr;
    int32_t* item_counter = nullptr;
    unsigned long long* seed_dev = nullptr;
    CubeDev* dcubes = nullptr;
    Item* ditems = nullptr;

    BatchState() = default;
    BatchState(const BatchState&) = delete;
    ~BatchState() { dev_free(scratch); }

    void build(int32_t n, const float* eps_cat, const int64_t* eps_off, const int32_t* n_cells, int32_t lattice,
               const uint64_t* n_walks, const int64_t* out_off, int32_t* hits_cat, int32_t* steps_cat,
               const mw_tune* tune) {
        n_cubes = n;
        L = default_launch(tune, 0);
        threads = 64 * L.waves;
        const int want_form = tune ? tune->tile_form : 0;
        std::vector<CubeDev> cubes(n_cubes);
        std::vector<Plan> plans(n_cubes);
        size_t table_total = 0;
        uint32_t max_lds_words = 4;
        for (int c = 0; c < n_cubes; ++c) {
            validate_cube(n_cells[c], lattice);
            MW_REQUIRE(eps_off[c] >= 0 && out_off[c] >= 0, MW_EINVAL, "negative offset for cube %d", c);
            plans[c] = plan_cube(n_cells[c], lattice, want_form);
            table_total += (size_t)plans[c].table_words * 4;
            total_walks += n_walks[c];
            if (plans[c].form != FORM_TGLOBAL) max_lds_words = std::max(max_lds_words, plans[c].table_words);
        }
        std::vector<int> order(n_cubes);
        for (int c = 0; c < n_cubes; ++c) order[c] = c;
        std::stable_sort(order.begin(), order.end(), [&](int a, int b) {
            const double ca = (double)n_cells[a] * n_cells[a] * n_walks[a];
            const double cb = (double)n_cells[b] * n_cells[b] * n_walks[b];
            return ca > cb;
        });
        const uint64_t iw = L.item_walks ? L.item_walks : (uint64_t)threads * 16;
        std::vector<Item> items;
        for (int c : order)
            for (uint64_t w = 0; w < n_walks[c]; w += iw) items.push_back(Item{c, 0, w, std::min(w + iw, n_walks[c])});
        MW_REQUIRE(items.size() < (1ull << 31), MW_ELIMIT, "too many work items");
        n_items = (uint32_t)items.size();
        const size_t hdr = 256;
        const size_t cubes_bytes = (sizeof(CubeDev) * n_cubes + 255) / 256 * 256;
        const size_t items_bytes = (sizeof(Item) * std::max<size_t>(items.size(), 1) + 255) / 256 * 256;
        scratch = (char*)dev_alloc(hdr + cubes_bytes + items_bytes + table_total + 256);
        bad = (int*)scratch;
        step_total = (unsigned long long*)(scratch + 8);
        item_counter = (int32_t*)(scratch + 16);
        seed_dev = (unsigned long long*)(scratch + 24);
        dcubes = (CubeDev*)(scratch + hdr);
        ditems = (Item*)(scratch + hdr + cubes_bytes);
        char* tables = scratch + hdr + cubes_bytes + items_bytes;
        size_t toff = 0;
        for (int c = 0; c < n_cubes; ++c) {
            const Plan& p = plans[c];
            CubeDev& C = cubes[c];
            C.eps = eps_cat + eps_off[c];
            C.table = (uint32_t*)(tables + toff);
            toff += (size_t)p.table_words * 4;
            C.hits = hits_cat + out_off[c];
            C.steps = steps_cat ? steps_cat + out_off[c] : nullptr;
            C.walk0 = 0;
            C.n_walks = n_walks[c];
            C.n = n_cells[c];
            C.lattice = lattice;
            C.form = p.form;
            C.P = p.P;
            C.table_words = p.table_words;
            C.t4_words = p.t4_words;
            C.c1 = (uint32_t)c;
            const int cen = lattice == MW_LATTICE_VERTEX ? n_cells[c] / 2 : (n_cells[c] - 1) / 2 + 1;
            C.start = cen * (p.P * p.P + p.P + 1);
        }
        MW_HIP(hipMemcpy(dcubes, cubes.data(), sizeof(CubeDev) * n_cubes, hipMemcpyHostToDevice));
        if (!items.empty())
            MW_HIP(hipMemcpy(ditems, items.data(), sizeof(Item) * items.size(), hipMemcpyHostToDevice));
        lds = (size_t)max_lds_words * 4;
        blocks = (int)std::max<size_t>(1, std::min<size_t>(items.size(), (size_t)num_cus() * blocks_per_cu(lds)));
        allow_large_lds();
    }

    // reset + prep + walk; the seed is read from seed_dev
    void enqueue(hipStream_t st, bool with_walk = true) const {
        reset_kernel<<<1, 1, 0, st>>>(bad, step_total, item_counter);
        prep_kernel<<<dim3(64, n_cubes), 256, 0, st>>>(dcubes, bad);
        if (with_walk && n_items)
            walk_kernel<<<blocks, threads, lds, st>>>(dcubes, ditems, (int32_t)n_items, 0, item_counter, seed_dev,
                                                       L.groups, step_total, L.wpl);
    }
};

void check_batch_args(int32_t n_cubes, const float* eps_cat, const int64_t* eps_off, const int32_t* n_cells,
                      const uint64_t* n_walks, const int64_t* out_off, int32_t* hits_cat) {
    MW_REQUIRE(n_cubes >= 0, MW_EINVAL, "n_cubes < 0");
    MW_REQUIRE(n_cubes <= 65535, MW_ELIMIT, "at most 65535 cubes per batch (got %d)", n_cubes);
    if (n_cubes == 0) return;
    MW_REQUIRE(eps_cat && eps_off && n_cells && n_walks && out_off && hits_cat, MW_EINVAL,
               "null argument to a batch call");
}

// Tuned launch settings keyed by the batch's shape (cube-size histogram and
// walk-count scale); filled by mw_autotune_batch.
std::mutex g_tune_mu;
std::map<std::vector<int64_t>, mw_tune> g_tuned;
std::string g_tune_loaded;  // the cache file last read

// Tuned settings persist across processes in the JSON file named by
// MWALK_TUNE_CACHE (when set): {"<device name>": [{"key": [...18 ints],
// "tune": [tile_form, waves_per_wg, refill_every, item_walks,
// walks_per_lane]}, ...]}.  The file holds this device's entries only; it is
// read at the first batch call after MWALK_TUNE_CACHE names it (its entries
// replace those in memory for the same batch shapes) and rewritten after
// every autotune.
std::string tune_device_name() {
    int dev = 0;
    hipDeviceProp_t prop{};
    if (hipGetDevice(&dev) != hipSuccess || hipGetDeviceProperties(&prop, dev) != hipSuccess) return "unknown";
    return std::string(prop.gcnArchName);
}

void load_tune_cache() {  // with g_tune_mu held
    const char* path = getenv("MWALK_TUNE_CACHE");
    if (!path || !*path || g_tune_loaded == path) return;
    g_tune_loaded = path;
    FILE* f = fopen(path, "r");
    if (!f) return;
    std::string text;
    char buf[4096];
    size_t got;
    while ((got = fread(buf, 1, sizeof buf, f)) > 0) text.append(buf, got);
    fclose(f);
    const std::string dev = "\"" + tune_device_name() + "\"";
    size_t at = text.find(dev);
    if (at == std::string::npos) return;
    // entries: every "key": [...] followed by "tune": [...] (the file holds
    // one device's list)
    auto ints = [&](size_t from, std::vector<int64_t>& out) -> size_t {
        const size_t b = text.find('[', from), e = text.find(']', b);
        if (b == std::string::npos || e == std::string::npos) return std::string::npos;
        out.clear();
        const char* p = text.c_str() + b + 1;
        const char* q = text.c_str() + e;
        while (p < q) {
            char* next = nullptr;
            const long long v = strtoll(p, &next, 10);
            if (next == p) {
                ++p;
                continue;
            }
            out.push_back(v);
            p = next;
        }
        return e + 1;
    };
    size_t pos = at;
    for (;;) {
        const size_t k = text.find("\"key\"", pos);
        if (k == std::string::npos) break;
        std::vector<int64_t> key, tv;
        const size_t after_key = ints(k, key);
        if (after_key == std::string::npos) break;
        const size_t t = text.find("\"tune\"", after_key);
        if (t == std::string::npos) break;
        pos = ints(t, tv);
        if (pos == std::string::npos) break;
        if ((key.size() == 18 || (key.size() == 3 && key[0] == -1)) && tv.size() == 5)
            g_tuned[key] = mw_tune{(int32_t)tv[0], (int32_t)tv[1], (int32_t)tv[2], (int32_t)tv[3], (int32_t)tv[4]};
    }
}

void save_tune_cache() {  // with g_tune_mu held
    const char* path = getenv("MWALK_TUNE_CACHE");
    if (!path || !*path) return;
    std::string out = "{\"" + tune_device_name() + "\": [";
    bool first = true;
    for (const auto& kv : g_tuned) {
        out += first ? "\n  {\"key\": [" : ",\n  {\"key\": [";
        first = false;
        for (size_t i = 0; i < kv.first.size(); ++i) out += (i ? ", " : "") + std::to_string(kv.first[i]);
        const mw_tune& t = kv.second;
        out += "], \"tune\": [" + std::to_string(t.tile_form) + ", " + std::to_string(t.waves_per_wg) + ", " +
               std::to_string(t.refill_every) + ", " + std::to_string(t.item_walks) + ", " +
               std::to_string(t.walks_per_lane) + "]}";
    }
    out += "\n]}\n";
    const std::string tmp = std::string(path) + ".tmp";
    FILE* f = fopen(tmp.c_str(), "w");
    if (!f) return;
    const bool ok = fwrite(out.data(), 1, out.size(), f) == out.size();
    if (fclose(f) == 0 && ok) rename(tmp.c_str(), path);
}

std::vector<int64_t> batch_signature(int32_t n_cubes, const int32_t* n_cells, const uint64_t* n_walks,
                                     int32_t lattice) {
    std::vector<int64_t> sig(18, 0);
    sig[0] = lattice;
    uint64_t tot = 0;
    for (int c = 0; c < n_cubes; ++c) {
        sig[1 + std::min(15, n_cells[c] / 4)] += 1;
        tot += n_walks[c];
    }
    sig[17] = (int64_t)std::log2((double)tot + 1.0);
    for (int b = 1; b <= 16; ++b) sig[b] = (int64_t)std::log2((double)sig[b] + 1.0);
    return sig;
}

}  // namespace

// FRW walker launch geometry (resident waves per CU) tuned by frw_autotune,
// kept with the batch settings (key [-1, n, expand m], value in the waves
// field) and in the same MWALK_TUNE_CACHE file.
bool frw_tuned_waves(int n, int expand_m, int* waves) {
    std::lock_guard<std::mutex> g(g_tune_mu);
    load_tune_cache();
    auto it = g_tuned.find(std::vector<int64_t>{-1, n, expand_m});
    if (it == g_tuned.end()) return false;
    *waves = it->second.waves_per_wg;
    return true;
}

void frw_store_waves(int n, int expand_m, int waves) {
    std::lock_guard<std::mutex> g(g_tune_mu);
    load_tune_cache();
    g_tuned[std::vector<int64_t>{-1, n, expand_m}] = mw_tune{0, waves, 0, 0, 0};
    save_tune_cache();
}

}  // namespace mw

using namespace mw;

extern "C" mw_status mw_transition_batch(int32_t n_cubes, const float* eps_cat, const int64_t* eps_off,
                                         const int32_t* n_cells, int32_t lattice, const uint64_t* n_walks,
                                         const int64_t* out_off, uint64_t seed, int32_t* hits_cat,
                                         int32_t* steps_cat, const mw_tune* tune, void* stream) {
    return guarded([&] {
        check_batch_args(n_cubes, eps_cat, eps_off, n_cells, n_walks, out_off, hits_cat);
        if (n_cubes == 0) return;
        hipStream_t st = (hipStream_t)stream;
        mw_tune tuned{};
        if (!tune) {
            std::lock_guard<std::mutex> g(g_tune_mu);
            load_tune_cache();
            auto it = g_tuned.find(batch_signature(n_cubes, n_cells, n_walks, lattice));
            if (it != g_tuned.end()) {
                tuned = it->second;
                tune = &tuned;
            }
        }
        BatchState B;
        B.build(n_cubes, eps_cat, eps_off, n_cells, lattice, n_walks, out_off, hits_cat, steps_cat, tune);
        seed_kernel<<<1, 1, 0, st>>>(B.seed_dev, seed);
        B.enqueue(st, false);
        int h_bad = 0;
        MW_HIP(hipMemcpyAsync(&h_bad, B.bad, sizeof h_bad, hipMemcpyDeviceToHost, st));
        MW_HIP(hipStreamSynchronize(st));
        MW_REQUIRE(!h_bad, MW_EINVAL, "permittivity outside [1e-3, 1e3]");
        if (B.n_items)
            walk_kernel<<<B.blocks, B.threads, B.lds, st>>>(B.dcubes, B.ditems, (int32_t)B.n_items, 0, B.item_counter,
                                                             B.seed_dev, B.L.groups, B.step_total, B.L.wpl);
        MW_HIP(hipGetLastError());
        MW_HIP(hipStreamSynchronize(st));
    });
}

extern "C" mw_status mw_autotune_batch(int32_t n_cubes, const float* eps_cat, const int64_t* eps_off,
                                       const int32_t* n_cells, int32_t lattice, const uint64_t* n_walks,
                                       const int64_t* out_off, int32_t* hits_cat, int32_t* steps_cat,
                                       mw_tune* best, void* stream) {
    return guarded([&] {
        check_batch_args(n_cubes, eps_cat, eps_off, n_cells, n_walks, out_off, hits_cat);
        MW_REQUIRE(best, MW_EINVAL, "null output");
        *best = mw_tune{0, 16, 8, 0, 1};
        if (n_cubes == 0) return;
        hipStream_t st = (hipStream_t)stream;
        hipEvent_t e0, e1;
        MW_HIP(hipEventCreate(&e0));
        MW_HIP(hipEventCreate(&e1));
        struct EG {
            hipEvent_t a, b;
            ~EG() {
                (void)hipEventDestroy(a);
                (void)hipEventDestroy(b);
            }
        } eg{e0, e1};
        auto time_of = [&](const mw_tune& t) {
            BatchState B;
            B.build(n_cubes, eps_cat, eps_off, n_cells, lattice, n_walks, out_off, hits_cat, steps_cat, &t);
            seed_kernel<<<1, 1, 0, st>>>(B.seed_dev, 0x5eedull);
            B.enqueue(st, false);
            int h_bad = 0;
            MW_HIP(hipMemcpyAsync(&h_bad, B.bad, sizeof h_bad, hipMemcpyDeviceToHost, st));
            MW_HIP(hipStreamSynchronize(st));
            MW_REQUIRE(!h_bad, MW_EINVAL, "permittivity outside [1e-3, 1e3]");
            float best_ms = 1e30f;
            for (int rep = 0; rep < 2; ++rep) {
                reset_kernel<<<1, 1, 0, st>>>(B.bad, B.step_total, B.item_counter);
                MW_HIP(hipEventRecord(e0, st));
                walk_kernel<<<B.blocks, B.threads, B.lds, st>>>(B.dcubes, B.ditems, (int32_t)B.n_items, 0,
                                                                 B.item_counter, B.seed_dev, B.L.groups, B.step_total,
                                                                 B.L.wpl);
                MW_HIP(hipEventRecord(e1, st));
                MW_HIP(hipEventSynchronize(e1));
                float ms = 0.f;
                MW_HIP(hipEventElapsedTime(&ms, e0, e1));
                best_ms = std::min(best_ms, ms);
            }
            return best_ms;
        };
        // coordinate search: tile form, waves per workgroup, refill interval,
        // walks per work item, interleaved walks per lane
        mw_tune cur{0, 16, 8, 0, 1};
        float cur_ms = time_of(cur);
        auto try_set = [&](int field, const std::vector<int>& vals) {
            for (int v : vals) {
                mw_tune t = cur;
                int* f = field == 0   ? &t.tile_form
                         : field == 1 ? &t.waves_per_wg
                         : field == 2 ? &t.refill_every
                         : field == 3 ? &t.item_walks
                                      : &t.walks_per_lane;
                if (*f == v) continue;
                *f = v;
                const float ms = time_of(t);
                if (ms < cur_ms) {
                    cur_ms = ms;
                    cur = t;
                }
            }
        };
        try_set(0, {2});
        try_set(1, {4, 8});
        try_set(2, {4, 16});
        const int thr = 64 * cur.waves_per_wg;
        try_set(3, {thr * 4, thr * 64});
        try_set(4, {2, 4});
        *best = cur;
        std::lock_guard<std::mutex> g(g_tune_mu);
        g_tuned[batch_signature(n_cubes, n_cells, n_walks, lattice)] = cur;
        save_tune_cache();
    });
}

// A batch captured once as a graph of (reset, prep, walk) kernels and
// replayed with a new seed per run.
struct mw_batch_plan {
    BatchState B;
    hipGraph_t graph = nullptr;
    hipGraphExec_t exec = nullptr;
    unsigned long long* seed_host = nullptr;
    ~mw_batch_plan() {
        if (exec) (void)hipGraphExecDestroy(exec);
        if (graph) (void)hipGraphDestroy(graph);
        if (seed_host) (void)hipHostFree(seed_host);
    }
};

extern "C" mw_status mw_tune_lookup(int32_t n_cubes, const int32_t* n_cells, const uint64_t* n_walks,
                                    int32_t lattice, mw_tune* out, int32_t* found) {
    return guarded([&] {
        MW_REQUIRE(n_cubes > 0 && n_cells && n_walks && out && found, MW_EINVAL, "bad arguments");
        std::lock_guard<std::mutex> g(g_tune_mu);
        load_tune_cache();
        auto it = g_tuned.find(batch_signature(n_cubes, n_cells, n_walks, lattice));
        *found = it != g_tuned.end() ? 1 : 0;
        if (*found) *out = it->second;
    });
}

extern "C" mw_status mw_batch_plan_create(int32_t n_cubes, const float* eps_cat, const int64_t* eps_off,
                                          const int32_t* n_cells, int32_t lattice, const uint64_t* n_walks,
                                          const int64_t* out_off, int32_t* hits_cat, int32_t* steps_cat,
                                          const mw_tune* tune, mw_batch_plan** out) {
    return guarded([&] {
        MW_REQUIRE(out, MW_EINVAL, "null output handle");
        check_batch_args(n_cubes, eps_cat, eps_off, n_cells, n_walks, out_off, hits_cat);
        MW_REQUIRE(n_cubes > 0, MW_EINVAL, "empty batch");
        mw_tune tuned{};
        if (!tune) {
            std::lock_guard<std::mutex> g(g_tune_mu);
            load_tune_cache();
            auto it = g_tuned.find(batch_signature(n_cubes, n_cells, n_walks, lattice));
            if (it != g_tuned.end()) {
                tuned = it->second;
                tune = &tuned;
            }
        }
        auto P = std::make_unique<mw_batch_plan>();
        P->B.build(n_cubes, eps_cat, eps_off, n_cells, lattice, n_walks, out_off, hits_cat, steps_cat, tune);
        // validate the permittivities once, eagerly
        hipStream_t st = nullptr;
        MW_HIP(hipStreamCreateWithFlags(&st, hipStreamNonBlocking));
        struct SG {
            hipStream_t s;
            ~SG() { (void)hipStreamDestroy(s); }
        } sg{st};
        P->B.enqueue(st, false);
        int h_bad = 0;
        MW_HIP(hipMemcpyAsync(&h_bad, P->B.bad, sizeof h_bad, hipMemcpyDeviceToHost, st));
        MW_HIP(hipStreamSynchronize(st));
        MW_REQUIRE(!h_bad, MW_EINVAL, "permittivity outside [1e-3, 1e3]");
        MW_HIP(hipHostMalloc((void**)&P->seed_host, sizeof(unsigned long long), hipHostMallocDefault));
        MW_HIP(hipStreamBeginCapture(st, hipStreamCaptureModeThreadLocal));
        P->B.enqueue(st, true);
        MW_HIP(hipStreamEndCapture(st, &P->graph));
        MW_HIP(hipGraphInstantiate(&P->exec, P->graph, nullptr, nullptr, 0));
        *out = P.release();
    });
}

extern "C" mw_status mw_batch_plan_run(mw_batch_plan* P, uint64_t seed, void* stream) {
    return guarded([&] {
        MW_REQUIRE(P, MW_EINVAL, "null plan");
        hipStream_t st = (hipStream_t)stream;
        // the previous run's copy of the seed must have completed before the
        // pinned word is rewritten
        MW_HIP(hipStreamSynchronize(st));
        *P->seed_host = seed;
        MW_HIP(hipMemcpyAsync(P->B.seed_dev, P->seed_host, sizeof(unsigned long long), hipMemcpyHostToDevice, st));
        MW_HIP(hipGraphLaunch(P->exec, st));
    });
}

extern "C" mw_status mw_batch_plan_destroy(mw_batch_plan* P) {
    return guarded([&] {
        if (!P) return;
        (void)hipDeviceSynchronize();
        delete P;
    });
}
