// mwo.cpp — CPU oracle for FRW capacitance extraction with MicroWalk
// transitions (Huang & Yu, arXiv 2507.09730).
//
// TEST INFRASTRUCTURE ONLY.  This file is the plain, slow reference that the
// GPU library is checked against.  Only the test suite, the smoke check and
// the benchmark's CPU-baseline leg may load it.  It shares no code, header or
// table with the GPU library; it is built from this file alone with
// `g++ -O2 -ffp-contract=off -shared -fPIC`.
//
// Both node placements are implemented for FRW: the vertex lattice (nodes at
// cell corners, the default) and the cell-centred lattice of Sec. III-A
// (nodes at voxel centres, Eq. (6) coefficients, lattice = 1).
//
// Arithmetic is binary64 except where the method is specified in integers
// (cell and link codes, thresholds, Philox words).  Each function names the
// passage of the paper it follows; readings of points the paper leaves open
// are stated where they are used.
//
// Parity status: every function below is pinned by a CPU test against values
// the paper or the mathematics fixes, except the first-transition weight of
// non-stratified (homogenised) first cubes and the voxelisation bias of the
// series parallel-plate case, which are "parity unpinned" (checked only for
// self-consistency: reciprocity, row sums, GPU agreement).

#include <algorithm>
#include <atomic>
#include <cmath>
#include <cstdint>
#include <cstring>
#include <map>
#include <memory>
#include <mutex>
#include <thread>
#include <vector>

namespace {

// ---------------------------------------------------------------------------
// Philox4x32-10 (Salmon, Moraes, Dror & Shaw, "Parallel random numbers: as
// easy as 1, 2, 3", SC'11).  Round: two 32x32->64 products of counter words 0
// and 2 with the round multipliers; the high halves are xored with the other
// counter word and a key word; the key is advanced by the Weyl constants
// between rounds.
// ---------------------------------------------------------------------------
void philox4x32_10(const uint32_t ctr_in[4], const uint32_t key_in[2], uint32_t out[4]) {
    uint32_t c[4] = {ctr_in[0], ctr_in[1], ctr_in[2], ctr_in[3]};
    uint32_t k0 = key_in[0], k1 = key_in[1];
    for (int r = 0; r < 10; ++r) {
        if (r > 0) {
            k0 += 0x9E3779B9u;
            k1 += 0xBB67AE85u;
        }
        uint64_t p0 = (uint64_t)0xD2511F53u * c[0];
        uint64_t p1 = (uint64_t)0xCD9E8D57u * c[2];
        uint32_t hi0 = (uint32_t)(p0 >> 32), lo0 = (uint32_t)p0;
        uint32_t hi1 = (uint32_t)(p1 >> 32), lo1 = (uint32_t)p1;
        uint32_t n0 = hi1 ^ c[1] ^ k0;
        uint32_t n2 = hi0 ^ c[3] ^ k1;
        c[0] = n0;
        c[1] = lo1;
        c[2] = n2;
        c[3] = lo0;
    }
    for (int i = 0; i < 4; ++i) out[i] = c[i];
}

// Word s of the stream identified by (seed, c1, walk, purpose).
uint32_t rng_word(uint64_t seed, uint32_t c1, uint64_t walk, uint32_t purpose, uint64_t s) {
    uint32_t key[2] = {(uint32_t)seed, (uint32_t)(seed >> 32)};
    uint32_t ctr[4] = {(uint32_t)(s >> 2), c1, (uint32_t)walk,
                       (uint32_t)((walk >> 32) & 0xffffffu) | (purpose << 24)};
    uint32_t out[4];
    philox4x32_10(ctr, key, out);
    return out[s & 3];
}

double u01(uint32_t u) { return ((double)u + 0.5) * (1.0 / 4294967296.0); }

enum { PURPOSE_MW = 0, PURPOSE_GAUSS = 1, PURPOSE_FIRST = 2, PURPOSE_TABLE = 3 };

// ---------------------------------------------------------------------------
// Integer codes and thresholds.
//
// Sec. III-A, Eq. (6): the walk at node v moves to neighbour i with
// probability alpha_i / sum(alpha).  On the vertex lattice the normalised
// alpha of a link is its face conductance: the sum of the permittivities of
// the four cells that share the link (each cell code is rint(eps * 2^16)).
// On the cell lattice alpha is Eq. (6) verbatim, stored as
// rint(alpha * 2^24).  Prefix sums S_k of the six codes (order -x,+x,-y,+y,
// -z,+z) give thresholds T_k = ceil(S_k 2^32 / S_5); a uniform 32-bit word u
// picks direction #{k <= 4 : u >= T_k}.
// ---------------------------------------------------------------------------
uint64_t vertex_cell_code(float eps) { return (uint64_t)std::nearbyint((double)eps * 65536.0); }

uint64_t cell_link_code(float eps_nb, float eps_v) {
    double a = (double)eps_nb / ((double)eps_nb + (double)eps_v);
    return (uint64_t)std::nearbyint(a * 16777216.0);
}

void thresholds_from_codes(const uint64_t g[6], uint32_t T[5]) {
    uint64_t S[6];
    uint64_t acc = 0;
    for (int d = 0; d < 6; ++d) {
        acc += g[d];
        S[d] = acc;
    }
    // 128-bit numerator: cut links of MicroWalk-E can push S_k past 2^32
    for (int k = 0; k < 5; ++k)
        T[k] = (uint32_t)((((unsigned __int128)S[k] << 32) + S[5] - 1) / S[5]);
}

int choose_direction(uint32_t u, const uint32_t T[5]) {
    int d = 0;
    for (int k = 0; k < 5; ++k)
        if (u >= T[k]) ++d;
    return d;
}

const int DIR[6][3] = {{-1, 0, 0}, {1, 0, 0}, {0, -1, 0}, {0, 1, 0}, {0, 0, -1}, {0, 0, 1}};

// Vertex lattice over n^3 cells with codes e[(k*n+j)*n+i]; nodes (i,j,k) in
// [0,n]^3, interior [1,n-1]^3.  Link code of direction d at interior node.
uint64_t vertex_link(const std::vector<uint64_t>& e, int n, int i, int j, int k, int d) {
    auto E = [&](int x, int y, int z) { return e[((size_t)z * n + y) * n + x]; };
    switch (d) {
        case 0: return E(i - 1, j - 1, k - 1) + E(i - 1, j, k - 1) + E(i - 1, j - 1, k) + E(i - 1, j, k);
        case 1: return E(i, j - 1, k - 1) + E(i, j, k - 1) + E(i, j - 1, k) + E(i, j, k);
        case 2: return E(i - 1, j - 1, k - 1) + E(i, j - 1, k - 1) + E(i - 1, j - 1, k) + E(i, j - 1, k);
        case 3: return E(i - 1, j, k - 1) + E(i, j, k - 1) + E(i - 1, j, k) + E(i, j, k);
        case 4: return E(i - 1, j - 1, k - 1) + E(i, j - 1, k - 1) + E(i - 1, j, k - 1) + E(i, j, k - 1);
        default: return E(i - 1, j - 1, k) + E(i, j - 1, k) + E(i - 1, j, k) + E(i, j, k);
    }
}

// Hit index of a boundary node of the vertex lattice (exactly one coordinate
// on {0, n}).
int vertex_hit_index(int n, int i, int j, int k) {
    int M = n - 1;
    int c[3] = {i, j, k};
    for (int ax = 0; ax < 3; ++ax) {
        if (c[ax] == 0 || c[ax] == n) {
            int side = c[ax] == n ? 1 : 0;
            int a = ax == 0 ? c[1] : c[0];
            int b = ax == 2 ? c[1] : c[2];
            return (2 * ax + side) * M * M + (b - 1) * M + (a - 1);
        }
    }
    return -1;
}

void vertex_node_of_hit(int n, int hit, int node[3]) {
    int M = n - 1;
    int f = hit / (M * M), rem = hit % (M * M);
    int b = rem / M + 1, a = rem % M + 1;
    int ax = f / 2, side = f % 2;
    int o0 = ax == 0 ? 1 : 0, o1 = ax == 2 ? 1 : 2;
    node[ax] = side ? n : 0;
    node[o0] = a;
    node[o1] = b;
}

// Alg. 3 on the vertex lattice: from the centre node, repeat {direction from
// the node's thresholds; move} until a boundary node is reached.
int microwalk_vertex(const std::vector<uint64_t>& e, int n, const int start[3], uint64_t seed,
                     uint32_t c1, uint64_t walk, int32_t* steps_out, int node_out[3]) {
    int p[3] = {start[0], start[1], start[2]};
    uint64_t s = 0;
    for (;;) {
        if (s >= (1ull << 30)) {
            if (steps_out) *steps_out = (int32_t)s;
            return -1;
        }
        uint64_t g[6];
        for (int d = 0; d < 6; ++d) g[d] = vertex_link(e, n, p[0], p[1], p[2], d);
        uint32_t T[5];
        thresholds_from_codes(g, T);
        uint32_t u = rng_word(seed, c1, walk, PURPOSE_MW, s);
        int d = choose_direction(u, T);
        for (int a = 0; a < 3; ++a) p[a] += DIR[d][a];
        ++s;
        if (p[0] == 0 || p[0] == n || p[1] == 0 || p[1] == n || p[2] == 0 || p[2] == n) {
            if (steps_out) *steps_out = (int32_t)s;
            if (node_out)
                for (int a = 0; a < 3; ++a) node_out[a] = p[a];
            return vertex_hit_index(n, p[0], p[1], p[2]);
        }
    }
}

// MicroWalk-E (Sec. III-B, Fig. 3(b)): Alg. 3 on the vertex lattice of an
// expanded cube whose interior nodes may be absorbing (inside a conductor or
// beyond a grounded window face).  absorb[(k*(n+1)+j)*(n+1)+i] = -1 for a free
// node, else the net that absorbs the walk (n_nets = grounded enclosure).
// Reading of "adjusts the lattice accordingly": a link from a free node into
// an absorbing node is cut where it enters the conductor (or meets the
// grounded face), at a fraction theta of its length (at least 1/16, which
// keeps the codes bounded), and its code becomes rint(code / theta) — the
// Shortley-Weller treatment of a Dirichlet boundary between nodes, exact for
// linear potentials; the walk that takes it is absorbed.  Returns the hit index of a boundary node, or -2 with *net_out
// set when an absorbing interior node is reached.  Same random stream as
// Alg. 3.
typedef double (*ThetaFn)(const void* ctx, const int p[3], int d);
int microwalk_vertex_e(const std::vector<uint64_t>& e, const std::vector<int32_t>& absorb, int n, uint64_t seed,
                       uint32_t c1, uint64_t walk, int32_t* steps_out, int* net_out, ThetaFn theta = nullptr,
                       const void* ctx = nullptr) {
    int p[3] = {n / 2, n / 2, n / 2};
    uint64_t s = 0;
    for (;;) {
        if (s >= (1ull << 30)) {
            if (steps_out) *steps_out = (int32_t)s;
            return -1;
        }
        uint64_t g[6];
        for (int d = 0; d < 6; ++d) {
            g[d] = vertex_link(e, n, p[0], p[1], p[2], d);
            if (theta) {
                int q[3] = {p[0] + DIR[d][0], p[1] + DIR[d][1], p[2] + DIR[d][2]};
                bool interior = q[0] > 0 && q[0] < n && q[1] > 0 && q[1] < n && q[2] > 0 && q[2] < n;
                if (interior && absorb[((size_t)q[2] * (n + 1) + q[1]) * (n + 1) + q[0]] >= 0) {
                    const double th = theta(ctx, p, d);
                    g[d] = (uint64_t)std::nearbyint((double)g[d] / th);
                }
            }
        }
        uint32_t T[5];
        thresholds_from_codes(g, T);
        uint32_t u = rng_word(seed, c1, walk, PURPOSE_MW, s);
        int d = choose_direction(u, T);
        for (int a = 0; a < 3; ++a) p[a] += DIR[d][a];
        ++s;
        if (p[0] == 0 || p[0] == n || p[1] == 0 || p[1] == n || p[2] == 0 || p[2] == n) {
            if (steps_out) *steps_out = (int32_t)s;
            return vertex_hit_index(n, p[0], p[1], p[2]);
        }
        const int32_t a = absorb[((size_t)p[2] * (n + 1) + p[1]) * (n + 1) + p[0]];
        if (a >= 0) {
            if (steps_out) *steps_out = (int32_t)s;
            *net_out = a;
            return -2;
        }
    }
}

// Alg. 3 on the cell-centred lattice of Sec. III-A (nodes at voxel centres,
// boundary nodes at panel centres, coefficients of Eq. 6).
int microwalk_cell(const float* eps, int N, uint64_t seed, uint32_t c1, uint64_t walk, int32_t* steps_out) {
    int p[3] = {(N - 1) / 2, (N - 1) / 2, (N - 1) / 2};
    uint64_t s = 0;
    auto EPS = [&](int x, int y, int z) { return eps[((size_t)z * N + y) * N + x]; };
    for (;;) {
        if (s >= (1ull << 30)) {
            if (steps_out) *steps_out = (int32_t)s;
            return -1;
        }
        uint64_t g[6];
        float ev = EPS(p[0], p[1], p[2]);
        for (int d = 0; d < 6; ++d) {
            int q[3] = {p[0] + DIR[d][0], p[1] + DIR[d][1], p[2] + DIR[d][2]};
            bool inside = q[0] >= 0 && q[0] < N && q[1] >= 0 && q[1] < N && q[2] >= 0 && q[2] < N;
            g[d] = inside ? cell_link_code(EPS(q[0], q[1], q[2]), ev) : (1ull << 24);
        }
        uint32_t T[5];
        thresholds_from_codes(g, T);
        uint32_t u = rng_word(seed, c1, walk, PURPOSE_MW, s);
        int d = choose_direction(u, T);
        for (int a = 0; a < 3; ++a) p[a] += DIR[d][a];
        ++s;
        for (int ax = 0; ax < 3; ++ax) {
            if (p[ax] < 0 || p[ax] >= N) {
                int side = p[ax] >= N ? 1 : 0;
                int a = ax == 0 ? p[1] : p[0];
                int b = ax == 2 ? p[1] : p[2];
                if (steps_out) *steps_out = (int32_t)s;
                return (2 * ax + side) * N * N + b * N + a;
            }
        }
    }
}

// ---------------------------------------------------------------------------
// Exact discrete SGF of the vertex lattice (Eqs. 7-8, 11).
//
// With integer link codes G (symmetric: a link has the same code seen from
// both ends) and D_v = sum of the six codes at v, the chain of Alg. 3 has
// Q_II = D^-1 G_II, so (I - Q_II)^-1 = (D - G_II)^-1 D.  Solving
// (D - G_II) z = e_src once gives the exit distribution from the source,
// P_b = sum_v z_v G_vb (Eq. 8 via Theorem 1) and the expected number of steps
// E(tau) = sum_v z_v D_v (Eq. 11).  D - G_II is symmetric positive definite;
// the solve is Jacobi-preconditioned conjugate gradients to a relative
// residual of 1e-14.
// ---------------------------------------------------------------------------
struct VertexSystem {
    int n, M;
    std::vector<double> g;  // 6 per interior node
    std::vector<double> D;
    size_t idx(int i, int j, int k) const { return ((size_t)(k - 1) * M + (j - 1)) * M + (i - 1); }
};

VertexSystem build_vertex_system(const std::vector<uint64_t>& e, int n) {
    VertexSystem S;
    S.n = n;
    S.M = n - 1;
    size_t NI = (size_t)S.M * S.M * S.M;
    S.g.resize(NI * 6);
    S.D.resize(NI);
    for (int k = 1; k < n; ++k)
        for (int j = 1; j < n; ++j)
            for (int i = 1; i < n; ++i) {
                size_t v = S.idx(i, j, k);
                double D = 0;
                for (int d = 0; d < 6; ++d) {
                    double gd = (double)vertex_link(e, n, i, j, k, d);
                    S.g[v * 6 + d] = gd;
                    D += gd;
                }
                S.D[v] = D;
            }
    return S;
}

void apply_vertex(const VertexSystem& S, const std::vector<double>& x, std::vector<double>& y) {
    int n = S.n;
    for (int k = 1; k < n; ++k)
        for (int j = 1; j < n; ++j)
            for (int i = 1; i < n; ++i) {
                size_t v = S.idx(i, j, k);
                double acc = S.D[v] * x[v];
                for (int d = 0; d < 6; ++d) {
                    int q[3] = {i + DIR[d][0], j + DIR[d][1], k + DIR[d][2]};
                    if (q[0] == 0 || q[0] == n || q[1] == 0 || q[1] == n || q[2] == 0 || q[2] == n) continue;
                    acc -= S.g[v * 6 + d] * x[S.idx(q[0], q[1], q[2])];
                }
                y[v] = acc;
            }
}

bool solve_vertex(const VertexSystem& S, const std::vector<double>& b, std::vector<double>& x) {
    size_t N = S.D.size();
    x.assign(N, 0.0);
    std::vector<double> r = b, z(N), p(N), Ap(N);
    double bnorm = 0;
    for (double v : b) bnorm += v * v;
    bnorm = std::sqrt(bnorm);
    if (bnorm == 0) return true;
    for (size_t i = 0; i < N; ++i) z[i] = r[i] / S.D[i];
    p = z;
    double rz = 0;
    for (size_t i = 0; i < N; ++i) rz += r[i] * z[i];
    for (int it = 0; it < 50000; ++it) {
        apply_vertex(S, p, Ap);
        double pAp = 0;
        for (size_t i = 0; i < N; ++i) pAp += p[i] * Ap[i];
        double alpha = rz / pAp;
        double rn = 0;
        for (size_t i = 0; i < N; ++i) {
            x[i] += alpha * p[i];
            r[i] -= alpha * Ap[i];
            rn += r[i] * r[i];
        }
        if (std::sqrt(rn) <= 1e-14 * bnorm) return true;
        for (size_t i = 0; i < N; ++i) z[i] = r[i] / S.D[i];
        double rz2 = 0;
        for (size_t i = 0; i < N; ++i) rz2 += r[i] * z[i];
        double beta = rz2 / rz;
        rz = rz2;
        for (size_t i = 0; i < N; ++i) p[i] = z[i] + beta * p[i];
    }
    return false;
}

// Exit distribution P (6 M^2 entries, hit-index order) and E(tau) from
// interior source node src.
bool sgf_vertex(const VertexSystem& S, const int src[3], std::vector<double>& P, double* etau) {
    int n = S.n, M = S.M;
    std::vector<double> b(S.D.size(), 0.0), z;
    b[S.idx(src[0], src[1], src[2])] = 1.0;
    if (!solve_vertex(S, b, z)) return false;
    P.assign((size_t)6 * M * M, 0.0);
    double et = 0;
    for (int k = 1; k < n; ++k)
        for (int j = 1; j < n; ++j)
            for (int i = 1; i < n; ++i) {
                size_t v = S.idx(i, j, k);
                et += z[v] * S.D[v];
                for (int d = 0; d < 6; ++d) {
                    int q[3] = {i + DIR[d][0], j + DIR[d][1], k + DIR[d][2]};
                    if (q[0] == 0 || q[0] == n || q[1] == 0 || q[1] == n || q[2] == 0 || q[2] == n)
                        P[vertex_hit_index(n, q[0], q[1], q[2])] += z[v] * S.g[v * 6 + d];
                }
            }
    if (etau) *etau = et;
    return true;
}

// ---------------------------------------------------------------------------
// Exact discrete SGF of the cell-centred lattice (Sec. III-A; Eqs. 7-8, 11).
//
// The Eq. (6) codes of a node are normalised by its own permittivity, so the
// code of a link seen from its two ends differs and G is not symmetric.  The
// chain of Alg. 3 is still Q_II = D^-1 G_II; the source row of
// (I - Q_II)^-1 Q_IB is P_b = sum_v y_v G_vb with (D - G_II)^T y = e_src,
// and E(tau) = sum_v y_v D_v.  The solve is Jacobi-preconditioned BiCGSTAB
// (van der Vorst) to a relative residual of 1e-14, checked on the true
// residual and restarted from the current iterate when the recursive one
// has drifted.
// ---------------------------------------------------------------------------
struct CellSystem {
    int N;
    std::vector<uint64_t> g;  // 6 per node: Eq. (6) codes, 2^24 towards a boundary panel
    std::vector<double> D;
};

CellSystem build_cell_system(const std::vector<float>& eps, int N) {
    CellSystem S;
    S.N = N;
    const size_t NI = (size_t)N * N * N;
    S.g.resize(NI * 6);
    S.D.resize(NI);
    auto EPS = [&](int x, int y, int z) { return eps[((size_t)z * N + y) * N + x]; };
    for (int k = 0; k < N; ++k)
        for (int j = 0; j < N; ++j)
            for (int i = 0; i < N; ++i) {
                const size_t v = ((size_t)k * N + j) * N + i;
                uint64_t sum = 0;
                for (int d = 0; d < 6; ++d) {
                    const int q[3] = {i + DIR[d][0], j + DIR[d][1], k + DIR[d][2]};
                    const bool inside = q[0] >= 0 && q[0] < N && q[1] >= 0 && q[1] < N && q[2] >= 0 && q[2] < N;
                    const uint64_t c = inside ? cell_link_code(EPS(q[0], q[1], q[2]), EPS(i, j, k)) : (1ull << 24);
                    S.g[v * 6 + d] = c;
                    sum += c;
                }
                S.D[v] = (double)sum;
            }
    return S;
}

// y = (D - G_II)^T x
void apply_cell_t(const CellSystem& S, const std::vector<double>& x, std::vector<double>& y) {
    const int N = S.N;
    y.assign(x.size(), 0.0);
    for (size_t v = 0; v < x.size(); ++v) y[v] = S.D[v] * x[v];
    for (int k = 0; k < N; ++k)
        for (int j = 0; j < N; ++j)
            for (int i = 0; i < N; ++i) {
                const size_t v = ((size_t)k * N + j) * N + i;
                for (int d = 0; d < 6; ++d) {
                    const int q[3] = {i + DIR[d][0], j + DIR[d][1], k + DIR[d][2]};
                    if (q[0] < 0 || q[0] >= N || q[1] < 0 || q[1] >= N || q[2] < 0 || q[2] >= N) continue;
                    y[((size_t)q[2] * N + q[1]) * N + q[0]] -= (double)S.g[v * 6 + d] * x[v];
                }
            }
}

static double norm2(const std::vector<double>& a) {
    double s = 0;
    for (double v : a) s += v * v;
    return std::sqrt(s);
}
static double dotp(const std::vector<double>& a, const std::vector<double>& b) {
    double s = 0;
    for (size_t i = 0; i < a.size(); ++i) s += a[i] * b[i];
    return s;
}

bool solve_cell_t(const CellSystem& S, const std::vector<double>& b, std::vector<double>& x) {
    const size_t NI = S.D.size();
    x.assign(NI, 0.0);
    const double bn = norm2(b);
    if (bn == 0) return true;
    std::vector<double> r(NI), rh(NI), p(NI), v(NI), s(NI), t(NI), y(NI), z(NI), ax(NI);
    for (int restart = 0; restart < 8; ++restart) {
        apply_cell_t(S, x, ax);
        for (size_t i = 0; i < NI; ++i) r[i] = b[i] - ax[i];
        if (norm2(r) <= 1e-14 * bn) return true;
        rh = r;
        std::fill(p.begin(), p.end(), 0.0);
        std::fill(v.begin(), v.end(), 0.0);
        double rho = 1, alpha = 1, omega = 1;
        for (int it = 0; it < 20000; ++it) {
            const double rho1 = dotp(rh, r);
            if (rho1 == 0) break;
            const double beta = (rho1 / rho) * (alpha / omega);
            for (size_t i = 0; i < NI; ++i) p[i] = r[i] + beta * (p[i] - omega * v[i]);
            for (size_t i = 0; i < NI; ++i) y[i] = p[i] / S.D[i];
            apply_cell_t(S, y, v);
            alpha = rho1 / dotp(rh, v);
            for (size_t i = 0; i < NI; ++i) {
                s[i] = r[i] - alpha * v[i];
                x[i] += alpha * y[i];
            }
            if (norm2(s) <= 1e-14 * bn) break;
            for (size_t i = 0; i < NI; ++i) z[i] = s[i] / S.D[i];
            apply_cell_t(S, z, t);
            omega = dotp(t, s) / dotp(t, t);
            for (size_t i = 0; i < NI; ++i) {
                x[i] += omega * z[i];
                r[i] = s[i] - omega * t[i];
            }
            rho = rho1;
            if (norm2(r) <= 1e-14 * bn || omega == 0) break;
        }
    }
    apply_cell_t(S, x, ax);
    for (size_t i = 0; i < NI; ++i) r[i] = b[i] - ax[i];
    return norm2(r) <= 1e-14 * bn;
}

// Hit index of boundary panel (axis ax, side, in-face coordinates a, b) of
// the cell lattice, as microwalk_cell numbers them.
int cell_hit_index(int N, int ax, int side, int a, int b) { return (2 * ax + side) * N * N + b * N + a; }

// Exit distribution P (6 N^2 entries, hit-index order) and E(tau) from the
// node (voxel) src.
bool sgf_cell(const CellSystem& S, const int src[3], std::vector<double>& P, double* etau) {
    const int N = S.N;
    std::vector<double> b(S.D.size(), 0.0), y;
    b[((size_t)src[2] * N + src[1]) * N + src[0]] = 1.0;
    if (!solve_cell_t(S, b, y)) return false;
    P.assign((size_t)6 * N * N, 0.0);
    double et = 0;
    for (int k = 0; k < N; ++k)
        for (int j = 0; j < N; ++j)
            for (int i = 0; i < N; ++i) {
                const size_t v = ((size_t)k * N + j) * N + i;
                et += y[v] * S.D[v];
                for (int d = 0; d < 6; ++d) {
                    const int q[3] = {i + DIR[d][0], j + DIR[d][1], k + DIR[d][2]};
                    const int ax = d / 2;
                    if (q[ax] >= 0 && q[ax] < N) continue;
                    const int a = ax == 0 ? q[1] : q[0];
                    const int bb = ax == 2 ? q[1] : q[2];
                    P[cell_hit_index(N, ax, q[ax] >= N ? 1 : 0, a, bb)] += y[v] * (double)S.g[v * 6 + d];
                }
            }
    if (etau) *etau = et;
    return true;
}

// ---------------------------------------------------------------------------
// Geometry (Alg. 1 input) and voxelisation of transition cubes.
// ---------------------------------------------------------------------------
struct Box {
    double lo[3], hi[3];
    int net;     // conductors
    float eps;   // dielectrics
};

struct Structure {
    std::vector<Box> cond;
    int n_nets = 0;
    std::vector<Box> diel;
    std::vector<double> layer_z0;
    std::vector<float> layer_eps;
    double wlo[3], whi[3];
    int bc[6];
};

const double EPS0 = 8.8541878128e-3;  // vacuum permittivity, fF/um
const int HOP_CAP = 100000;
const int MAX_BOXES = 16;  // dielectric boxes of one GPU cube mask (kernel_limits only)

double box_point_dist(const Box& b, const double p[3]) {
    double d = 0;
    for (int a = 0; a < 3; ++a) {
        double da = std::max(std::max(b.lo[a] - p[a], p[a] - b.hi[a]), 0.0);
        d = std::max(d, da);
    }
    return d;
}

// Largest conductor-free cube around p (L-infinity distance to the nearest
// conductor or grounded window face).  nearest = net index, or n_nets for a
// grounded face.
double structure_dist(const Structure& S, const double p[3], int* nearest) {
    double best = INFINITY;
    int who = S.n_nets;
    for (const Box& b : S.cond) {
        double d = box_point_dist(b, p);
        if (d < best) {
            best = d;
            who = b.net;
        }
    }
    for (int a = 0; a < 3; ++a) {
        if (S.bc[2 * a] == 0) {
            double d = p[a] - S.wlo[a];
            if (d < best) {
                best = d;
                who = S.n_nets;
            }
        }
        if (S.bc[2 * a + 1] == 0) {
            double d = S.whi[a] - p[a];
            if (d < best) {
                best = d;
                who = S.n_nets;
            }
        }
    }
    if (nearest) *nearest = who;
    return best;
}

// Number of dielectric boxes touching the cube [c-R, c+R] (faces clipped to
// the window at symmetry walls).
int boxes_touching(const Structure& S, const double c[3], double R) {
    int cnt = 0;
    for (const Box& b : S.diel) {
        bool touch = true;
        for (int a = 0; a < 3; ++a) {
            double lo = c[a] - R, hi = c[a] + R;
            if (S.bc[2 * a] == 1) lo = std::max(lo, S.wlo[a]);
            if (S.bc[2 * a + 1] == 1) hi = std::min(hi, S.whi[a]);
            if (!(b.lo[a] <= hi && b.hi[a] >= lo)) touch = false;
        }
        cnt += touch;
    }
    return cnt;
}

// Cube-size rule (reading of "build the transition cube centred at r",
// Alg. 3, and of the conductor-free cubes of Sec. III-B): the largest
// conductor-free cube, R = the distance d from c to the nearest conductor or
// grounded face.
//
// kernel_limits (test option, never the default): the GPU kernel keeps the
// dielectric boxes of a cube in a 16-bit mask and halves a cube while more
// than MAX_BOXES boxes touch it.  Any conductor-free cube gives a valid
// transition, so the halving changes which cube is used, not what the
// estimator converges to; the option reproduces it so that single walks can
// be compared with the kernel's one by one.  Returns R <= 0 when no halving
// helps.
double cube_half_size(const Structure& S, const double c[3], double R, bool kernel_limits) {
    if (!kernel_limits) return R;
    for (int it = 0; it < 40; ++it) {
        if (boxes_touching(S, c, R) <= MAX_BOXES) return R;
        R *= 0.5;
    }
    return -1.0;
}

// Conductors holding part of the open cube (c-R, c+R), the cube clipped to
// the window at symmetry walls.
int conductors_touching(const Structure& S, const double c[3], double R) {
    int cnt = 0;
    for (const Box& b : S.cond) {
        bool touch = true;
        for (int a = 0; a < 3; ++a) {
            double lo = c[a] - R, hi = c[a] + R;
            if (S.bc[2 * a] == 1) lo = std::max(lo, S.wlo[a]);
            if (S.bc[2 * a + 1] == 1) hi = std::min(hi, S.whi[a]);
            if (!(b.lo[a] < hi && b.hi[a] > lo)) touch = false;
        }
        cnt += touch;
    }
    return cnt;
}

// Expanded-cube size rule of MicroWalk-E (reading; Sec. III-B fixes the
// expansion factor, 5x, and says the lattice is adjusted to the conductors):
// the half-size is n d / (2 m) with m = max(1, round(n / (2 E))), so that the
// nearest conductor face or grounded face, at L-infinity distance d, lies on
// a node plane (m nodes from the centre); it stops at symmetry walls (no
// larger than the distance from c to any symmetry wall, so no node needs
// folding), and is never below d.
//
// kernel_limits (test option): the GPU kernel also halves the cube, not below
// d, while more than MAX_BOXES dielectric boxes or MAX_EXP_COND conductors
// touch it (the widths of its per-cube bit masks), and applies the ordinary
// rule once it is back at d.  Returns the half-size (<= 0: no valid cube).
const int MAX_EXP_COND = 7;  // conductors inside one expanded cube (kernel_limits)

double expanded_half_size(const Structure& S, const double c[3], double d, double E, int n, bool kernel_limits) {
    const int m = std::max(1, (int)std::lround(n / (2.0 * E)));
    double R = n * d / (2.0 * m);
    for (int a = 0; a < 3; ++a) {
        if (S.bc[2 * a] == 1) R = std::min(R, c[a] - S.wlo[a]);
        if (S.bc[2 * a + 1] == 1) R = std::min(R, S.whi[a] - c[a]);
    }
    R = std::max(R, d);
    if (!kernel_limits) return R;
    for (int it = 0; it < 64 && R > d; ++it) {
        if (boxes_touching(S, c, R) <= MAX_BOXES && conductors_touching(S, c, R) <= MAX_EXP_COND) return R;
        R = std::max(0.5 * R, d);
    }
    return cube_half_size(S, c, d, true);
}

// Mirror folding of a coordinate at Neumann window faces.
double fold(const Structure& S, int a, double x) {
    for (int it = 0; it < 64; ++it) {
        if (x < S.wlo[a] && S.bc[2 * a] == 1)
            x = 2 * S.wlo[a] - x;
        else if (x > S.whi[a] && S.bc[2 * a + 1] == 1)
            x = 2 * S.whi[a] - x;
        else
            break;
    }
    return x;
}

// Permittivity at a point (after folding): the last dielectric box that
// contains it (half-open), else the background layer that contains z.
float eps_at(const Structure& S, const double p[3]) {
    for (int b = (int)S.diel.size() - 1; b >= 0; --b) {
        const Box& B = S.diel[b];
        if (p[0] >= B.lo[0] && p[0] < B.hi[0] && p[1] >= B.lo[1] && p[1] < B.hi[1] && p[2] >= B.lo[2] &&
            p[2] < B.hi[2])
            return B.eps;
    }
    int L = (int)S.layer_z0.size();
    int l = 0;
    for (int q = 1; q < L; ++q)
        if (p[2] >= S.layer_z0[q]) l = q;
    return S.layer_eps[l];
}

// A voxelised transition cube: n^3 cells of size h around centre c.  Cell
// (i,j,k) takes the permittivity at its centre (reading of "constant
// permittivity per voxel", Sec. III-A).
struct Cube {
    int n;
    double c[3], R, h;
    std::vector<uint64_t> e;  // vertex cell codes
    std::vector<float> ep;    // cell permittivities (the cell lattice's Eq. 6 uses them)
    int cls;                  // 0 uniform, 1 stratified, 2 non-stratified
    int axis;                 // stratification axis (0..2) when cls <= 1
    uint8_t full[3];          // per axis: every present region spans all cells
};

double cell_centre(const Cube& C, int a, int i) { return C.c[a] - C.R + (i + 0.5) * C.h; }

// Region-level stratification (reading of "stratified dielectrics",
// Sec. II-B/III-C): the regions are the dielectric boxes and background
// layers.  A region is present in the cube when it contains at least one cell
// centre.  The cube is stratified along axis s when every present region
// contains whole planes normal to s, and uniform when every present region
// contains the whole cube.  Regions are axis-aligned, so their cell sets are
// products of per-axis index sets; the test uses those counts.
void build_cube(const Structure& S, const double c[3], double R, int n, Cube& C) {
    C.n = n;
    for (int a = 0; a < 3; ++a) C.c[a] = c[a];
    C.R = R;
    C.h = 2 * R / n;
    C.e.assign((size_t)n * n * n, 0);
    C.ep.assign((size_t)n * n * n, 0.f);
    std::vector<double> f[3];
    for (int a = 0; a < 3; ++a) {
        f[a].resize(n);
        for (int i = 0; i < n; ++i) f[a][i] = fold(S, a, cell_centre(C, a, i));
    }
    for (int k = 0; k < n; ++k)
        for (int j = 0; j < n; ++j)
            for (int i = 0; i < n; ++i) {
                double p[3] = {f[0][i], f[1][j], f[2][k]};
                const float ev = eps_at(S, p);
                C.e[((size_t)k * n + j) * n + i] = vertex_cell_code(ev);
                C.ep[((size_t)k * n + j) * n + i] = ev;
            }
    // per-region per-axis membership counts
    bool full_axis[3] = {true, true, true};
    auto account = [&](const double lo[3], const double hi[3]) {
        int cnt[3];
        for (int a = 0; a < 3; ++a) {
            cnt[a] = 0;
            for (int i = 0; i < n; ++i)
                if (f[a][i] >= lo[a] && f[a][i] < hi[a]) ++cnt[a];
        }
        if (cnt[0] == 0 || cnt[1] == 0 || cnt[2] == 0) return;  // not present
        for (int a = 0; a < 3; ++a)
            if (cnt[a] != n) full_axis[a] = false;
    };
    for (const Box& B : S.diel) account(B.lo, B.hi);
    int L = (int)S.layer_z0.size();
    for (int l = 0; l < L; ++l) {
        double lo[3] = {-INFINITY, -INFINITY, l == 0 ? -INFINITY : S.layer_z0[l]};
        double hi[3] = {INFINITY, INFINITY, l + 1 < L ? S.layer_z0[l + 1] : INFINITY};
        account(lo, hi);
    }
    for (int a = 0; a < 3; ++a) C.full[a] = full_axis[a];
    // stratified along s <=> regions full along both other axes
    auto strat = [&](int s) { return full_axis[(s + 1) % 3] && full_axis[(s + 2) % 3]; };
    if (full_axis[0] && full_axis[1] && full_axis[2]) {
        C.cls = 0;
        C.axis = 2;
    } else if (strat(2)) {
        C.cls = 1;
        C.axis = 2;
    } else if (strat(0)) {
        C.cls = 1;
        C.axis = 0;
    } else if (strat(1)) {
        C.cls = 1;
        C.axis = 1;
    } else {
        C.cls = 2;
        C.axis = -1;
    }
}

// Absorbing interior nodes of an expanded cube (MicroWalk-E): a node at or
// beyond a grounded window face belongs to the enclosure (net n_nets); else,
// after folding at symmetry walls, a node inside or on a conductor box takes
// that conductor's net (the first such box).  Boundary nodes stay free: the
// next hop's distance test absorbs a walk that stops inside a conductor.
std::vector<int32_t> absorbing_nodes(const Structure& S, const Cube& C) {
    const int n = C.n;
    std::vector<int32_t> ab((size_t)(n + 1) * (n + 1) * (n + 1), -1);
    for (int k = 1; k < n; ++k)
        for (int j = 1; j < n; ++j)
            for (int i = 1; i < n; ++i) {
                const int q[3] = {i, j, k};
                double p[3];
                int net = -1;
                for (int a = 0; a < 3; ++a) {
                    const double x = C.c[a] - C.R + q[a] * C.h;
                    if ((S.bc[2 * a] == 0 && x <= S.wlo[a]) || (S.bc[2 * a + 1] == 0 && x >= S.whi[a])) net = S.n_nets;
                    p[a] = fold(S, a, x);
                }
                if (net < 0)
                    for (const Box& b : S.cond)
                        if (p[0] >= b.lo[0] && p[0] <= b.hi[0] && p[1] >= b.lo[1] && p[1] <= b.hi[1] &&
                            p[2] >= b.lo[2] && p[2] <= b.hi[2]) {
                            net = b.net;
                            break;
                        }
                ab[((size_t)k * (n + 1) + j) * (n + 1) + i] = net;
            }
    return ab;
}

// Fraction theta in (0, 1] of the link from node p in direction d at which
// the segment enters a conductor or reaches a grounded face (bisection).
struct ThetaCtx {
    const Structure* S;
    const Cube* C;
};
bool absorbing_point(const Structure& S, const double x[3]) {
    double p[3];
    for (int a = 0; a < 3; ++a) {
        if ((S.bc[2 * a] == 0 && x[a] <= S.wlo[a]) || (S.bc[2 * a + 1] == 0 && x[a] >= S.whi[a])) return true;
        p[a] = fold(S, a, x[a]);
    }
    for (const Box& b : S.cond)
        if (p[0] >= b.lo[0] && p[0] <= b.hi[0] && p[1] >= b.lo[1] && p[1] <= b.hi[1] && p[2] >= b.lo[2] &&
            p[2] <= b.hi[2])
            return true;
    return false;
}
double link_theta(const void* vctx, const int q[3], int d) {
    const ThetaCtx& T = *(const ThetaCtx*)vctx;
    double lo = 0.0, hi = 1.0;
    for (int it = 0; it < 40; ++it) {
        const double mid = 0.5 * (lo + hi);
        double x[3];
        for (int a = 0; a < 3; ++a) x[a] = T.C->c[a] - T.C->R + (q[a] + mid * DIR[d][a]) * T.C->h;
        if (absorbing_point(*T.S, x))
            hi = mid;
        else
            lo = mid;
    }
    return std::max(hi, 1.0 / 16.0);
}

bool stratified_along(const Cube& C, int s) {
    if (C.cls == 0) return true;
    return C.full[(s + 1) % 3] && C.full[(s + 2) % 3];
}

// Codes of the planes normal to s of a stratified cube (cell with other
// coordinates 0 represents its plane).
std::vector<uint64_t> plane_codes(const Cube& C, int s) {
    int n = C.n;
    std::vector<uint64_t> seq(n);
    for (int p = 0; p < n; ++p) {
        int q[3] = {0, 0, 0};
        q[s] = p;
        seq[p] = C.e[((size_t)q[2] * n + q[1]) * n + q[0]];
    }
    return seq;
}

// "Homogenize" branch of the first-transition treatment (Fig. 4, Table II
// note a): each plane normal to a takes the mean code of its n^2 cells,
// rounded half to even.
std::vector<uint64_t> homogenised_codes(const Cube& C, int a) {
    int n = C.n;
    std::vector<uint64_t> seq(n);
    uint64_t area = (uint64_t)n * n;
    for (int p = 0; p < n; ++p) {
        uint64_t sum = 0;
        for (int u = 0; u < n; ++u)
            for (int v = 0; v < n; ++v) {
                int q[3];
                q[a] = p;
                q[(a + 1) % 3] = u;
                q[(a + 2) % 3] = v;
                sum += C.e[((size_t)q[2] * n + q[1]) * n + q[0]];
            }
        uint64_t qt = sum / area, rem = sum % area;
        if (2 * rem > area || (2 * rem == area && (qt & 1))) ++qt;
        seq[p] = qt;
    }
    return seq;
}

// Cell lattice: a plane is described by its permittivity (the float's bit
// pattern), since Eq. (6) combines permittivities, not codes.
uint64_t float_bits(float f) {
    uint32_t u;
    std::memcpy(&u, &f, 4);
    return u;
}
float bits_float(uint64_t b) {
    const uint32_t u = (uint32_t)b;
    float f;
    std::memcpy(&f, &u, 4);
    return f;
}

std::vector<uint64_t> plane_eps(const Cube& C, int s) {
    int n = C.n;
    std::vector<uint64_t> seq(n);
    for (int p = 0; p < n; ++p) {
        int q[3] = {0, 0, 0};
        q[s] = p;
        seq[p] = float_bits(C.ep[((size_t)q[2] * n + q[1]) * n + q[0]]);
    }
    return seq;
}

// Homogenised first cube on the cell lattice: each plane normal to a takes
// the mean permittivity of its n^2 cells, rounded to float.  The binary64 sum
// is exact in any order (at most 2^10 cells of permittivity in [1e-3, 1e3]).
std::vector<uint64_t> homogenised_eps(const Cube& C, int a) {
    int n = C.n;
    std::vector<uint64_t> seq(n);
    for (int p = 0; p < n; ++p) {
        double sum = 0;
        for (int u = 0; u < n; ++u)
            for (int v = 0; v < n; ++v) {
                int q[3];
                q[a] = p;
                q[(a + 1) % 3] = u;
                q[(a + 2) % 3] = v;
                sum += (double)C.ep[((size_t)q[2] * n + q[1]) * n + q[0]];
            }
        seq[p] = float_bits((float)(sum / (double)(n * n)));
    }
    return seq;
}

std::vector<float> expand_layers_eps(const std::vector<uint64_t>& seq, int s, int n) {
    std::vector<float> e((size_t)n * n * n);
    for (int k = 0; k < n; ++k)
        for (int j = 0; j < n; ++j)
            for (int i = 0; i < n; ++i) {
                int q[3] = {i, j, k};
                e[((size_t)k * n + j) * n + i] = bits_float(seq[q[s]]);
            }
    return e;
}

// Face conductance of the link between two cells of the cell lattice, in
// permittivity units: the series (harmonic) combination over its two halves,
// the conductance behind Eq. (6).
double cell_face_eps(float a, float b) { return 2.0 * (double)a * (double)b / ((double)a + (double)b); }

std::vector<uint64_t> expand_layers(const std::vector<uint64_t>& seq, int s, int n) {
    std::vector<uint64_t> e((size_t)n * n * n);
    for (int k = 0; k < n; ++k)
        for (int j = 0; j < n; ++j)
            for (int i = 0; i < n; ++i) {
                int q[3] = {i, j, k};
                e[((size_t)k * n + j) * n + i] = seq[q[s]];
            }
    return e;
}

// ---------------------------------------------------------------------------
// SGF tables of stratified cubes ("analytical path" of the hybrid strategy,
// Sec. III-C).  The paper's AGF formulas are not part of the paper; the
// oracle uses the exact discrete SGF of the same lattice, which Theorem 1
// makes identical in distribution to MicroWalk on that cube.
// ---------------------------------------------------------------------------
struct HopTable {
    std::vector<double> P;  // 6 M^2
};

struct FirstTable {
    std::vector<double> Pc, Pp, Pm;  // sources c, c + e_a, c - e_a
    double Gp, Gm;                   // link conductances of c along +a, -a (eps units)
};

struct TableCache {
    std::mutex mu;
    std::map<std::vector<uint64_t>, std::shared_ptr<HopTable>> hop;
    std::map<std::vector<uint64_t>, std::shared_ptr<FirstTable>> first;
    std::atomic<uint64_t> misses{0};
};

std::shared_ptr<HopTable> hop_table(TableCache& TC, int lattice, int n, int s, const std::vector<uint64_t>& seq) {
    std::vector<uint64_t> key;
    key.push_back((uint64_t)lattice);
    key.push_back((uint64_t)n);
    key.push_back((uint64_t)s);
    key.insert(key.end(), seq.begin(), seq.end());
    {
        std::lock_guard<std::mutex> g(TC.mu);
        auto it = TC.hop.find(key);
        if (it != TC.hop.end()) return it->second;
    }
    auto T = std::make_shared<HopTable>();
    if (lattice == 1) {
        // cell lattice: the walk starts in the centre cell
        const CellSystem CS = build_cell_system(expand_layers_eps(seq, s, n), n);
        int src[3] = {(n - 1) / 2, (n - 1) / 2, (n - 1) / 2};
        if (!sgf_cell(CS, src, T->P, nullptr)) return nullptr;
    } else {
        auto e = expand_layers(seq, s, n);
        VertexSystem VS = build_vertex_system(e, n);
        int src[3] = {n / 2, n / 2, n / 2};
        if (!sgf_vertex(VS, src, T->P, nullptr)) return nullptr;
    }
    TC.misses++;
    std::lock_guard<std::mutex> g(TC.mu);
    TC.hop[key] = T;
    return T;
}

std::shared_ptr<FirstTable> first_table(TableCache& TC, int lattice, int n, int s, int a,
                                        const std::vector<uint64_t>& seq) {
    std::vector<uint64_t> key;
    key.push_back((uint64_t)lattice);
    key.push_back((uint64_t)n);
    key.push_back((uint64_t)s);
    key.push_back((uint64_t)a);
    key.insert(key.end(), seq.begin(), seq.end());
    {
        std::lock_guard<std::mutex> g(TC.mu);
        auto it = TC.first.find(key);
        if (it != TC.first.end()) return it->second;
    }
    auto T = std::make_shared<FirstTable>();
    if (lattice == 1) {
        // cell lattice: sources at the centre cell and its two neighbours
        // along a; G+-, the face conductances between them
        const std::vector<float> ep = expand_layers_eps(seq, s, n);
        const CellSystem CS = build_cell_system(ep, n);
        const int h0 = (n - 1) / 2;
        int c[3] = {h0, h0, h0};
        int cp[3] = {h0, h0, h0}, cm[3] = {h0, h0, h0};
        cp[a] += 1;
        cm[a] -= 1;
        if (!sgf_cell(CS, c, T->Pc, nullptr)) return nullptr;
        if (!sgf_cell(CS, cp, T->Pp, nullptr)) return nullptr;
        if (!sgf_cell(CS, cm, T->Pm, nullptr)) return nullptr;
        auto at = [&](const int q[3]) { return ep[((size_t)q[2] * n + q[1]) * n + q[0]]; };
        T->Gp = cell_face_eps(at(c), at(cp));
        T->Gm = cell_face_eps(at(c), at(cm));
        TC.misses++;
        std::lock_guard<std::mutex> g(TC.mu);
        TC.first[key] = T;
        return T;
    }
    auto e = expand_layers(seq, s, n);
    VertexSystem VS = build_vertex_system(e, n);
    int c[3] = {n / 2, n / 2, n / 2};
    int cp[3] = {c[0], c[1], c[2]}, cm[3] = {c[0], c[1], c[2]};
    cp[a] += 1;
    cm[a] -= 1;
    if (!sgf_vertex(VS, c, T->Pc, nullptr)) return nullptr;
    if (!sgf_vertex(VS, cp, T->Pp, nullptr)) return nullptr;
    if (!sgf_vertex(VS, cm, T->Pm, nullptr)) return nullptr;
    T->Gp = (double)vertex_link(e, n, c[0], c[1], c[2], 2 * a + 1) / (4.0 * 65536.0);
    T->Gm = (double)vertex_link(e, n, c[0], c[1], c[2], 2 * a) / (4.0 * 65536.0);
    TC.misses++;
    std::lock_guard<std::mutex> g(TC.mu);
    TC.first[key] = T;
    return T;
}

// Inverse-CDF sample of index b with probability weights[b] / sum.
int sample_index(const std::vector<double>& wts, double total, uint32_t u) {
    double x = u01(u) * total;
    double cum = 0;
    int last = -1;
    for (size_t b = 0; b < wts.size(); ++b) {
        if (wts[b] <= 0) continue;
        cum += wts[b];
        last = (int)b;
        if (x < cum) return (int)b;
    }
    return last;
}

// ---------------------------------------------------------------------------
// Gaussian surface (Alg. 1 input G).  Reading: every box of the master net is
// grown by g on all sides, g = half the smallest L-infinity gap between a box
// of the net and a box of any other net or a grounded window face; G is the
// boundary of the union of the grown boxes, restricted to the window (pieces
// lying outside it or on a symmetry wall carry no flux and are dropped; kept
// pieces are clipped to the window).  With one box this is the six faces of
// the grown box.  The boundary is found by cutting each grown face along every
// coordinate at which some grown box (or the window) starts or ends and
// testing the centre of every resulting rectangle: it is on the boundary when
// a point just outside it lies in no grown box.  Two coplanar faces with the
// same outward normal can both cover a rectangle; it is counted once, for the
// box that comes first in the input.
// ---------------------------------------------------------------------------
struct GFace {
    int axis, side;
    double plane;
    double lo[3], hi[3];
    double area;
};

// Importance-sampling patch of G (reading of the importance sampling of
// Alg. 1's first transition, applied to the Gaussian-surface point): a
// rectangle of a face, its area, its weight q = area x K(centre) (K the
// first-transition kernel sum at the patch centre) and the weight factor
// Q area / q (Q = sum of q) that keeps the estimator unbiased.
struct GPatch {
    int face;
    double lo[3], hi[3];
    double area, q, factor;
};

struct Gauss {
    double g;
    std::vector<GFace> faces;
    double area;
    std::vector<GPatch> patches;  // empty: uniform-area sampling
    double Q = 0;
};

static bool in_grown_open(const Box& b, double g, const double x[3]) {
    for (int a = 0; a < 3; ++a)
        if (!(x[a] > b.lo[a] - g && x[a] < b.hi[a] + g)) return false;
    return true;
}

bool build_gauss(const Structure& S, int master, Gauss& G) {
    std::vector<const Box*> M;
    for (const Box& b : S.cond)
        if (b.net == master) M.push_back(&b);
    if (M.empty()) return false;
    double g0 = INFINITY;
    for (const Box* m : M) {
        for (const Box& b : S.cond) {
            if (b.net == master) continue;
            double gap = 0;
            for (int a = 0; a < 3; ++a) gap = std::max(gap, std::max(b.lo[a] - m->hi[a], m->lo[a] - b.hi[a]));
            g0 = std::min(g0, gap);
        }
        for (int a = 0; a < 3; ++a) {
            if (S.bc[2 * a] == 0) g0 = std::min(g0, m->lo[a] - S.wlo[a]);
            if (S.bc[2 * a + 1] == 0) g0 = std::min(g0, S.whi[a] - m->hi[a]);
        }
    }
    if (!(g0 > 0) || !std::isfinite(g0)) return false;
    const double g = g0 / 2;
    G.g = g;
    G.faces.clear();
    G.area = 0;
    // every coordinate at which a grown box or the window starts or ends
    std::vector<double> cuts[3];
    for (int a = 0; a < 3; ++a) {
        cuts[a].push_back(S.wlo[a]);
        cuts[a].push_back(S.whi[a]);
        for (const Box* m : M) {
            cuts[a].push_back(m->lo[a] - g);
            cuts[a].push_back(m->hi[a] + g);
        }
        std::sort(cuts[a].begin(), cuts[a].end());
        cuts[a].erase(std::unique(cuts[a].begin(), cuts[a].end()), cuts[a].end());
    }
    for (size_t i = 0; i < M.size(); ++i)
        for (int a = 0; a < 3; ++a)
            for (int side = 0; side < 2; ++side) {
                const double plane = side ? M[i]->hi[a] + g : M[i]->lo[a] - g;
                if (!(plane > S.wlo[a] && plane < S.whi[a])) continue;
                const int t0 = (a + 1) % 3, t1 = (a + 2) % 3;
                const int ta = std::min(t0, t1), tb = std::max(t0, t1);
                const double elo[2] = {std::max(M[i]->lo[ta] - g, S.wlo[ta]), std::max(M[i]->lo[tb] - g, S.wlo[tb])};
                const double ehi[2] = {std::min(M[i]->hi[ta] + g, S.whi[ta]), std::min(M[i]->hi[tb] + g, S.whi[tb])};
                const double eta = 1e-9 * (S.whi[a] - S.wlo[a]);
                for (size_t u = 0; u + 1 < cuts[ta].size(); ++u) {
                    const double u0 = cuts[ta][u], u1 = cuts[ta][u + 1];
                    if (u0 < elo[0] || u1 > ehi[0]) continue;
                    for (size_t v = 0; v + 1 < cuts[tb].size(); ++v) {
                        const double v0 = cuts[tb][v], v1 = cuts[tb][v + 1];
                        if (v0 < elo[1] || v1 > ehi[1]) continue;
                        double out[3];
                        out[a] = plane + (side ? eta : -eta);
                        out[ta] = 0.5 * (u0 + u1);
                        out[tb] = 0.5 * (v0 + v1);
                        bool covered = false;
                        for (const Box* m : M) covered = covered || in_grown_open(*m, g, out);
                        if (covered) continue;
                        bool counted = false;
                        for (size_t j = 0; j < i; ++j) {
                            const double pj = side ? M[j]->hi[a] + g : M[j]->lo[a] - g;
                            if (pj == plane && out[ta] > M[j]->lo[ta] - g && out[ta] < M[j]->hi[ta] + g &&
                                out[tb] > M[j]->lo[tb] - g && out[tb] < M[j]->hi[tb] + g)
                                counted = true;
                        }
                        if (counted) continue;
                        GFace F;
                        F.axis = a;
                        F.side = side;
                        F.plane = plane;
                        F.lo[a] = F.hi[a] = plane;
                        F.lo[ta] = u0;
                        F.hi[ta] = u1;
                        F.lo[tb] = v0;
                        F.hi[tb] = v1;
                        F.area = (u1 - u0) * (v1 - v0);
                        G.faces.push_back(F);
                        G.area += F.area;
                    }
                }
            }
    return !G.faces.empty();
}

// ---------------------------------------------------------------------------
// One walk of Alg. 1: Gaussian-surface sample, first transition with weight,
// transitions until absorption.  Returns the net (n_nets = env) and omega.
// ---------------------------------------------------------------------------
struct WalkStats {
    uint64_t hops = 0, micro_steps = 0, hop_class[3] = {0, 0, 0}, first_branch[4] = {0, 0, 0, 0};
    uint64_t env = 0, hop_cap = 0;
};

struct FrwParams {
    int n;
    int hybrid;
    double delta_abs;
    uint64_t seed;
    double expand = 1.0;  // MicroWalk-E expansion factor (1: plain MicroWalk)
    bool kernel_limits = false;  // reproduce the GPU kernel's cube halving (tests only)
    int lattice = 0;             // 0 vertex lattice, 1 cell-centred lattice (n odd)
};

// Exit point of hit index b of cube C: a boundary node of the vertex
// lattice, or the centre of a boundary panel of the cell lattice.
void exit_point(const Cube& C, int lattice, int b, double x[3]) {
    const int n = C.n;
    if (lattice == 1) {
        const int f = b / (n * n), rem = b % (n * n);
        const int ax = f / 2, side = f % 2;
        const int o0 = ax == 0 ? 1 : 0, o1 = ax == 2 ? 1 : 2;
        x[ax] = C.c[ax] + (side ? C.R : -C.R);
        x[o0] = C.c[o0] - C.R + (rem % n + 0.5) * C.h;
        x[o1] = C.c[o1] - C.R + (rem / n + 0.5) * C.h;
        return;
    }
    int node[3];
    vertex_node_of_hit(n, b, node);
    for (int q = 0; q < 3; ++q) x[q] = C.c[q] - C.R + node[q] * C.h;
}

// FirstTransition(r) kernel: the first cube centred at r on face F of G (it
// touches the master), its branch (Fig. 4 reading), and the flux weights
// w_b of its boundary nodes along the outward normal (Sec. II-A: the
// normal derivative of the discrete SGF by a centred difference).  Returns
// K = sum |w_b|, or a negative value when no valid cube exists.
double first_weights(const Structure& S, const Gauss& G, const GFace& F, const double r[3], const FrwParams& P,
                     TableCache& TC, Cube& C, std::vector<double>& w, int* branch_out) {
    const int n = P.n;
    int a = F.axis;
    double R = cube_half_size(S, r, std::min(structure_dist(S, r, nullptr), G.g), P.kernel_limits);
    if (R <= 0) return -1.0;
    build_cube(S, r, R, n, C);
    int branch, s;
    std::vector<uint64_t> seq;
    const bool cell = P.lattice == 1;
    if (C.cls == 0) {
        branch = 0;
        s = a;
        seq = cell ? plane_eps(C, a) : plane_codes(C, a);
    } else if (stratified_along(C, a)) {
        branch = 1;
        s = a;
        seq = cell ? plane_eps(C, a) : plane_codes(C, a);
    } else if (C.cls == 1) {
        branch = 2;
        s = C.axis;
        seq = cell ? plane_eps(C, s) : plane_codes(C, s);
    } else {
        branch = 3;
        s = a;
        seq = cell ? homogenised_eps(C, a) : homogenised_codes(C, a);
    }
    *branch_out = branch;
    auto FT = first_table(TC, P.lattice, n, s, a, seq);
    if (!FT) return -1.0;
    // flux stencil along the outward normal
    const std::vector<double>& Pout = F.side ? FT->Pp : FT->Pm;
    const std::vector<double>& Pin = F.side ? FT->Pm : FT->Pp;
    double Gout = F.side ? FT->Gp : FT->Gm;
    double Gin = F.side ? FT->Gm : FT->Gp;
    size_t NB = FT->Pc.size();
    w.assign(NB, 0.0);
    double K = 0;
    for (size_t b = 0; b < NB; ++b) {
        w[b] = (Gout * (FT->Pc[b] - Pout[b]) + Gin * (Pin[b] - FT->Pc[b])) / (2 * C.h);
        K += std::fabs(w[b]);
    }
    return K;
}

// Importance-sampling patches of G: every rectangle cut into nu x nv equal
// patches with edges at most edge (nu = ceil(length / edge)), each weighted
// by q = area x K(patch centre).
bool build_patches(const Structure& S, Gauss& G, double edge, const FrwParams& P, TableCache& TC) {
    G.patches.clear();
    G.Q = 0;
    Cube C;
    std::vector<double> w;
    for (size_t f = 0; f < G.faces.size(); ++f) {
        const GFace& F = G.faces[f];
        const int t0 = (F.axis + 1) % 3, t1 = (F.axis + 2) % 3;
        const int ta = std::min(t0, t1), tb = std::max(t0, t1);
        const double la = F.hi[ta] - F.lo[ta], lb = F.hi[tb] - F.lo[tb];
        const int nu = std::max(1, (int)std::ceil(la / edge)), nv = std::max(1, (int)std::ceil(lb / edge));
        for (int j = 0; j < nv; ++j)
            for (int i = 0; i < nu; ++i) {
                GPatch Pt;
                Pt.face = (int)f;
                Pt.lo[F.axis] = Pt.hi[F.axis] = F.plane;
                Pt.lo[ta] = F.lo[ta] + la * i / nu;
                Pt.hi[ta] = F.lo[ta] + la * (i + 1) / nu;
                Pt.lo[tb] = F.lo[tb] + lb * j / nv;
                Pt.hi[tb] = F.lo[tb] + lb * (j + 1) / nv;
                Pt.area = (Pt.hi[ta] - Pt.lo[ta]) * (Pt.hi[tb] - Pt.lo[tb]);
                double c[3];
                for (int q = 0; q < 3; ++q) c[q] = 0.5 * (Pt.lo[q] + Pt.hi[q]);
                c[F.axis] = F.plane;
                int br;
                const double K = first_weights(S, G, F, c, P, TC, C, w, &br);
                if (!(K > 0)) return false;
                Pt.q = Pt.area * K;
                G.Q += Pt.q;
                G.patches.push_back(Pt);
            }
    }
    for (GPatch& Pt : G.patches) Pt.factor = G.Q * Pt.area / Pt.q;
    return true;
}

bool frw_walk(const Structure& S, const Gauss& G, int master, const FrwParams& P, TableCache& TC, uint64_t walk,
              int* net_out, double* omega_out, WalkStats& st) {
    int n = P.n;
    // GaussianSurfaceSampling(G): a rectangle by area (uniform on G) or, with
    // importance sampling, a patch by its weight q; then a uniform point on it
    uint32_t w0 = rng_word(P.seed, 0, walk, PURPOSE_GAUSS, 0);
    uint32_t w1 = rng_word(P.seed, 0, walk, PURPOSE_GAUSS, 1);
    uint32_t w2 = rng_word(P.seed, 0, walk, PURPOSE_GAUSS, 2);
    const bool is = !G.patches.empty();
    const size_t cnt = is ? G.patches.size() : G.faces.size();
    double xa = u01(w0) * (is ? G.Q : G.area), cum = 0;
    size_t fi = cnt - 1;
    for (size_t f = 0; f < cnt; ++f) {
        cum += is ? G.patches[f].q : G.faces[f].area;
        if (xa < cum) {
            fi = f;
            break;
        }
    }
    const GFace& F = G.faces[is ? G.patches[fi].face : fi];
    const double* lo = is ? G.patches[fi].lo : F.lo;
    const double* hi = is ? G.patches[fi].hi : F.hi;
    const double factor = is ? G.patches[fi].factor : G.area;
    double r[3];
    int t0 = (F.axis + 1) % 3, t1 = (F.axis + 2) % 3;
    int ta = std::min(t0, t1), tb = std::max(t0, t1);
    r[F.axis] = F.plane;
    r[ta] = lo[ta] + u01(w1) * (hi[ta] - lo[ta]);
    r[tb] = lo[tb] + u01(w2) * (hi[tb] - lo[tb]);

    // FirstTransition(r): cube centred on G touching the master; the next
    // point b ~ |w_b| / K, weight eps0 K sign(w_b) times |G| (uniform) or
    // the patch factor Q area / q (importance sampling).
    Cube C;
    std::vector<double> w;
    int branch;
    const double K = first_weights(S, G, F, r, P, TC, C, w, &branch);
    if (!(K > 0)) return false;
    st.first_branch[branch]++;
    std::vector<double> aw(w.size());
    for (size_t b = 0; b < w.size(); ++b) aw[b] = std::fabs(w[b]);
    int b = sample_index(aw, K, rng_word(P.seed, 0, walk, PURPOSE_FIRST, 0));
    double omega = EPS0 * factor * K * (w[b] > 0 ? 1.0 : -1.0);
    // The walker's position is folded back into the window at symmetry
    // walls: by mirror symmetry the folded point has the same potential.
    double x[3], xe[3];
    exit_point(C, P.lattice, b, xe);
    for (int q = 0; q < 3; ++q) x[q] = fold(S, q, xe[q]);

    // Transition loop.
    for (uint32_t t = 1;; ++t) {
        int nearest;
        double d = structure_dist(S, x, &nearest);
        if (d <= P.delta_abs) {
            *net_out = nearest;
            *omega_out = omega;
            if (nearest == S.n_nets) st.env++;
            return true;
        }
        if ((int)t > HOP_CAP) {
            st.hop_cap++;
            *net_out = S.n_nets;
            *omega_out = omega;
            return true;
        }
        st.hops++;
        const double Rh = cube_half_size(S, x, d, P.kernel_limits);
        if (Rh <= 0) return false;
        build_cube(S, x, Rh, n, C);
        st.hop_class[C.cls]++;
        int hb;
        if (P.hybrid && C.cls <= 1) {
            auto HT = hop_table(TC, P.lattice, n, C.axis,
                                P.lattice == 1 ? plane_eps(C, C.axis) : plane_codes(C, C.axis));
            if (!HT) return false;
            hb = sample_index(HT->P, 1.0, rng_word(P.seed, t, walk, PURPOSE_TABLE, 0));
        } else if (P.expand > 1.0) {
            // MicroWalk-E: the transition cube grows to E times the
            // conductor-free size and may hold conductors (Sec. III-B)
            const double Re = expanded_half_size(S, x, d, P.expand, n, P.kernel_limits);
            if (Re <= 0) return false;
            build_cube(S, x, Re, n, C);
            const std::vector<int32_t> ab = absorbing_nodes(S, C);
            int32_t steps = 0;
            int net = -1;
            ThetaCtx TCx{&S, &C};
            hb = microwalk_vertex_e(C.e, ab, n, P.seed, t, walk, &steps, &net, link_theta, &TCx);
            st.micro_steps += (uint64_t)steps;
            if (hb == -2) {
                *net_out = net;
                *omega_out = omega;
                if (net == S.n_nets) st.env++;
                return true;
            }
            if (hb < 0) return false;
        } else if (P.lattice == 1) {
            // Alg. 3 on the cell-centred lattice from the centre cell
            int32_t steps = 0;
            hb = microwalk_cell(C.ep.data(), n, P.seed, t, walk, &steps);
            st.micro_steps += (uint64_t)steps;
            if (hb < 0) return false;
        } else {
            int start[3] = {n / 2, n / 2, n / 2};
            int32_t steps = 0;
            hb = microwalk_vertex(C.e, n, start, P.seed, t, walk, &steps, nullptr);
            st.micro_steps += (uint64_t)steps;
            if (hb < 0) return false;
        }
        exit_point(C, P.lattice, hb, xe);
        for (int q = 0; q < 3; ++q) x[q] = fold(S, q, xe[q]);
    }
}

Structure make_structure(const double* cond, int n_cond, int n_nets, const double* diel, int n_diel,
                         const double* layer_z0, const double* layer_eps, int n_layers, const double* win,
                         const int32_t* bc) {
    Structure S;
    for (int i = 0; i < n_cond; ++i) {
        Box b;
        for (int a = 0; a < 3; ++a) {
            b.lo[a] = cond[i * 7 + a];
            b.hi[a] = cond[i * 7 + 3 + a];
        }
        b.net = (int)cond[i * 7 + 6];
        b.eps = 0;
        S.cond.push_back(b);
    }
    S.n_nets = n_nets;
    for (int i = 0; i < n_diel; ++i) {
        Box b;
        for (int a = 0; a < 3; ++a) {
            b.lo[a] = diel[i * 7 + a];
            b.hi[a] = diel[i * 7 + 3 + a];
        }
        b.net = -1;
        b.eps = (float)diel[i * 7 + 6];
        S.diel.push_back(b);
    }
    for (int l = 0; l < n_layers; ++l) {
        S.layer_z0.push_back(layer_z0[l]);
        S.layer_eps.push_back((float)layer_eps[l]);
    }
    for (int a = 0; a < 3; ++a) {
        S.wlo[a] = win[a];
        S.whi[a] = win[3 + a];
    }
    for (int f = 0; f < 6; ++f) S.bc[f] = bc[f];
    return S;
}

}  // namespace

// ---------------------------------------------------------------------------
// C interface (ctypes).  Return 0 on success, negative on failure.
// ---------------------------------------------------------------------------
extern "C" {

int mwo_philox4x32_10(const uint32_t* ctr, const uint32_t* key, uint32_t* out) {
    philox4x32_10(ctr, key, out);
    return 0;
}

int mwo_rng_words(uint64_t seed, uint32_t c1, uint64_t walk, uint32_t purpose, uint64_t s0, int64_t count,
                  uint32_t* out) {
    for (int64_t i = 0; i < count; ++i) out[i] = rng_word(seed, c1, walk, purpose, s0 + (uint64_t)i);
    return 0;
}

// Vertex lattice cell codes rint(eps * 2^16).
int mwo_vertex_codes(const float* eps, int64_t count, uint64_t* codes) {
    for (int64_t i = 0; i < count; ++i) codes[i] = vertex_cell_code(eps[i]);
    return 0;
}

// Link codes (6 per interior node, node order ((k-1)M+(j-1))M+(i-1)) and
// thresholds (5 per node) of the vertex lattice.
int mwo_vertex_thresholds(const float* eps, int n, uint64_t* links, uint32_t* T) {
    if (n < 2 || n % 2) return -1;
    std::vector<uint64_t> e((size_t)n * n * n);
    for (size_t i = 0; i < e.size(); ++i) e[i] = vertex_cell_code(eps[i]);
    int M = n - 1;
    for (int k = 1; k < n; ++k)
        for (int j = 1; j < n; ++j)
            for (int i = 1; i < n; ++i) {
                size_t v = ((size_t)(k - 1) * M + (j - 1)) * M + (i - 1);
                uint64_t g[6];
                for (int d = 0; d < 6; ++d) g[d] = vertex_link(e, n, i, j, k, d);
                if (links)
                    for (int d = 0; d < 6; ++d) links[v * 6 + d] = g[d];
                if (T) thresholds_from_codes(g, T + v * 5);
            }
    return 0;
}

// Link codes and thresholds of the cell lattice (Eq. 6), node order
// (k*N+j)*N+i.
int mwo_cell_thresholds(const float* eps, int N, uint64_t* links, uint32_t* T) {
    if (N < 1 || N % 2 == 0) return -1;
    auto EPS = [&](int x, int y, int z) { return eps[((size_t)z * N + y) * N + x]; };
    for (int k = 0; k < N; ++k)
        for (int j = 0; j < N; ++j)
            for (int i = 0; i < N; ++i) {
                size_t v = ((size_t)k * N + j) * N + i;
                uint64_t g[6];
                for (int d = 0; d < 6; ++d) {
                    int q[3] = {i + DIR[d][0], j + DIR[d][1], k + DIR[d][2]};
                    bool inside = q[0] >= 0 && q[0] < N && q[1] >= 0 && q[1] < N && q[2] >= 0 && q[2] < N;
                    g[d] = inside ? cell_link_code(EPS(q[0], q[1], q[2]), EPS(i, j, k)) : (1ull << 24);
                }
                if (links)
                    for (int d = 0; d < 6; ++d) links[v * 6 + d] = g[d];
                if (T) thresholds_from_codes(g, T + v * 5);
            }
    return 0;
}

int mwo_choose_direction(uint32_t u, const uint32_t* T) { return choose_direction(u, T); }

// Alg. 3, n_walks walks with ids first_walk.. on one cube.
int mwo_microwalk(const float* eps, int n, int lattice, uint64_t n_walks, uint64_t first_walk, uint64_t seed,
                  uint32_t cube_index, int32_t* hits, int32_t* steps) {
    if (lattice == 0) {
        if (n < 2 || n % 2) return -1;
        std::vector<uint64_t> e((size_t)n * n * n);
        for (size_t i = 0; i < e.size(); ++i) e[i] = vertex_cell_code(eps[i]);
        int start[3] = {n / 2, n / 2, n / 2};
        for (uint64_t w = 0; w < n_walks; ++w) {
            int32_t st;
            hits[w] = microwalk_vertex(e, n, start, seed, cube_index, first_walk + w, &st, nullptr);
            if (steps) steps[w] = st;
        }
        return 0;
    }
    if (n < 1 || n % 2 == 0) return -1;
    for (uint64_t w = 0; w < n_walks; ++w) {
        int32_t st;
        hits[w] = microwalk_cell(eps, n, seed, cube_index, first_walk + w, &st);
        if (steps) steps[w] = st;
    }
    return 0;
}

// Exact exit distribution (Eq. 8) and E(tau) (Eq. 11) of the vertex lattice
// from interior source node src, given cell codes.
int mwo_sgf_vertex(const uint64_t* codes, int n, const int32_t* src, double* P, double* etau) {
    if (n < 2 || n % 2) return -1;
    std::vector<uint64_t> e(codes, codes + (size_t)n * n * n);
    VertexSystem VS = build_vertex_system(e, n);
    std::vector<double> Pv;
    int s[3] = {src[0], src[1], src[2]};
    if (!sgf_vertex(VS, s, Pv, etau)) return -2;
    std::copy(Pv.begin(), Pv.end(), P);
    return 0;
}

// Exact exit distribution and E(tau) of the cell-centred lattice (N odd)
// from cell src, given the N^3 cell permittivities.
int mwo_sgf_cell(const float* eps, int N, const int32_t* src, double* P, double* etau) {
    if (N < 1 || N % 2 == 0) return -1;
    const CellSystem CS = build_cell_system(std::vector<float>(eps, eps + (size_t)N * N * N), N);
    std::vector<double> Pv;
    int s[3] = {src[0], src[1], src[2]};
    if (!sgf_cell(CS, s, Pv, etau)) return -2;
    std::copy(Pv.begin(), Pv.end(), P);
    return 0;
}

// Voxelisation + classification of one transition cube of a structure.
// out_codes: n^3 vertex cell codes; out_cls: [class, axis].
int mwo_build_cube(const double* cond, int n_cond, int n_nets, const double* diel, int n_diel,
                   const double* layer_z0, const double* layer_eps, int n_layers, const double* win,
                   const int32_t* bc, const double* centre, double R, int n, uint64_t* out_codes,
                   int32_t* out_cls) {
    Structure S = make_structure(cond, n_cond, n_nets, diel, n_diel, layer_z0, layer_eps, n_layers, win, bc);
    Cube C;
    build_cube(S, centre, R, n, C);
    std::copy(C.e.begin(), C.e.end(), out_codes);
    out_cls[0] = C.cls;
    out_cls[1] = C.axis;
    return 0;
}

// MicroWalk-E (Sec. III-B) on one expanded cube of a structure: the cube
// centred at `centre` with half-size R and n cells, its absorbing nodes and
// cut links as in the FRW walk; walks first_walk.. with Philox c1 = c1.
// hits[w] = boundary hit index, or -2 when the walk was absorbed inside the
// cube (nets[w] = that net, n_nets for the grounded enclosure; else -1).
int mwo_microwalk_e_cube(const double* cond, int n_cond, int n_nets, const double* diel, int n_diel,
                         const double* layer_z0, const double* layer_eps, int n_layers, const double* win,
                         const int32_t* bc, const double* centre, double R, int n, uint64_t n_walks,
                         uint64_t first_walk, uint64_t seed, uint32_t c1, int32_t* hits, int32_t* nets,
                         int32_t* steps) {
    if (n < 2 || n % 2) return -1;
    Structure S = make_structure(cond, n_cond, n_nets, diel, n_diel, layer_z0, layer_eps, n_layers, win, bc);
    Cube C;
    build_cube(S, centre, R, n, C);
    const std::vector<int32_t> ab = absorbing_nodes(S, C);
    if (ab[((size_t)(n / 2) * (n + 1) + n / 2) * (n + 1) + n / 2] >= 0) return -2;  // centre absorbing
    ThetaCtx TCx{&S, &C};
    for (uint64_t w = 0; w < n_walks; ++w) {
        int32_t st = 0;
        int net = -1;
        hits[w] = microwalk_vertex_e(C.e, ab, n, seed, c1, first_walk + w, &st, &net, link_theta, &TCx);
        nets[w] = hits[w] == -2 ? net : -1;
        if (steps) steps[w] = st;
    }
    return 0;
}

// Transition tables of a stratified cube (plane codes seq[n] along axis s),
// as the walks use them (Sec. III-C; the exact discrete SGF, Eq. 8).
// Hop table: exit distribution P (6 M^2) from the centre node.
// lattice 1: the cell-centred lattice (n odd, 6 n^2 entries from the centre
// cell); seq then holds the planes' permittivities as float bit patterns.
int mwo_hop_table(int lattice, int n, int s, const uint64_t* seq, double* P) {
    if (lattice != 0 && lattice != 1) return -1;
    if (n < 2 || (lattice == 0 ? n % 2 != 0 : n % 2 == 0) || s < 0 || s > 2) return -1;
    TableCache TC;
    auto T = hop_table(TC, lattice, n, s, std::vector<uint64_t>(seq, seq + n));
    if (!T) return -2;
    std::copy(T->P.begin(), T->P.end(), P);
    return 0;
}

// First-transition table for normal axis a: exit distributions from the
// centre c and from c +- e_a, and the link conductances G+, G- of c along a.
int mwo_first_table(int lattice, int n, int s, int a, const uint64_t* seq, double* Pc, double* Pp, double* Pm,
                    double* Gp, double* Gm) {
    if (lattice != 0 && lattice != 1) return -1;
    if (n < 3 || (lattice == 0 ? n % 2 != 0 : n % 2 == 0) || s < 0 || s > 2 || a < 0 || a > 2) return -1;
    TableCache TC;
    auto T = first_table(TC, lattice, n, s, a, std::vector<uint64_t>(seq, seq + n));
    if (!T) return -2;
    std::copy(T->Pc.begin(), T->Pc.end(), Pc);
    std::copy(T->Pp.begin(), T->Pp.end(), Pp);
    std::copy(T->Pm.begin(), T->Pm.end(), Pm);
    *Gp = T->Gp;
    *Gm = T->Gm;
    return 0;
}

// Largest conductor-free cube query (half-size and nearest net).
int mwo_dist(const double* cond, int n_cond, int n_nets, const double* win, const int32_t* bc, const double* p,
             double* d, int32_t* nearest) {
    Structure S = make_structure(cond, n_cond, n_nets, nullptr, 0, nullptr, nullptr, 0, win, bc);
    int who;
    *d = structure_dist(S, p, &who);
    *nearest = who;
    return 0;
}

// Gaussian surface: returns g and |G|; faces as [axis, side, plane, lo3, hi3, area].
int mwo_gauss(const double* cond, int n_cond, int n_nets, const double* win, const int32_t* bc, int master,
              double* g, double* area, double* faces, int32_t cap, int32_t* n_faces) {
    Structure S = make_structure(cond, n_cond, n_nets, nullptr, 0, nullptr, nullptr, 0, win, bc);
    Gauss G;
    if (!build_gauss(S, master, G)) return -1;
    *g = G.g;
    *area = G.area;
    *n_faces = (int32_t)G.faces.size();
    if ((int32_t)G.faces.size() > cap) return -2;
    for (size_t f = 0; f < G.faces.size(); ++f) {
        double* o = faces + f * 10;
        o[0] = G.faces[f].axis;
        o[1] = G.faces[f].side;
        o[2] = G.faces[f].plane;
        for (int a = 0; a < 3; ++a) {
            o[3 + a] = G.faces[f].lo[a];
            o[6 + a] = G.faces[f].hi[a];
        }
        o[9] = G.faces[f].area;
    }
    return 0;
}

// Alg. 1 for master net `master`, walks first_walk .. first_walk+n_walks-1.
// row/se: n_nets+1 entries (last = env).  score_net/score_w: per walk (may be
// NULL).  stats: [walks, hops, micro_steps, cls0, cls1, cls2, br0..br3,
// misses, env, hop_cap] (13 entries, may be NULL).  threads >= 1 splits the
// walk range into contiguous blocks; results do not depend on it.
int mwo_frw_extract(const double* cond, int n_cond, int n_nets, const double* diel, int n_diel,
                    const double* layer_z0, const double* layer_eps, int n_layers, const double* win,
                    const int32_t* bc, int master, uint64_t n_walks, uint64_t first_walk, uint64_t seed, int n,
                    int hybrid, double abs_tol_rel, double expand, int kernel_limits, double gauss_is, int lattice,
                    int threads, double* row, double* se, int32_t* score_net, double* score_w, uint64_t* stats) {
    if (n_walks < 2 || (lattice != 0 && lattice != 1)) return -1;
    // vertex lattice: n even (a centre node); cell lattice: n odd (a centre
    // cell), plain MicroWalk only
    if (lattice == 0 ? (n < 4 || n % 2 != 0) : (n < 3 || n % 2 == 0 || expand > 1.0)) return -1;
    Structure S = make_structure(cond, n_cond, n_nets, diel, n_diel, layer_z0, layer_eps, n_layers, win, bc);
    Gauss G;
    if (!build_gauss(S, master, G)) return -2;
    double diag = 0;
    for (int a = 0; a < 3; ++a) diag += (S.whi[a] - S.wlo[a]) * (S.whi[a] - S.wlo[a]);
    FrwParams P{n, hybrid, abs_tol_rel * std::sqrt(diag), seed, expand < 1.0 ? 1.0 : expand, kernel_limits != 0,
                lattice};
    TableCache TC;
    // importance sampling over G: patches of edge at most gauss_is x g
    if (gauss_is > 0 && !build_patches(S, G, gauss_is * G.g, P, TC)) return -4;
    std::vector<int32_t> nets(n_walks);
    std::vector<double> om(n_walks);
    if (threads < 1) threads = 1;
    std::vector<WalkStats> wst(threads);
    std::atomic<int> failed{0};
    auto worker = [&](int tid) {
        uint64_t lo = n_walks * (uint64_t)tid / threads, hi = n_walks * (uint64_t)(tid + 1) / threads;
        for (uint64_t k = lo; k < hi && !failed; ++k) {
            int net;
            double o;
            if (!frw_walk(S, G, master, P, TC, first_walk + k, &net, &o, wst[tid])) {
                failed = 1;
                return;
            }
            nets[k] = net;
            om[k] = o;
        }
    };
    if (threads == 1) {
        worker(0);
    } else {
        std::vector<std::thread> th;
        for (int t = 0; t < threads; ++t) th.emplace_back(worker, t);
        for (auto& t : th) t.join();
    }
    if (failed) return -3;
    // Alg. 1 scoring: C_ik accumulates omega of walks ending on k; averages
    // over n_path.  Standard errors from the per-net second moments.
    int K = n_nets + 1;
    std::vector<double> s1(K, 0.0), s2(K, 0.0);
    for (uint64_t k = 0; k < n_walks; ++k) {
        s1[nets[k]] += om[k];
        s2[nets[k]] += om[k] * om[k];
    }
    double nw = (double)n_walks;
    for (int j = 0; j < K; ++j) {
        double m = s1[j] / nw;
        row[j] = m;
        double var = (s2[j] / nw - m * m) / (nw - 1);
        se[j] = std::sqrt(std::max(var, 0.0));
    }
    if (score_net)
        for (uint64_t k = 0; k < n_walks; ++k) score_net[k] = nets[k];
    if (score_w)
        for (uint64_t k = 0; k < n_walks; ++k) score_w[k] = om[k];
    if (stats) {
        WalkStats tot;
        for (auto& w : wst) {
            tot.hops += w.hops;
            tot.micro_steps += w.micro_steps;
            for (int c = 0; c < 3; ++c) tot.hop_class[c] += w.hop_class[c];
            for (int c = 0; c < 4; ++c) tot.first_branch[c] += w.first_branch[c];
            tot.env += w.env;
            tot.hop_cap += w.hop_cap;
        }
        stats[0] = n_walks;
        stats[1] = tot.hops;
        stats[2] = tot.micro_steps;
        for (int c = 0; c < 3; ++c) stats[3 + c] = tot.hop_class[c];
        for (int c = 0; c < 4; ++c) stats[6 + c] = tot.first_branch[c];
        stats[10] = TC.misses.load();
        stats[11] = tot.env;
        stats[12] = tot.hop_cap;
    }
    return 0;
}

}  // extern "C"
