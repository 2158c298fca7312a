/*
 * libmwalk — floating-random-walk (FRW) capacitance extraction whose
 * transitions inside non-stratified dielectric cubes use MicroWalk
 * (Huang & Yu, "Efficient FRW Transitions via Stochastic Finite Differences
 * for Handling Non-Stratified Dielectrics", arXiv 2507.09730).
 *
 * C ABI of the MI355X (gfx950) library. Conventions for every entry point:
 *   - Every call returns an mw_status: 0 on success, a negative code on error.
 *     No C++ exception crosses this boundary.  mw_last_error() returns a
 *     thread-local, NUL-terminated message describing the last failure of the
 *     calling thread (empty string after a success).
 *   - Outputs are written only on success (device outputs of stream-ordered
 *     calls: only by kernels that the call enqueued after validation).
 *   - The caller owns every array passed in or out.  The library copies what
 *     it keeps (structures, request descriptions) and never frees caller
 *     memory.
 *   - "device" pointers are HIP device allocations on the current device;
 *     "host" pointers are ordinary host memory.  `stream` is a hipStream_t
 *     (NULL = the legacy default stream); stream-ordered calls enqueue their
 *     kernels there and return without waiting, unless stated otherwise.
 *   - Lengths are in micrometres, permittivities are relative (eps0 is
 *     applied inside), capacitances are in femtofarads.
 *   - Validation rejects, before any device work: relative permittivities
 *     outside [1e-3, 1e3]; lattice sizes outside [2, 64] (vertex lattice: even
 *     n, cell lattice: odd n); null pointers where a buffer is required.
 *
 * Random numbers (shared contract with any reimplementation): every random
 * 32-bit word is one output word of Philox4x32-10 (Salmon, Moraes, Dror &
 * Shaw, SC'11) with key = (seed & 0xffffffff, seed >> 32) and counter
 *   c0 = s >> 2            (s = running index of the word within the stream)
 *   c1 = hop index t (FRW) or cube index (transition APIs)
 *   c2 = walk & 0xffffffff
 *   c3 = ((walk >> 32) & 0xffffff) | (purpose << 24)
 * taking output word s & 3.  Purposes: 0 MicroWalk step, 1 Gaussian-surface
 * sample, 2 first-transition sample, 3 stratified-table sample.
 */
#ifndef LIBMWALK_H
#define LIBMWALK_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef int32_t mw_status;
#define MW_OK 0
#define MW_EINVAL (-1)    /* bad argument                                  */
#define MW_ENOMEM (-2)    /* device or host allocation failed              */
#define MW_EDEVICE (-3)   /* HIP runtime error                             */
#define MW_EBUSY (-4)     /* server queue full                             */
#define MW_ENOTREADY (-5) /* server result not ready yet                   */
#define MW_EGEOM (-6)     /* invalid geometry                              */
#define MW_ELIMIT (-7)    /* a documented capacity limit was exceeded      */

/* Finite-difference lattice of a transition cube with n cells per axis.
 * MW_LATTICE_VERTEX: nodes at cell corners, (n+1)^3 nodes, (n-1)^3 interior
 *   unknowns, start node (n/2,n/2,n/2) (n even).  Link probability of a
 *   direction is proportional to the sum of the four cell codes around the
 *   link (finite-volume face permittivity; equal to the normalised
 *   coefficients of Eq. (6) written for this node placement).
 * MW_LATTICE_CELL: nodes at voxel centres as in Sec. III-A (Fig. 2), N^3
 *   interior nodes plus 6N^2 boundary panel nodes, coefficients of Eq. (6)
 *   verbatim, start node ((N-1)/2, ...) (N odd).                             */
#define MW_LATTICE_VERTEX 0
#define MW_LATTICE_CELL 1

/* Boundary condition of each window face, order -x,+x,-y,+y,-z,+z. */
#define MW_BC_DIRICHLET 0 /* grounded enclosure: absorbs walks into "env" */
#define MW_BC_NEUMANN 1   /* mirror symmetry plane                        */

const char* mw_last_error(void);

/* Selects the HIP device used by subsequent calls of this thread and
 * initialises per-device state.  Optional: the first call on a device does it. */
mw_status mw_init(int32_t device);

/* ------------------------------------------------------------------------
 * mw_transition — Alg. 3 (MicroWalk) on one voxelised transition cube.
 *
 * Runs n_walks independent micro-walks from the cube's start node until each
 * reaches a boundary node (Alg. 3; Theorem 1 makes the hit distribution equal
 * to the discrete SGF P_eps = e_c^T A_II^-1 A_IB of Eq. (8)).  Walk w (for w
 * in [first_walk, first_walk + n_walks)) uses Philox words of purpose 0 with
 * c1 = cube_index; step s consumes word s.  The direction of a step is
 * d = #{k in 0..4 : u >= T_k}, with T_k = ceil(S_k * 2^32 / S_5) and S_k the
 * prefix sums of the six integer link codes in direction order
 * -x,+x,-y,+y,-z,+z.  Cell codes: vertex lattice e = rint(eps * 2^16);
 * cell lattice link code rint(eps_i / (eps_i + eps_v) * 2^24) to an interior
 * neighbour and 2^24 to a boundary panel (Eq. 6), both in binary64.
 *
 * eps        device, n^3 floats, cell (i,j,k) at eps[(k*n + j)*n + i].
 * n_cells    n: 2..64, even for the vertex lattice, odd for the cell lattice.
 * hit_idx    device, n_walks int32: boundary hit index.  Vertex lattice:
 *            f*M^2 + (b-1)*M + (a-1), M = n-1; cell lattice: f*N^2 + b*N + a;
 *            f = 2*axis + side (side 1 = the +axis face), (a, b) the two
 *            other node coordinates in ascending axis order.  -1 if the walk
 *            exceeded 2^30 steps (cannot happen for valid permittivities).
 * steps      device, n_walks int32 step counts tau, or NULL.
 * Ordering: the permittivity range check needs one device round trip, so the
 * call enqueues the table preparation on `stream`, waits for it (and for the
 * work queued before it on that stream), then enqueues the walks and returns
 * without waiting for them.                                                 */
mw_status mw_transition(const float* eps, int32_t n_cells, int32_t lattice,
                        uint64_t n_walks, uint64_t first_walk, uint64_t seed,
                        uint32_t cube_index, int32_t* hit_idx, int32_t* steps,
                        void* stream);

/* ------------------------------------------------------------------------
 * mw_transition_noalloc — mw_transition for callers that cannot allocate
 * device memory (code under HIP graph capture, tight serving loops, harnesses
 * that forbid hipMalloc).  Same arguments, results bit-identical to
 * mw_transition.  Instead of a per-call allocation it uses a static device
 * array of MW_NOALLOC_SCRATCH_BYTES per device (the cube descriptor, counters
 * and the prepared threshold or cell-code table: 256 bytes plus about 20
 * bytes per lattice node; vertex-lattice cubes up to n = 48 fit).  It calls no
 * hipMalloc, hipFree or allocating library routine.  MW_ELIMIT when the cube's
 * table does not fit (the error names both sizes).  Every call on a device
 * shares that device's array, which keeps the last call's contents; the
 * counters are cleared by a kernel at the start of each call.  Calls that
 * overlap on one device (other host threads, or other streams) race on the
 * array and give wrong results: the caller serialises them.  Like
 * mw_transition it waits on `stream` for the permittivity range check before
 * enqueueing the walks.                                                     */
#define MW_NOALLOC_SCRATCH_BYTES (4u << 20)
mw_status mw_transition_noalloc(const float* eps, int32_t n_cells, int32_t lattice,
                                uint64_t n_walks, uint64_t first_walk, uint64_t seed,
                                uint32_t cube_index, int32_t* hit_idx, int32_t* steps,
                                void* stream);

/* Tuning knobs of the batched MicroWalk launch.  Zero fields mean "use the
 * autotuned or default value". */
typedef struct {
    int32_t tile_form;      /* 1 threshold rows in LDS, 2 cell-code tile in LDS */
    int32_t waves_per_wg;   /* 1..16                                          */
    int32_t refill_every;   /* steps between lane refills: 4, 8 or 16         */
    int32_t item_walks;     /* walks per (cube, walk-range) work item         */
    int32_t walks_per_lane; /* interleaved walks per lane: 1, 2 or 4          */
} mw_tune;

/* ------------------------------------------------------------------------
 * mw_transition_batch — many cubes of uneven size in one persistent launch.
 *
 * Cube c (0 <= c < n_cubes) has n_cells[c] cells per axis, its eps grid at
 * eps_cat + eps_off[c] (device, layout as mw_transition) and runs n_walks[c]
 * walks 0..n_walks[c]-1 with Philox c1 = c.  Its hits (and steps) go to
 * hits_cat + out_off[c] (device).  Results are bit-identical to calling
 * mw_transition(eps_c, n_c, lattice, n_walks[c], 0, seed, c, ...) per cube,
 * for every tuning.  eps_off, n_cells, n_walks, out_off are host arrays.
 * tune may be NULL (the setting mw_autotune_batch found for a batch of the
 * same shape, else defaults).
 * Synchronous: waits on `stream` for the permittivity range check of the
 * prepared tables, then for the walks; the host arrays may be reused once the
 * call returns.  (mw_batch_plan_run is the stream-ordered form.)           */
mw_status mw_transition_batch(int32_t n_cubes, const float* eps_cat,
                              const int64_t* eps_off, const int32_t* n_cells,
                              int32_t lattice, const uint64_t* n_walks,
                              const int64_t* out_off, uint64_t seed,
                              int32_t* hits_cat, int32_t* steps_cat,
                              const mw_tune* tune, void* stream);

/* Autotuner of the batched launch: times the batch's walk kernel under
 * candidate tunings (tile form, waves per workgroup, refill interval, walks
 * per work item, interleaved walks per lane; coordinate search) and writes
 * the fastest to *best.  Later mw_transition_batch and mw_batch_plan_create
 * calls with tune == NULL on a batch of the same shape (histogram of cube
 * sizes in buckets of 4 cells and walk-count scale) use it.  When the
 * environment variable MWALK_TUNE_CACHE names a file, tuned settings are
 * kept there as JSON (per device architecture) and read by later processes.
 * Writes hits/steps as a side effect (with an internal seed).  Synchronous. */
mw_status mw_autotune_batch(int32_t n_cubes, const float* eps_cat,
                            const int64_t* eps_off, const int32_t* n_cells,
                            int32_t lattice, const uint64_t* n_walks,
                            const int64_t* out_off, int32_t* hits_cat,
                            int32_t* steps_cat, mw_tune* best, void* stream);

/* The setting a batch call with tune == NULL would use for a batch of this
 * shape (found = 1), from this process's autotuning or the MWALK_TUNE_CACHE
 * file; found = 0 when there is none (defaults apply).  Host arrays.        */
mw_status mw_tune_lookup(int32_t n_cubes, const int32_t* n_cells, const uint64_t* n_walks,
                         int32_t lattice, mw_tune* out, int32_t* found);

/* A batch prepared once (cube descriptors, work items, table buffers) and
 * captured as a HIP graph (counter reset, table preparation, walk kernels).
 * mw_batch_plan_run replays it on `stream` with a new seed; results equal
 * mw_transition_batch with the same arguments and seed.  The plan keeps the
 * device pointers given at creation: eps_cat may change between runs (its
 * values must stay in [1e-3, 1e3]; the range is checked at creation only),
 * outputs are rewritten by every run.  Runs on one plan are serialised by the
 * plan (each run waits for the previous run's seed upload).                */
typedef struct mw_batch_plan mw_batch_plan;
mw_status mw_batch_plan_create(int32_t n_cubes, const float* eps_cat,
                               const int64_t* eps_off, const int32_t* n_cells,
                               int32_t lattice, const uint64_t* n_walks,
                               const int64_t* out_off, int32_t* hits_cat,
                               int32_t* steps_cat, const mw_tune* tune,
                               mw_batch_plan** out);
mw_status mw_batch_plan_run(mw_batch_plan* plan, uint64_t seed, void* stream);
mw_status mw_batch_plan_destroy(mw_batch_plan* plan);

/* ------------------------------------------------------------------------
 * Geometry (Alg. 1 input: a 3-D structure of conductors and dielectrics).
 *
 * Conductor boxes are half-open [lo, hi) per axis and belong to nets
 * 0..n_nets-1; a net owns one or more boxes, which may touch or overlap
 * (boxes of different nets may not overlap).  Dielectric boxes override the
 * background; a later box wins where boxes overlap.  The background is a
 * stack of layers in z: layer l covers z in [layer_z0[l], layer_z0[l+1]) with
 * relative permittivity layer_eps[l]; the first layer extends to -inf and the
 * last to +inf, layer_z0 ascending.  The window [win_lo, win_hi) encloses the
 * structure; bc[] holds MW_BC_* per face (-x,+x,-y,+y,-z,+z).              */
typedef struct {
    float lo[3], hi[3];
    int32_t net;
} mw_cond_box;

typedef struct {
    float lo[3], hi[3];
    float eps;
} mw_diel_box;

typedef struct {
    int32_t n_cond;
    const mw_cond_box* cond; /* host */
    int32_t n_nets;
    int32_t n_diel;
    const mw_diel_box* diel; /* host */
    int32_t n_layers;
    const float* layer_z0;  /* host, n_layers */
    const float* layer_eps; /* host, n_layers */
    float win_lo[3], win_hi[3];
    uint8_t bc[6];
} mw_structure_desc;

typedef struct mw_structure mw_structure;

/* Copies the description to the device and builds the uniform-grid
 * acceleration structure (per grid cell: the conductors that can be nearest
 * to a point of the cell and the dielectric boxes that a conductor-free cube
 * centred in the cell can touch).  MW_EGEOM on overlapping boxes of different
 * nets, a net with no box, a net index outside [0, n_nets), boxes outside the
 * window or empty boxes; a net may own several boxes (multi-box nets).      */
mw_status mw_structure_create(const mw_structure_desc* desc, mw_structure** out);
mw_status mw_structure_destroy(mw_structure* s);

typedef struct {
    int32_t n_cells;          /* cube lattice size: even, 4..32, on the vertex
                                 lattice (default 16); odd, 3..31, on the cell
                                 lattice (default 15)                       */
    int32_t hybrid;           /* 1 (default): stratified non-first cubes use
                                 the exact SGF table, the rest MicroWalk
                                 (Sec. III-C); 0: every non-first cube uses
                                 MicroWalk                                  */
    int32_t expand;           /* MicroWalk-E (Sec. III-B, Fig. 3(b)): 0 or 1
                                 off; E > 1: MicroWalk hops use cubes of
                                 half-size n d / (2 m), m = max(1,
                                 round(n / (2 E))), d the conductor-free
                                 half-size (E = 5, n = 16: 4 d), which may
                                 hold conductors: walks reaching a node inside
                                 a conductor or beyond a grounded face end
                                 there, links into such nodes are cut at the
                                 face (Shortley-Weller).  The cube stops at
                                 symmetry walls and is halved, not below d,
                                 while it touches more than 16 dielectric
                                 boxes or 7 conductors.  n / (2 m) may not
                                 exceed 4.                                  */
    int32_t plain;            /* 0 (default): persistent walker launches (a
                                 lane takes a new walk as soon as its walk
                                 ends); 1: the plain form, one walker launch
                                 per transition round (each launch moves every
                                 live walk by one transition, survivors are
                                 queued for the next launch).  Per-walk
                                 results are the same in both forms.        */
    double target_rel_3sigma; /* stop when 3*SE(C_mm)/|C_mm| <= target; 0 =
                                 run exactly walk_budget walks              */
    double abs_tol_rel;       /* absorption distance / window diagonal;
                                 default 1e-6                               */
    uint64_t first_walk;      /* id of the first walk (resume point)         */
    uint64_t batch_walks;     /* walks between checks of the target (a
                                 multiple of 65536 after rounding up for
                                 frw_extract); 0 = 65536 for frw_extract    */
    double gauss_is;          /* sampling of the Gaussian-surface point.  0
                                 (default): uniform by area, weight factor
                                 |G|.  > 0: importance sampling over G (the
                                 first transition of Alg. 1 is importance
                                 sampling with its weight): every surface
                                 rectangle is cut into equal patches of edge
                                 at most gauss_is * g, patch p is drawn with
                                 probability q_p / Q, q_p = area_p K(c_p) / h
                                 (the first-transition kernel sum at its
                                 centre, computed once per extraction), the
                                 point is uniform on it and the weight factor
                                 is Q area_p / q_p.  The estimator keeps its
                                 expectation; its variance drops where K
                                 varies over G.  0 or in [0.05, 64].       */
    int32_t lattice;          /* MW_LATTICE_VERTEX (0, default): nodes at the
                                 cell corners; the walk starts at the centre
                                 node and leaves through a boundary node.
                                 MW_LATTICE_CELL (1): Sec. III-A as written,
                                 nodes at the voxel centres with the Eq. (6)
                                 coefficients; the walk starts in the centre
                                 cell and leaves through the centre of a
                                 boundary panel.  Stratified tables and
                                 first-transition weights use the same
                                 lattice (the face permittivity of a link
                                 between two cells is their series value
                                 2 e1 e2 / (e1 + e2)); homogenised first cubes
                                 take each plane's mean permittivity.  The
                                 cell lattice needs an odd n_cells and plain
                                 MicroWalk (expand <= 1).                   */
} frw_options;

typedef struct {
    uint64_t walks;           /* completed walks (n_path)                   */
    uint64_t hops;            /* non-first transitions                      */
    uint64_t micro_steps;     /* Alg. 3 loop iterations                      */
    uint64_t hop_class[3];    /* non-first cubes: uniform, stratified, other */
    uint64_t first_branch[4]; /* first cubes: uniform, stratified along the
                                 surface normal, stratified along another
                                 axis, homogenised                          */
    uint64_t cache_miss;      /* SGF tables built                           */
    uint64_t env_absorbed;    /* walks ending on a grounded window face     */
    uint64_t hop_cap;         /* walks stopped by the 1e5-hop cap           */
    uint64_t launches;        /* walker-kernel launches                      */
    double seconds;           /* wall time of the call                      */
    double walker_seconds;    /* summed duration of the walker-kernel launches
                                 (HIP events on the launch stream, also
                                 inside a replayed launch graph)            */
    double gauss_g;           /* frw_extract: growth g of the master's
                                 Gaussian surface (um); 0 for the matrix    */
    double gauss_area;        /* frw_extract: its area (um^2); 0 for the
                                 matrix                                     */
    uint64_t gauss_faces;     /* frw_extract: its rectangles; 0 for the
                                 matrix                                     */
    uint64_t cube_halved;     /* transitions (first and non-first) whose cube
                                 the capacity rule (MW_MAX_REGIONS dielectric
                                 boxes, or the MicroWalk-E limits) made
                                 smaller than the conductor-free, or
                                 expanded, size                             */
    uint64_t walks_launched;  /* frw_extract: walks walked, including those
                                 after the checkpoint where the target was
                                 met (not in the row); the counters above
                                 count the work of all of them               */
} frw_stats;

/* ------------------------------------------------------------------------
 * frw_extract — Alg. 1 for master net `master`: one row of the capacitance
 * matrix.  Walk w = first_walk + k (k < number of walks run): Gaussian-
 * surface sample, first transition with weight omega, transitions until the
 * walk lands on a conductor (net k) or a grounded window face ("env"); then
 * C_{master,k} += omega.  cap_row[j] = sum of omega over walks ending on net j
 * divided by the number of walks (fF); cap_row[n_nets] is the env column.
 * stderr_row[j] is the standard error of cap_row[j].  Runs walk_budget walks,
 * or, when options->target_rel_3sigma > 0, stops at the first checkpoint
 * (every options->batch_walks walks, rounded up to a multiple of 65536;
 * default 65536, at most 2^27) where 3 SE(C_mm) / |C_mm| <= target, and
 * the row holds exactly the walks up to that checkpoint.  The walks are run in launches of
 * several checkpoints, sized from the walk count the last such call on this
 * structure, master and rule needed; walks after the stopping checkpoint are
 * dropped (stats->walks_launched counts them).  Walk scores are summed per
 * net in fp32 with compensated (Kahan) sums per block of 4096 walks, in
 * fp64 over each group of 16 blocks and then over the groups in walk order,
 * so a row is the same for any split into launches: a target-mode row
 * equals the fixed-budget row of the same number of walks.
 * score_net/score_w (device, walk_budget entries each, or NULL): per-walk net
 * index (n_nets for env) and fp32 weight, indexed by walk - first_walk;
 * entries from stats->walks on are unspecified.
 * The structure keeps the call's device buffers (per master and options, at
 * most four sets, each sized for the largest launch: 2^23 walks with a
 * target, up to 2^26 without) for later calls, with HIP graphs of the usual
 * launch that later calls replay (set MWALK_FRW_GRAPHS=0 for eager
 * launches; results are the same); mw_structure_destroy frees them.  Calls
 * on one structure from several threads are safe.
 * stats may be NULL.  Synchronous: returns after the result is on the host.
 * Transition cubes are the largest conductor-free cubes, halved while they
 * touch more than MW_MAX_REGIONS dielectric boxes; MW_ELIMIT if more than
 * MW_MAX_REGIONS dielectric boxes overlap at one point.                     */
#define MW_MAX_REGIONS 16
mw_status frw_extract(mw_structure* s, int32_t master, uint64_t walk_budget,
                      uint64_t seed, const frw_options* options,
                      double* cap_row, double* stderr_row, frw_stats* stats,
                      int32_t* score_net, float* score_w);

/* ------------------------------------------------------------------------
 * frw_autotune — launch geometry of the FRW walker kernel: times the walker
 * on `walks` walks of this extraction (walk ids options->first_walk on,
 * Philox key seed) with 4, 6, 8, ... up to the most resident waves per CU
 * that its LDS allows, and keeps the fastest for the lattice size and
 * MicroWalk-E setting of the options; later extractions, matrix calls and
 * servers use it (also across processes through MWALK_TUNE_CACHE).  The
 * geometry changes no per-walk result.  *waves_per_cu receives the choice.
 * Synchronous.                                                              */
mw_status frw_autotune(mw_structure* s, int32_t master, uint64_t walks, uint64_t seed,
                       const frw_options* options, int32_t* waves_per_cu);

/* ------------------------------------------------------------------------
 * mw_table_cache_clear — empties the transition-table cache of lattice size
 * n_cells (even 4..32: vertex lattice; odd 3..31: cell lattice) on the
 * current device; later calls rebuild the
 * tables they need (the tables are pure functions of their keys, so no
 * result changes).  Must not run while an extraction or server uses that
 * cache.  MW_EINVAL for a bad size.  Synchronous.                          */
mw_status mw_table_cache_clear(int32_t n_cells);

/* ------------------------------------------------------------------------
 * mw_sgf_table — one entry of the transition-table cache (the "analytical
 * path" of the hybrid strategy, Sec. III-C), built on the device if missing,
 * copied to the host.  Used to check the tables against an independent exact
 * solve; extraction calls never need it.
 *
 * The cube has n_cells = n cells per axis on the vertex lattice and is
 * stratified along `axis`: plane p normal to it (p = 0..n-1, ascending
 * coordinate) has cell code plane_codes[p] = rint(eps_p * 2^16).
 * kind 0 (hop table): the exit distribution P_b of the walk from the centre
 *   node (Eq. 8 via Theorem 1), b the vertex-lattice hit index
 *   (f*M^2 + (b1-1)*M + (a-1), M = n-1, as mw_transition).
 * kind 1 (first-transition table, normal axis `normal_axis`): the flux
 *   weights w_b = [G+ (P^c_b - P^+_b) + G- (P^-_b - P^c_b)] / 2 of the
 *   centre node c and its two neighbours c +- e_normal, G+-  the link
 *   conductances of c along +-normal in units of eps (the four cell codes of
 *   the link / 2^18); sampled in proportion to |w_b|.
 * cdf        host, 6 M^2 uint32: cdf[b] = ceil(2^32 * (sum of the weights of
 *            entries <= b) / (sum of all weights)), clamped to 2^32 - 1 (a
 *            word u samples the first b with cdf[b] > u).
 * sign_bits  host, ceil(6 M^2 / 32) uint32 or NULL: kind 1, bit b set when
 *            w_b > 0 (kind 0: unspecified).
 * kh         host, 1 float or NULL: kind 1, sum_b |w_b| (the first-transition
 *            weight is eps0 |G| kh / h times the sign); kind 0: 0.
 * n_cells even in 4..32; codes in [66, 65536000] (eps in [1e-3, 1e3]).
 * Cell-centred lattice (Sec. III-A, frw_options.lattice = 1): n_cells odd in
 *   3..31, plane_codes[p] the bit pattern of the plane's float permittivity
 *   (in [1e-3, 1e3]), M = n, the walk starts in the centre cell, b is the
 *   panel index f*n^2 + b1*n + a (as mw_transition's cell lattice), and G+-
 *   are the series permittivities 2 e_c e_+- / (e_c + e_+-) of the centre
 *   cell and its neighbours along the normal.
 * MW_ELIMIT when the cache is full.  Synchronous.                          */
mw_status mw_sgf_table(int32_t n_cells, int32_t kind, int32_t axis, int32_t normal_axis,
                       const uint32_t* plane_codes, uint32_t* cdf, uint32_t* sign_bits, float* kh);

/* ------------------------------------------------------------------------
 * frw_extract_matrix — Alg. 1 for n_masters masters (distinct net indices in
 * masters[]): rows of the capacitance matrix.  Master i runs
 * walks_per_master walks with Philox key seed + i, walk ids first_walk on;
 * each row equals frw_extract(s, masters[i], walks_per_master, seed + i,
 * options) up to fp32 summation order.  The masters' walks share rounds
 * (one set of walker launches and one reduction per round).  With
 * options->target_rel_3sigma > 0 a master stops once its own C_mm meets the
 * target (checked every options->batch_walks walks, or only at the end when
 * that is 0).
 * cap, stderr (host, n_masters x (n_nets+1), row-major): rows as in
 * frw_extract.  cap_sym (host, n_masters x n_masters, or NULL): the
 * symmetrised block over the listed masters, (C[a][m_b] + C[b][m_a]) / 2 off
 * the diagonal and C[a][m_a] on it (the matrix is symmetric in exact
 * arithmetic; Maxwell reciprocity).  stats may be NULL; its walks field sums
 * all masters.  Errors as frw_extract; MW_EINVAL for a repeated master.   */
mw_status frw_extract_matrix(mw_structure* s, int32_t n_masters,
                             const int32_t* masters, uint64_t walks_per_master,
                             uint64_t seed, const frw_options* options,
                             double* cap, double* stderr_, double* cap_sym,
                             frw_stats* stats);

/* ------------------------------------------------------------------------
 * Serving: a request loop over one device with continuous batching.
 *
 * mw_server_submit copies the structure description and returns a ticket.
 * A preparation thread takes queued requests in arrival order while their
 * device footprint (structure, grid index, reduction partials, accumulators)
 * fits within hbm_budget_bytes, and uploads each structure and builds its
 * grid index on a stream of its own, while rounds run.  A round worker runs
 * rounds of a fixed walk capacity over every prepared request: the
 * longest-running one gets up to three quarters of it, the rest goes to the
 * requests with the fewest remaining walks first, and capacity they leave
 * goes back to the longest-running one; each share is that request's next
 * walk ids (from 0).  All shares of a round run in one set of kernel
 * launches, one reduction launch and one result copy, so requests that
 * arrive while others run join at the next round and their work overlaps on
 * the device.  The server's own round buffers (per-walk scores of one round,
 * parked-walk queues; about 0.8 GB) are allocated at the first round and
 * are not counted in the budget.  A request completes
 * when walk_budget walks have run or options->target_rel_3sigma is met
 * (checked after each of its rounds).  Per-walk results are those of
 * frw_extract(structure, master, walk_budget, seed, options) run alone; rows
 * agree with it to fp32 summation order (1e-6 relative).
 * MW_ELIMIT at poll time if a request's footprint alone exceeds the budget;
 * MW_EBUSY from submit when the queue holds max_queue requests.            */
typedef struct mw_server mw_server;

typedef struct {
    uint64_t submitted, completed, failed;
    uint64_t rounds, walks;
    uint64_t resident_bytes;      /* current admitted footprint               */
    uint64_t max_resident_bytes;  /* peak admitted footprint (<= budget)      */
    uint64_t max_concurrent;      /* peak number of requests in one round     */
} mw_server_stats;

mw_status mw_server_create(size_t hbm_budget_bytes, const frw_options* options,
                           mw_server** out);
mw_status mw_server_submit(mw_server* srv, const mw_structure_desc* desc,
                           int32_t master, uint64_t walk_budget, uint64_t seed,
                           uint64_t* ticket);
/* MW_ENOTREADY until the request has finished; then cap_row/stderr_row
 * (n_nets+1 entries of the request's structure) and, if non-NULL, stats and
 * latency_s (completion minus submission, seconds) are written.  A failed
 * request returns its error code. */
mw_status mw_server_poll(mw_server* srv, uint64_t ticket, double* cap_row,
                         double* stderr_row, frw_stats* stats, double* latency_s);
mw_status mw_server_get_stats(mw_server* srv, mw_server_stats* out);
/* Stops admitting, finishes the running requests, fails the queued ones,
 * joins the worker and frees the server. */
mw_status mw_server_destroy(mw_server* srv);

#ifdef __cplusplus
}
#endif
#endif /* LIBMWALK_H */
