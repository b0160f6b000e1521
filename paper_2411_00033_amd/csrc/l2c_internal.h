// l2c_internal.h -- plan structure, geometry and launch entry points shared by the
// host driver (l2c_api.hip) and the kernels (l2c_exec.hip, l2c_plan.hip).
//
// Geometry (arXiv 2411.00033, Sec. 3.1).  With L levels and half leaf side s:
//   * the padded length is N = s 2^(L+2) (Eq. (Ntot));
//   * level g (0 = coarsest) cuts the index line into 2^(g+2) nodes of 2 h_g
//     entries, h_g = s 2^(L-g-1); the finest level L-1 has P = 2^(L+1) nodes of 2s;
//   * block b of level g (b < b_g = 2^(g+1)-1, Eq. (Nb)) holds the submatrices
//     (p,q) = (0,0), (0,1), (1,1): row node 2b+p against column node 2b+q+2
//     (Eq. (globalij)); r = p + q(q+1)/2 (Eq. (cfrompq));
//   * Eq. (flevels)/(zlevels): the children of node t are nodes 2t and 2t+1 of the
//     next finer level.
// The upward work vectors w (Eq. (wTf)) of every level live in one array: level g
// starts at node offset 2^(g+2) - 4, each node holds [sigma][k] = 2 x M doubles, and
// the array has 2^(L+2) - 4 nodes per item.
//
// Execution subtrees.  k_main gives each workgroup the 2^kd finest nodes below one
// node R of level groot = L-1-kd.  Its "own" far-field blocks are the complete blocks
// of levels groot+1 .. L-1 below R (2^kd - 1 blocks); the blocks of levels 0..groot
// (shared by several workgroups: the ancestors of R) form the "top" table.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

#define L2C_MAX_LEVELS 40

// Ranks with compiled kernels (even: the far-field layout packs pairs of FP64).
#define L2C_FOR_EACH_RANK(X) X(12) X(16) X(18) X(20) X(24)

namespace l2c {

constexpr int kThreads = 256;        // threads per workgroup of the execution kernels
constexpr int kUpDepth = 6;          // finest nodes per k_up workgroup = 2^kUpDepth
constexpr int kTopDepth = 6;         // levels reduced by one k_top workgroup
constexpr int kMainDepth = 6;        // at most 2^kMainDepth finest nodes per k_main workgroup
constexpr int kNearRows = 8;         // same-parity rows per thread in the near-field loop
constexpr int kMainThreads = 512;    // k_main: 8 waves, two per SIMD (FP64 issue needs >= 2)
constexpr int kNearItems = 1;        // near-field work items per k_main thread
constexpr int kMainLds = 160 * 1024; // LDS of one gfx950 CU: k_main runs one workgroup per CU
constexpr int64_t kMaxItemsPerLaunch = 32768;  // grid.y limit with margin
// Batched form (l2c_batched.hip): 16 transforms per matrix-core tile, one wave per
// subtree of 2^depth nodes in each of its three kernels.
constexpr int kBatUpDepth = 3;
constexpr int kBatTopDepth = 3;
// kb_main subtree depth, every form: at depth 3 its FP64 LDS (the near field's staged input,
// Q window and output rows; the FP64 tile form's far-field tiles) would leave room for one
// workgroup per CU
constexpr int kBatMainDepth = 2;
__host__ __device__ constexpr int bat_main_depth(int) { return kBatMainDepth; }
constexpr int64_t kBatMaxTiles = 32768;        // tiles (of 16 items) per launch

__host__ __device__ inline int64_t node_offset(int g) { return (int64_t(1) << (g + 2)) - 4; }

// Far-field tables.
//   top:    levels 0..groot, level-major, block-major, [r][k][l] row-major (M x M each);
//           level g starts at block (2^(g+1) - 2 - g).
//   bottom: per subtree R (R < 2^(groot+2)), its 2^kd - 1 own blocks, finest depth
//           first (depth d = kd, kd-1, ..., 1 below R, 2^(d-1) blocks each, left to
//           right; depth d starts at block 2^kd - 2^d, see slot_depth).  "Slot"
//           (j, k) = row k of the three submatrices of local block j (3M doubles).
//           Slots are grouped 64 at a time (one wavefront); 16-byte chunk c of slot
//           lane l of group G is at ((G * (3M/2) + c) * 64 + l) * 16 bytes, so every
//           wavefront load instruction reads 1 KiB of contiguous memory.  Each subtree
//           owns sub_groups groups; slots past (2^kd - 1) M are zero.
struct Geometry {
    int L, M, s;
    int ku, kt, kd;           // subtree depths of k_up, k_top, k_main
    int groot;                // L - 1 - kd
    int sub_groups;           // wavefront groups per subtree in the bottom table
    int64_t NT;               // workspace nodes per item
    int64_t NF;               // tree-top nodes, levels 0..groot: node_offset(groot + 1)
    int64_t NX;               // k_fused exchange nodes per item: NF, then 2 (kd-1) per unit
};

struct ExecArgs {
    const double *in;
    double *out;
    int64_t n;           // valid length of every item
    // ragged batches: per item of this launch its length and vectors (null: n, in + item n,
    // out + item n)
    const int64_t *item_n;
    const double *const *item_in;
    double *const *item_out;
    int64_t batch;
    int dir;             // 0 leg2cheb, 1 cheb2leg
    Geometry geo;
    const double *T;     // [2][s][M]
    const double *B0;    // [M][M]
    const double *Ptab;  // [2 s + 2 kNearRows]: kNearRows - 1 zeros, then the near-field factor P_d
    const double *ahat_top;
    const double *ahat_bot;
    double *w;           // [batch][NT][2][M]
    double *pub;         // k_fused: [2][pub_items][NX][2][M] exchange nodes, half (epoch & 1) in use
    int64_t pub_items;   // k_fused: items of one half of pub
    unsigned epoch;      // k_fused: launch number
    int *status;         // k_fused: status words (host-mapped); word k set to 1 when a wait of kind k gave up
    uint64_t wait_ticks; // k_fused: bound of the waits inside a workgroup, in wall-clock ticks
    uint64_t poll_ticks; // k_fused: bound of the waits for other workgroups, in wall-clock ticks
    const int *top_sched; // k_fused: [units][kTopSchedInts] tree-top table per unit (built at plan time)
    // k_main: the far-field part of step (3) for the own blocks, computed by k_regen
    // ([batch][subtrees][own nodes][2][M]); null: k_main streams the stored bottom table
    const double *cfar = nullptr;
};

// Ints per unit of k_fused's tree-top table (reduction schedule and item nodes).
constexpr int kTopSchedInts = 128;

// Status words of the single-launch path (ExecArgs::status), one per kind of wait; the
// plan reports word k as bit k (leg2cheb_plan_status).
constexpr int kStatusExchange = 0;   // a poll of another workgroup's exchange nodes
constexpr int kStatusWorkers = 1;    // a barrier of the worker waves, or of the near-field waves
constexpr int kStatusStream = 2;     // the streaming wave waiting for the workers' depth flags
constexpr int kStatusWords = 4;

// Device arrays of a ragged batch, one entry per item of the launch sequence.
struct ItemArrays {
    const int64_t *n;
    const double *const *in;
    double *const *out;
};

}  // namespace l2c

struct l2c_plan_s {
    int64_t n, n_pad;
    int L, s, M, direction, precision, leaf;
    int device;
    int64_t nb, nc;
    l2c::Geometry geo;
    double *d_top = nullptr;    // far-field table, levels 0..groot
    double *d_bot = nullptr;    // far-field table, levels groot+1..L-1 (subtree-major)
    double *d_T = nullptr;      // [2][s][M]
    double *d_B = nullptr;      // [2][M][M] (B(0), B(1))
    double *d_P = nullptr;      // near-field factor table, see ExecArgs::Ptab
    double *d_XG = nullptr;     // [M] Chebyshev-Gauss points
    double *d_D = nullptr;      // [M][M] cos(k (m+1/2) pi / M)
    double *d_w = nullptr;
    int64_t ws_batch = 0;       // items the workspace holds
    int64_t top_bytes = 0, bot_bytes = 0;
    int64_t table_bytes = 0;
    hipEvent_t ev_before = nullptr, ev_after = nullptr;
    // single-launch path (k_fused)
    bool fused_ok = false;      // geometry, LDS and co-residency allow it
    bool fused_on = true;       // caller preference (leg2cheb_plan_set_option)
    int64_t fused_items = 0;    // items per k_fused launch (all workgroups co-resident)
    double *d_pub = nullptr;    // ExecArgs::pub, fused_items items per half
    int *d_topsch = nullptr;    // ExecArgs::top_sched
    int *h_status = nullptr;    // kStatusWords words of pinned, device-mapped host memory
    int *d_status = nullptr;    // the device address of h_status
    unsigned epoch = 0;
    int64_t poll_us = 1000000;  // bound of the waits for other workgroups (L2C_OPT_EXCHANGE_TIMEOUT_US)
    int clock_khz = 0;          // wall-clock rate of the device (hipDeviceAttributeWallClockRate)
    // batched form (precision L2C_FP32): tables in the form's type and a workspace of
    // [tiles][NT][2][16 x 16] tiles; the FP64 Ahat tables are released after packing
    void *d_bA = nullptr;       // Ahat, [blocks][3][64][4] A operands
    void *d_bT = nullptr;       // [2][s][M]
    void *d_bB = nullptr;       // [M][M] (nodal basis: [2][M][M], B(0) then B(1))
    void *d_bP = nullptr;       // [2s]
    int basis = 0;              // l2c_basis
    int64_t max_batch = 0;      // as requested at plan time
    int cache_refs = 0;         // > 0: a shared plan of the plan cache (leg2cheb_plan_cached)
    void *d_bQ = nullptr;       // [n_pad + 2s]
    void *d_bw = nullptr;
    bool tile64 = false;        // an FP64 plan that executes in the FP64 tile form (l2c_batched.hip)
    float *d_bS = nullptr;      // FP16X2: [blocks][3] factors undoing each submatrix's scaling
    int64_t bw_tiles = 0;
    // FP64 batches of short transforms (l2c_dense.hip): per parity the dense coefficient
    // matrix of Alg. 1, [2][HP][HP]
    double *d_dense = nullptr;
    // short FP64 transforms (n <= kDirectMaxN, max_batch n^2 <= direct_max_work(n)): Alg. 1 row
    // by row (k_direct) instead of the multipole kernels for executes within the same
    // work bound, unless switched off (leg2cheb_plan_set_option)
    bool direct_ok = false;
    bool direct_on = true;
    // k_direct's factor tables: P_d for d < ceil(n/2), then Q_S for S < n + 17 (plans with
    // L = 0, and plans with direct_ok)
    double *d_dir = nullptr;
    // Lambda((y-x)/2) per level and offset, [L][2][M][M] (the plan's samples, l2c_regen.hip)
    double *d_lm = nullptr;
    // far-field blocks below the subtree roots recomputed in every execute (L2C_TABLES_REGEN,
    // l2c_regen.hip): no bottom table; the far-field part of step (3) per own node,
    // [ws_batch][subtrees][own nodes][2][M]
    bool regen = false;
    double *d_cf = nullptr;
};

namespace l2c {
// l2c_exec.hip
// k_direct is faster than Alg. 4 (by measurement) while n <= kDirectMaxN and
// batch n^2 <= direct_max_work(n): its work grows as n^2 per transform, and above
// n = 4096 its LDS band (3 n / 2 doubles) leaves room for one workgroup per CU
constexpr int64_t kDirectMaxN = 8192;
inline int64_t direct_max_work(int64_t n) { return n <= 4096 ? int64_t(1) << 27 : int64_t(1) << 26; }
int64_t direct_table_len(int64_t n);
hipError_t direct_build(const l2c_plan_s &p, double *tab, hipStream_t stream);
hipError_t launch_direct(const l2c_plan_s &p, const double *in, double *out, int64_t batch, hipStream_t stream,
                         const ItemArrays *ia = nullptr);
hipError_t launch_execute(const l2c_plan_s &p, const double *in, double *out, int64_t batch,
                          hipStream_t stream, const ItemArrays *ia = nullptr);
// kernel attributes of the plan's FP64 launches, set once per process (plan time)
hipError_t prepare_launches(const l2c_plan_s &p);
// leg2cheb_execute_noalloc: the three-launch path with w in a fixed device array of
// kNoallocScratchBytes (resolved per device by noalloc_scratch)
constexpr size_t kNoallocScratchBytes = size_t(64) << 20;
hipError_t noalloc_scratch(int device, double **ptr);
hipError_t launch_execute_scratch(const l2c_plan_s &p, const double *in, double *out, int64_t batch,
                                  hipStream_t stream, double *w);
// l2c_fused.hip
bool fused_supported(int M);
hipError_t fused_max_items(const l2c_plan_s &p, int64_t *items);
// k_fused's tree-top table of every unit, into a new device array (synchronous).
hipError_t fused_top_table(const l2c_plan_s &p, int **dst);
hipError_t launch_fused(l2c_plan_s &p, const double *in, double *out, int64_t batch, hipStream_t stream,
                        const ItemArrays *ia = nullptr);
// l2c_batched.hip
hipError_t batched_build_tables(const l2c_plan_s &p, void *ahat_dst, void *q_dst, int64_t q_len, hipStream_t stream);
hipError_t launch_batched(const l2c_plan_s &p, const double *in, double *out, int64_t batch, hipStream_t stream,
                          const ItemArrays *ia = nullptr);
// The FP64 tile form: FP64 plans with rank <= 16, leaf <= 64 and max_batch >= kTile64MinBatch
// (one 16-transform tile or more) that the dense path does not take
constexpr int64_t kTile64MinBatch = 16;
// l2c_dense.hip: FP64 plans with L >= 1, n <= kDenseMaxN and max_batch >= kDenseMinBatch
constexpr int64_t kDenseMaxN = 4096, kDenseMinBatch = 64;
int64_t dense_hp(int64_t n);
hipError_t dense_build(const l2c_plan_s &p, double *D, hipStream_t stream);
hipError_t launch_dense(const l2c_plan_s &p, const double *in, double *out, int64_t batch, hipStream_t stream,
                        const ItemArrays *ia = nullptr);
// l2c_plan.hip
hipError_t launch_build_small(const l2c_plan_s &p, hipStream_t stream);   // T, P, XG, D
hipError_t launch_to_f32(const double *src, float *dst, int64_t n, hipStream_t stream);
hipError_t launch_build_ahat(const l2c_plan_s &p, hipStream_t stream);
hipError_t launch_export_ahat(const l2c_plan_s &p, double *dst_dev, hipStream_t stream);
// l2c_regen.hip: plans with L2C_TABLES_REGEN
hipError_t launch_build_lminus(const l2c_plan_s &p, hipStream_t stream);   // d_lm
// k_regen: the far-field part of step (3) of the own blocks of items 0..c.batch-1 of c
// into cf, from the upward vectors in c.w
hipError_t launch_regen(const l2c_plan_s &p, const ExecArgs &c, double *cf, hipStream_t stream);
// doubles of cf per item
inline int64_t regen_cf_per_item(const Geometry &G)
{
    return (int64_t(1) << (G.groot + 2)) * (2 * (int64_t(1) << G.kd) - 2) * 2 * G.M;
}

// Near-field LDS padding of k_main: the per-parity input g has node stride s + gpad and
// the Q table node stride 2s + qpad, odd when padded (distinct banks across 64 nodes).
// Used for s >= 2 kNearRows, where a row window crosses at most one node boundary.
__host__ __device__ inline int near_gpad(int s) { return (s >= 2 * kNearRows && !(s & 1)) ? 1 : 0; }
__host__ __device__ inline int near_qpad(int s) { return s >= 2 * kNearRows ? 1 : 0; }
__host__ __device__ inline int64_t near_gx(int s, int kd)
{
    return (int64_t)(s + near_gpad(s)) * ((1 << kd) + 1) + 2 * kNearRows + 4;
}
__host__ __device__ inline int64_t near_nq(int s, int kd)
{
    const int64_t qs = 2 * s + near_qpad(s);
    return qs * ((1 << kd) + 1) + 3 * (int64_t)s + 2 * kNearRows;
}

// LDS of k_main (doubles): B(0), ancestor and own c, own-column w, and the padded
// near-field tables, later reused for T.
inline int64_t main_lds_doubles(int L, int M, int s, int kd)
{
    const int64_t R = kNearRows, nodes = int64_t(1) << kd;
    const int64_t own = 2 * nodes - 2, NS = 2 * M + 1;   // LDS node stride (one pad double)
    const int64_t nP = 2 * (int64_t)s + 2 * R;
    const int64_t near = 2 * near_gx(s, kd) + near_nq(s, kd) + nP, tz = 2 * (int64_t)s * M;
    return (int64_t)M * M + (int64_t)(L - kd) * NS + 2 * own * NS + (near > tz ? near : tz);
}

// Staging registers per k_main thread (column-node w and near-field input).
constexpr int kMainStageW = 9, kMainStageG = 9;

// k_fused (single launch, one workgroup per level-groot subtree, all co-resident).
// Waves 0 .. kStreamWaves-1 stream the subtree's far-field table; the other waves
// ("workers", kWorkThreads threads) do everything else.
constexpr int kFusedThreads = 512;
constexpr int kStreamWaves = 1;
constexpr int kWorkThreads = kFusedThreads - 64 * kStreamWaves;   // 448
constexpr int kWorkWaves = kWorkThreads / 64;                     // 7
constexpr int kFusedRows = 11;            // near-field rows per work item (3 items per node and parity at s = 31)
constexpr int kNearWaves = 6;             // worker waves that run the near field (one item per thread)
constexpr int kTopWave = 4;               // the wave (of the workgroup) that works above the unit
static_assert(kStreamWaves == 1 && kNearWaves == kWorkWaves - 1 && kTopWave > kStreamWaves && kTopWave < 8,
              "wave roles: one streamer, one top wave, the rest near-field waves");
constexpr int64_t kWaitUs = 1000000;      // bound of every wait inside a workgroup (1 s)
constexpr int kFusedStageG = 12, kFusedStageT = 4;   // staging registers per worker thread
// Both 32-bit halves of an exchange node value that the current launch has not written yet
// (a signalling NaN, which no arithmetic result is).
constexpr unsigned kPubEmptyHalf = 0x7FF00001u;

// Node offset of depth d in the k_fused w buffer: depth 0 is the subtree root alone;
// depth d >= 1 holds the subtree's 2^d nodes followed by nodes 0, 1 of the next subtree.
__host__ __device__ inline int fused_wofs(int d) { return d == 0 ? 0 : (1 << d) + 2 * d - 3; }

// Near-field input of k_fused: per parity, the unit's finest nodes plus two of the next
// unit (step (1) needs both, the near field one), node stride s + gpad; Q with node
// stride 2s + qpad.  A pad keeps the 64 lanes of a wave (64 nodes) on distinct banks.
// The near-field loop reads column m' < 2s + R - 1 of g (two node boundaries at most
// when R <= s + 1) and Q offsets c < 3s + 2R - 2 (one boundary when 2R - 3 < s); pads
// are used only where those bounds hold.
__host__ __device__ inline int fused_gpad(int s) { return (!(s & 1) && kFusedRows <= s + 1) ? 1 : 0; }
__host__ __device__ inline int fused_qpad(int s) { return 2 * kFusedRows - 3 < s ? 1 : 0; }
__host__ __device__ inline int64_t fused_gx(int s, int kd)
{
    return (int64_t)(s + fused_gpad(s)) * ((1 << kd) + 2) + 2 * kFusedRows + 4;
}
__host__ __device__ inline int64_t fused_nq(int s, int kd)
{
    return (int64_t)(2 * s + fused_qpad(s)) * ((1 << kd) + 1) + 3 * (int64_t)s + 2 * kFusedRows;
}

// Load items of the top wave: below level gl = groot - min(3, groot) a column node is
// reduced from the 2^(gl-g) level-gl nodes under it, at and above gl it is loaded.
__host__ __device__ inline int fused_top_items(int groot)
{
    const int H = groot < 3 ? groot : 3, gl = groot - H;
    return 2 * ((1 << (gl + 1)) - 2) + 2 * (H + 1);
}

// The near-field area: input, Q and P during the near field; afterwards the unit's
// output rows (node stride 2s+1; 2 GX exceeds them).
__host__ __device__ inline int64_t fused_near_area(int L, int M, int s, int kd)
{
    (void)L;
    (void)M;
    return 2 * fused_gx(s, kd) + fused_nq(s, kd) + 2 * (int64_t)s + 2 * kFusedRows;
}

// The T area: T for steps (1) and (5); in between, the tree-top nodes the top wave
// reduces while the near field runs (T is loaded again afterwards).
__host__ __device__ inline int64_t fused_t_area(int L, int M, int s, int kd)
{
    const int64_t t = 2 * (int64_t)s * M, items = fused_top_items(L - 1 - kd) * (2 * (int64_t)M + 1);
    return t > items ? t : items;
}

// Top-wave scratch of k_fused (doubles): the exchange's 2^min(3, groot) nodes of NS,
// later the chain's z [2 x 2M] and canc [(groot+1) x 2M].
__host__ __device__ inline int64_t fused_w7(int M, int groot)
{
    const int64_t chain = 4 * (int64_t)M + (int64_t)(groot + 1) * 2 * M;
    const int64_t exch = (int64_t(1) << (groot < 3 ? groot : 3)) * (2 * (int64_t)M + 1);
    return chain > exch ? chain : exch;
}

// LDS of k_fused (doubles): B(0), T, the near-field area, w (all depths plus neighbour
// nodes), own c, the root c, the top wave's scratch, a dummy node pair for stores of
// out-of-range slots, and 8 words of flags/counters.
inline int64_t fused_lds_doubles(int L, int M, int s, int kd)
{
    const int64_t nodes = int64_t(1) << kd, NS = 2 * M + 1;
    const int64_t WN = fused_wofs(kd + 1), own = 2 * nodes - 2;
    const int groot = L - 1 - kd;
    return (int64_t)M * M + fused_t_area(L, M, s, kd) + fused_near_area(L, M, s, kd) + WN * NS + own * NS + NS +
           fused_w7(M, groot) + 2 * NS + 4;
}

// Subtree depths for a plan with L >= 1 levels.
inline Geometry make_geometry(int L, int M, int s)
{
    Geometry g;
    g.L = L;
    g.M = M;
    g.s = s;
    g.ku = L - 1 < kUpDepth ? L - 1 : kUpDepth;
    g.kt = kTopDepth;
    // k_main: each thread takes up to kNearItems (finest node, parity, kNearRows rows)
    // items, and the workgroup's LDS must fit one CU
    const int nch = (s + kNearRows - 1) / kNearRows;
    int kd = L - 1 < kMainDepth ? L - 1 : kMainDepth;
    while (kd > 0 && (((1 << kd) * 2 * nch) > kMainThreads * kNearItems || main_lds_doubles(L, M, s, kd) * 8 > kMainLds ||
                      (2 * ((1 << kd) - 1)) * 2 * M > kMainStageW * kMainThreads ||
                      2 * (s * ((1 << kd) + 1) + kNearRows) > kMainStageG * kMainThreads))
        --kd;
    g.kd = kd;
    g.groot = L - 1 - g.kd;
    const int64_t slots = (((int64_t)1 << g.kd) - 1) * M;
    g.sub_groups = (int)((slots + 63) / 64);
    g.NT = ((int64_t)1 << (L + 2)) - 4;
    g.NF = node_offset(g.groot + 1);
    g.NX = g.NF + (g.kd >= 1 ? (int64_t(1) << (g.groot + 2)) * 2 * (g.kd - 1) : 0);
    return g;
}

// Local block j of a subtree (finest depth first) -> depth d (1..kd) and index i within
// the depth: depth d holds j in [2^kd - 2^d, 2^kd - 2^(d-1)).
__host__ __device__ inline void slot_depth(int j, int kd, int &d, int &i)
{
    const unsigned u = (1u << kd) - (unsigned)j;   // in (2^(d-1), 2^d], >= 2
    d = 32 - __builtin_clz(u - 1u);
    i = j - ((1 << kd) - (1 << d));
}

// The near-field factor table of a plan holds kPLead zeros and then P_d for
// d = 0 .. 2 s + kPLead; a kernel with R rows per item starts reading at kPLead - (R - 1).
constexpr int kPLead = 15;
inline int64_t p_table_len(int s) { return 2 * (int64_t)kPLead + 2 * (int64_t)s + 2; }

// First block of level g in the level-major enumeration.
__host__ __device__ inline int64_t level_block_offset(int g) { return ((int64_t)1 << (g + 1)) - 2 - g; }
}  // namespace l2c
