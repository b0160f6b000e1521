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

__host__ __device__ inline int64_t node_offset(int g) { return (int64_t(1) << (g + 2)) - 4; }

// Far-field tables.
//   top:    levels 0..groot, level-major, block-major, [r][k][l] row-major (M x M each);
//           level g starts at block (2^(g+1) - 2 - g).
//   bottom: per subtree R (R < 2^(groot+2)), its 2^kd - 1 own blocks in level order
//           (depth d = 1..kd below R, 2^(d-1) blocks each, left to right).  "Slot"
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
};

struct ExecArgs {
    const double *in;
    double *out;
    int64_t n;           // valid length of every item
    int64_t batch;
    int dir;             // 0 leg2cheb, 1 cheb2leg
    Geometry geo;
    const double *T;     // [2][s][M]
    const double *B0;    // [M][M]
    const double *ahat_top;
    const double *ahat_bot;
    double *w;           // [batch][NT][2][M]
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
    double *d_XG = nullptr;     // [M] Chebyshev-Gauss points
    double *d_D = nullptr;      // [M][M] cos(k (m+1/2) pi / M)
    double *d_w = nullptr;
    int64_t ws_batch = 0;       // items the workspace holds
    int64_t top_bytes = 0, bot_bytes = 0;
    int64_t table_bytes = 0;
    hipEvent_t ev_before = nullptr, ev_after = nullptr;
};

namespace l2c {
// l2c_exec.hip
hipError_t launch_execute(const l2c_plan_s &p, const double *in, double *out, int64_t batch,
                          hipStream_t stream);
// l2c_plan.hip
hipError_t launch_build_ahat(const l2c_plan_s &p, hipStream_t stream);
hipError_t launch_export_ahat(const l2c_plan_s &p, double *dst_dev, hipStream_t stream);

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
    return g;
}

// First block of level g in the level-major enumeration.
__host__ __device__ inline int64_t level_block_offset(int g) { return ((int64_t)1 << (g + 1)) - 2 - g; }
}  // namespace l2c
