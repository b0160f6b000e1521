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
// Per-node work vectors w (upward, Eq. (wTf)) and c (far field, step (3)) are stored
// for every level in one array: level g starts at node offset 2^(g+2) - 4, each
// node holds [sigma][k] = 2 x M doubles, and the array has 2^(L+2) - 4 nodes.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

#define L2C_MAX_LEVELS 40

// Ranks with compiled kernels (even: the far-field layout packs pairs of FP64).
#define L2C_FOR_EACH_RANK(X) X(12) X(16) X(18) X(20) X(24)

namespace l2c {

constexpr int kThreads = 256;        // threads per workgroup of every execution kernel
constexpr int kUpDepth = 5;          // finest-level nodes per upward workgroup = 2^kUpDepth
constexpr int kDownDepth = 4;        // finest-level nodes per downward workgroup = 2^kDownDepth
constexpr int kNearRows = 4;         // same-parity rows per thread in the near-field loop
constexpr int kFarItems = 8;         // batch items per far-field workgroup
constexpr int64_t kMaxItemsPerLaunch = 32768;  // grid.y limit with margin

__host__ __device__ inline int64_t node_offset(int g) { return (int64_t(1) << (g + 2)) - 4; }

// Far-field table layout.  Level g has b_g blocks; "slot" (b, k) (M slots per
// block) holds row k of the three submatrices of block b: 3M doubles.  Slots are
// grouped 64 at a time (one wavefront); within a group, 16-byte chunk c of slot
// lane l is stored at ((group * (3M/2) + c) * 64 + l) * 16 bytes, so each
// wavefront load instruction reads 1 KiB of contiguous memory.  Every level
// starts on a group boundary; slots past b_g * M are zero.
struct FarLayout {
    int L;
    int M;
    int64_t group_off[L2C_MAX_LEVELS + 1];   // first group of each level; [L] = total
};

struct ExecArgs {
    const double *in;
    double *out;
    int64_t n;           // valid length of every item
    int64_t n_pad;       // N
    int64_t batch;
    int L, s, M, dir;    // dir: 0 leg2cheb, 1 cheb2leg
    int ku, kd;          // subtree depths of the upward and downward kernels
    const double *T;     // [2][s][M]
    const double *B0;    // [M][M]
    const double *ahat;  // far-field layout
    double *w;           // [batch][NT][2][M]
    double *c;           // [batch][NT][2][M]
    int64_t NT;          // nodes per item
};

}  // namespace l2c

struct l2c_plan_s {
    int64_t n, n_pad;
    int L, s, M, direction, precision, leaf;
    int device;
    int64_t nb, nc;
    l2c::FarLayout far;
    int64_t NT;                 // workspace nodes per item
    double *d_ahat = nullptr;   // far-field table
    double *d_T = nullptr;      // [2][s][M]
    double *d_B = nullptr;      // [2][M][M] (B(0), B(1))
    double *d_XG = nullptr;     // [M] Chebyshev-Gauss points
    double *d_D = nullptr;      // [M][M] cos(k (m+1/2) pi / M)
    double *d_w = nullptr;
    double *d_c = nullptr;
    int64_t ws_batch = 0;       // items the workspace holds
    int64_t ahat_bytes = 0;
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
}  // namespace l2c
