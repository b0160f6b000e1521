// l2c_device.h -- device helpers shared by the execution kernels (l2c_exec.hip,
// l2c_fused.hip): LDS staging, the near-field factors, and the upward / downward
// transfers of Eq. (wtk) and step (4) with the even/odd-diagonal split of App. A2.
#pragma once
#include "l2c_internal.h"
#include "l2c_math.h"

// Phase timestamps for performance analysis, compiled in only with L2C_PHASE_TIMING (the
// product build defines nothing and the macro expands to nothing; paper_2411_00033_amd/
// phase_timing.py builds and reads the instrumented variant).  Slot (kern, unit, phase)
// keeps the latest wall-clock time at which lane 0 of any wave of the unit's workgroup
// passed the point (first item of the launch, units < 4096).  Each source file has its
// own copy of the table.
#ifdef L2C_PHASE_TIMING
constexpr int kPhaseKernels = 4, kPhaseUnits = 4096, kPhaseSlots = 24;
static __device__ unsigned long long l2c_phase_ts[kPhaseKernels * kPhaseUnits * kPhaseSlots];
#define L2C_TS(kern, ph)                                                                               \
    do {                                                                                               \
        if ((threadIdx.x & 63) == 0 && blockIdx.y == 0 && blockIdx.x < kPhaseUnits)                    \
            atomicMax(&l2c_phase_ts[((kern) * kPhaseUnits + blockIdx.x) * kPhaseSlots + (ph)], wall_clock64()); \
    } while (0)
#else
#define L2C_TS(kern, ph) \
    do {                 \
    } while (0)
#endif

namespace l2c {

__device__ __forceinline__ int wave_id() { return __builtin_amdgcn_readfirstlane(threadIdx.x >> 6); }

// A bounded wait, timed on the device's constant-rate wall clock: expired() is false
// until `ticks` have passed since its first call.  A wait loop reads the clock only every
// few polls, so a bound of 0 gives up after a handful of polls.
struct WaitClock {
    uint64_t end = 0;
    __device__ __forceinline__ bool expired(uint64_t ticks)
    {
        const uint64_t now = wall_clock64();
        if (end == 0) {
            end = now + ticks + 1;
            return false;
        }
        return now >= end;
    }
};

// Status word `word` of a single-launch execute set to 1 (a vector store to host-mapped
// memory, visible to the host once the kernel has ended).
__device__ __forceinline__ void raise_status(int *status, int word)
{
    __hip_atomic_store(status + word, 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_SYSTEM);
}

// Copy count doubles from global memory to LDS.  The loads of each round are issued
// together (U per thread) before any is waited for, so a round costs one memory
// latency instead of U.
template <int U, int NT = kThreads>
__device__ __forceinline__ void stage_lds(double *dst, const double *src, int count)
{
    for (int base = 0; base < count; base += U * NT) {
        double v[U];
#pragma unroll
        for (int u = 0; u < U; ++u) {
            const int e = base + u * NT + (int)threadIdx.x;
            v[u] = e < count ? src[e] : 0.0;
        }
#pragma unroll
        for (int u = 0; u < U; ++u) {
            const int e = base + u * NT + (int)threadIdx.x;
            if (e < count) dst[e] = v[u];
        }
    }
}

// ------------------------------------------------------------------------------------
// Near-field tables.  Both directions are written as
//     z_i = rs_i * sum_{j >= i, j - i even} P[(j-i)/2] * Q[(i+j)/2] * g_j
// leg2cheb (Eq. (hik)):  P = Q = lambda, g = f, rs = 1.
// cheb2leg: the reverse kernel of Eq. (Lxymod) with d = (j-i)/2, S = (i+j)/2 factors
// as L(i,j) = (2i+1) j * [lambda_d / (1-2d)] * [1 / (2S (2S+1) lambda_S)], so
// P_d = lambda_d/(1-2d), Q_S = 1/(2S(2S+1) lambda_S), g_j = j u_j, rs_i = 2i+1, u = c .* f.
// At d = 0 this product is sqrt(pi)/(2 lambda_i) = (pi/2)/a_ii, the diagonal of A^{-1}C
// for i >= 1; the (0,0) entry (where g_0 = 0 and Q_0 := 0) contributes u_0/2 = f_0,
// added separately.
__device__ __forceinline__ double near_P(int dir, int64_t d)
{
    const double lam = lambda_int(d);
    return dir == 0 ? lam : lam / (1.0 - 2.0 * (double)d);
}

__device__ __forceinline__ double near_Q(int dir, int64_t S)
{
    if (dir == 0) return lambda_int(S);
    if (S == 0) return 0.0;
    const double S2 = 2.0 * (double)S;
    return inv_lambda_int(S) / (S2 * (S2 + 1.0));
}

// Node arrays in LDS keep a node's [sigma][k] = 2M doubles followed by one pad double:
// the odd node stride 2M + 1 puts lanes that read consecutive nodes on distinct banks
// (the workspace in global memory keeps the dense stride 2M).
template <int M>
__host__ __device__ constexpr int lds_ns() { return 2 * M + 1; }

// Every LDS operand load of a transfer is issued before its first product: left to
// itself the scheduler interleaves loads and products in small batches and waits for
// each batch, which makes one transfer several LDS latencies long.
template <int NLOADS>
__device__ __forceinline__ void ops_first()
{
    __builtin_amdgcn_sched_group_barrier(0x100, NLOADS, 0);   // LDS reads
    __builtin_amdgcn_sched_group_barrier(0x00a, 256, 0);      // then VALU and matrix-core ops
}

// Upward transfer of one level (Eq. (wtk) with App. A2): for every parent node and
// parity, out_n = sum_{k<=n} b_nk z_{(n-k) mod 2, k} with z0 = w(2T) + w(2T+1) and
// z1 = w(2T) - w(2T+1) (B(1) is B(0) with its odd diagonals negated).
// Lane <-> (parent, parity); wave residue H = wave mod 4 takes the outputs n = H mod 4,
// so its rows of B(0) are the same for every lane: they are read from LDS into
// registers once per level (one wait), then every product uses registers only.
template <int M, int H>
__device__ __forceinline__ void up_level_h(const double *child, double *par, int pn, const double *Bl, int q0,
                                           int qstep)
{
    constexpr int NJ = (M - H + 3) / 4;               // outputs n = H + 4j < M
    double bv[NJ][M];
#pragma unroll
    for (int j = 0; j < NJ; ++j) {
#pragma unroll
        for (int k = 0; k <= H + 4 * j; ++k) bv[j][k] = Bl[(H + 4 * j) * M + k];
    }
    for (int q = q0; q < 2 * pn; q += qstep) {
        const int pnode = q >> 1, sig = q & 1;
        const double *wa = child + (2 * pnode) * lds_ns<M>() + sig * M;
        const double *wb = wa + lds_ns<M>();
        double xv[M], yv[M], z0[M], z1[M];
#pragma unroll
        for (int k = 0; k < M; ++k) {
            xv[k] = wa[k];
            yv[k] = wb[k];
        }
        ops_first<2 * M>();
#pragma unroll
        for (int k = 0; k < M; ++k) {
            z0[k] = xv[k] + yv[k];
            z1[k] = xv[k] - yv[k];
        }
        double *po = par + pnode * lds_ns<M>() + sig * M;
#pragma unroll
        for (int j = 0; j < NJ; ++j) {
            const int n = H + 4 * j;
            double acc = 0.0;
#pragma unroll
            for (int k = 0; k <= n; ++k) acc = fma(bv[j][k], ((n - k) & 1) ? z1[k] : z0[k], acc);
            po[n] = acc;
        }
    }
}

template <int M>
__device__ __forceinline__ void up_level(const double *child, double *par, int pn, const double *Bl)
{
    const int wv = wave_id(), nw = blockDim.x >> 6;
    const int q0 = (threadIdx.x & 63) + 64 * (wv >> 2), qstep = 64 * (nw >> 2);
    switch (wv & 3) {
    case 0: up_level_h<M, 0>(child, par, pn, Bl, q0, qstep); break;
    case 1: up_level_h<M, 1>(child, par, pn, Bl, q0, qstep); break;
    case 2: up_level_h<M, 2>(child, par, pn, Bl, q0, qstep); break;
    default: up_level_h<M, 3>(child, par, pn, Bl, q0, qstep); break;
    }
}

// Downward transfer of one level (step (4)): c(child) += B(p)^T c(parent), p = child's
// position in its parent.  With B(1) = B(0) with odd diagonals negated,
// (B(p)^T c)_n = s_p(n) sum_{k>=n} b_kn s_p(k) c_k, s_p(k) = (-1)^k if p = 1, else 1.
// cn children; parent of child v is v >> 1; p = v & 1 unless pfix >= 0 (then p = pfix).
template <int M, int H>
__device__ __forceinline__ void down_level_h(const double *par, double *cur, int cn, int pfix, const double *Bl,
                                             int q0, int qstep)
{
    constexpr int NJ = (M - H + 3) / 4;
    double bv[NJ][M];
#pragma unroll
    for (int j = 0; j < NJ; ++j) {
#pragma unroll
        for (int k = H + 4 * j; k < M; ++k) bv[j][k] = Bl[k * M + H + 4 * j];
    }
    for (int q = q0; q < 2 * cn; q += qstep) {
        const int v = q >> 1, sig = q & 1;
        const int p = pfix >= 0 ? pfix : (v & 1);
        const double *cp = par + (v >> 1) * lds_ns<M>() + sig * M;
        double cs[M];
#pragma unroll
        for (int k = 0; k < M; ++k) cs[k] = cp[k];
        ops_first<M>();
#pragma unroll
        for (int k = 0; k < M; ++k) cs[k] = (p && (k & 1)) ? -cs[k] : cs[k];
        double *co = cur + v * lds_ns<M>() + sig * M;
#pragma unroll
        for (int j = 0; j < NJ; ++j) {
            const int n = H + 4 * j;
            double acc = 0.0;
#pragma unroll
            for (int k = n; k < M; ++k) acc = fma(bv[j][k], cs[k], acc);
            co[n] += (p && (n & 1)) ? -acc : acc;
        }
    }
}

template <int M>
__device__ __forceinline__ void down_level(const double *par, double *cur, int cn, int pfix, const double *Bl)
{
    const int wv = wave_id(), nw = blockDim.x >> 6;
    const int q0 = (threadIdx.x & 63) + 64 * (wv >> 2), qstep = 64 * (nw >> 2);
    switch (wv & 3) {
    case 0: down_level_h<M, 0>(par, cur, cn, pfix, Bl, q0, qstep); break;
    case 1: down_level_h<M, 1>(par, cur, cn, pfix, Bl, q0, qstep); break;
    case 2: down_level_h<M, 2>(par, cur, cn, pfix, Bl, q0, qstep); break;
    default: down_level_h<M, 3>(par, cur, cn, pfix, Bl, q0, qstep); break;
    }
}

// The same two transfers for levels with few nodes: thread <-> (node pair q, output n)
// with n fixed per thread, so the thread's row (up) or column (down) of B(0) sits in
// registers for the whole kernel.  Only threads t < M * (blockDim / M) take part:
// n = t mod M, first pair q0 = t / M, step qstep = blockDim / M.
//
// Up: out_n = sum_k b_nk x_k + sum_k (-1)^(n-k) b_nk y_k for children x = w(2T), y = w(2T+1)
// (the same as B(0) x + B(1) y).  With brow[k] = b_nk (zero for k > n) and the y sums
// split by the parity of k, out_n = X + (-1)^n (Y_even - Y_odd): no selects in the loop.
// Four partial sums per product (k mod 4) keep the dependent FMA chains short.

template <int M>
__device__ __forceinline__ double up_pair(const double (&brow)[M], const double *x, const double *y, int n)
{
    double xv[M], yv[M];
#pragma unroll
    for (int k = 0; k < M; ++k) {
        xv[k] = x[k];
        yv[k] = y[k];
    }
    ops_first<2 * M>();
    double a[4] = {0.0, 0.0, 0.0, 0.0}, b[4] = {0.0, 0.0, 0.0, 0.0};
#pragma unroll
    for (int k = 0; k < M; ++k) {
        a[k & 3] = fma(brow[k], xv[k], a[k & 3]);
        b[k & 3] = fma(brow[k], yv[k], b[k & 3]);
    }
    const double ys = (b[0] + b[2]) - (b[1] + b[3]);
    return ((a[0] + a[1]) + (a[2] + a[3])) + ((n & 1) ? -ys : ys);
}

template <int M>
__device__ __forceinline__ void up_level_qn(const double *child, double *par, int pn, const double (&brow)[M],
                                            int n, int q0, int qstep)
{
    for (int q = q0; q < 2 * pn; q += qstep) {
        const int pnode = q >> 1, sig = q & 1;
        const double *wa = child + (2 * pnode) * lds_ns<M>() + sig * M;
        par[pnode * lds_ns<M>() + sig * M + n] = up_pair<M>(brow, wa, wa + lds_ns<M>(), n);
    }
}

// Down: (B(p)^T c)_n = s_p(n) sum_{k>=n} b_kn s_p(k) c_k with s_p(k) = (-1)^k for p = 1:
// with E = sum over even k and O = sum over odd k of b_kn c_k, this is E + O for p = 0
// and (-1)^n (E - O) for p = 1 (bcol[k] = b_kn, zero for k < n).
template <int M>
__device__ __forceinline__ void down_level_qn(const double *par, double *cur, int cn, int pfix,
                                              const double (&bcol)[M], int n, int q0, int qstep)
{
    for (int q = q0; q < 2 * cn; q += qstep) {
        const int v = q >> 1, sig = q & 1;
        const int p = pfix >= 0 ? pfix : (v & 1);
        const double *cp = par + (v >> 1) * lds_ns<M>() + sig * M;
        double cv[M];
#pragma unroll
        for (int k = 0; k < M; ++k) cv[k] = cp[k];
        ops_first<M>();
        double e0 = 0.0, e1 = 0.0, o0 = 0.0, o1 = 0.0;
#pragma unroll
        for (int k = 0; k < M; k += 4) {
            e0 = fma(bcol[k], cv[k], e0);
            if (k + 1 < M) o0 = fma(bcol[k + 1], cv[k + 1], o0);
            if (k + 2 < M) e1 = fma(bcol[k + 2], cv[k + 2], e1);
            if (k + 3 < M) o1 = fma(bcol[k + 3], cv[k + 3], o1);
        }
        const double E = e0 + e1, O = o0 + o1;
        cur[v * lds_ns<M>() + sig * M + n] += p ? ((n & 1) ? O - E : E - O) : E + O;
    }
}

// Copy nodes between the dense workspace layout (stride 2M) and the padded LDS layout
// (stride 2M + 1), U elements per thread per round (one wait per round).
template <int M, int U, int NT>
__device__ __forceinline__ void nodes_lds_to_global(double *dst, const double *src, int nodes)
{
    const int count = nodes * 2 * M;
    for (int base = 0; base < count; base += U * NT) {
        double v[U];
#pragma unroll
        for (int u = 0; u < U; ++u) {
            const int e = base + u * NT + (int)threadIdx.x;
            const int q = e / (2 * M);
            v[u] = e < count ? src[q * lds_ns<M>() + (e - q * 2 * M)] : 0.0;
        }
#pragma unroll
        for (int u = 0; u < U; ++u) {
            const int e = base + u * NT + (int)threadIdx.x;
            if (e < count) dst[e] = v[u];
        }
    }
}

template <int M, int U, int NT>
__device__ __forceinline__ void nodes_global_to_lds(double *dst, const double *src, int nodes)
{
    const int count = nodes * 2 * M;
    for (int base = 0; base < count; base += U * NT) {
        double v[U];
#pragma unroll
        for (int u = 0; u < U; ++u) {
            const int e = base + u * NT + (int)threadIdx.x;
            v[u] = e < count ? src[e] : 0.0;
        }
#pragma unroll
        for (int u = 0; u < U; ++u) {
            const int e = base + u * NT + (int)threadIdx.x;
            const int q = e / (2 * M);
            if (e < count) dst[q * lds_ns<M>() + (e - q * 2 * M)] = v[u];
        }
    }
}

// Upward step over a whole subtree held in LDS: level buffer d (0 = the 2^kt input nodes)
// starts at node 2 nodes - 2 (nodes >> d); every level goes to the workspace at the end.
template <int M>
__device__ __forceinline__ void subtree_up(double *lv, int nodes, int kt, const double *Bl)
{
    const int qstep = kThreads / M, n = (int)threadIdx.x % M, q0 = (int)threadIdx.x / M;
    const bool qn_ok = (int)threadIdx.x < M * qstep;
    double brow[M];
#pragma unroll
    for (int k = 0; k < M; ++k) brow[k] = Bl[(qn_ok ? n : 0) * M + k];
    for (int d = 1; d <= kt; ++d) {
        const int pn = nodes >> d;
        const double *child = lv + (2 * nodes - 2 * (nodes >> (d - 1))) * lds_ns<M>();
        double *par = lv + (2 * nodes - 2 * pn) * lds_ns<M>();
        if (2 * pn <= qstep) {
            if (qn_ok) up_level_qn<M>(child, par, pn, brow, n, q0, qstep);
        } else {
            up_level<M>(child, par, pn, Bl);
        }
        __syncthreads();
    }
}

}  // namespace l2c
