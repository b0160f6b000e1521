// l2c_fused.hip -- single-launch execution of Alg. 4 (steps (0)-(7)) for gfx950, FP64.
//
// One workgroup per subtree ("unit") of 2^kd finest nodes below node X of level
// groot = L-1-kd, all units of an item resident at once (one workgroup per CU).  A unit
// needs from the rest of the grid only
//   * nodes 0 and 1 of the next unit at every depth (its own far-field blocks reach two
//     nodes past its right edge, Eq. (globalij)); at the finest depth it computes them
//     itself from the input, at coarser depths it reads them, and
//   * the upward vectors of levels 0..groot, which combine every unit's root.
// Both travel through the workspace with per-node ready flags.  Every flag holds the
// number ("epoch") of the launch that last wrote the node, so flags never need clearing.
// The data are written and read with device-coherent accesses, and a flag is set only
// after the writes it covers have completed; nothing else crosses workgroups.
//
// Inside a workgroup the waves specialise.
//   Streamers (waves 0, 1) read the unit's far-field table (the dominant HBM traffic)
//   once the workers' staging loads are out, one 64-slot group (27.6 KiB at M = 18) in
//   flight per wave:
//   enough to keep HBM busy without queueing requests so deep that every other memory
//   access of the kernel waits behind them.  The table is laid out finest depth first,
//   and a group is multiplied (step (3)) as soon as the workers flag its depths ready.
//   Workers (waves 2..7) stage the input, B(0), T and the near-field tables; step (1)
//   for the unit's finest nodes (and two of the next unit); step (2) inside the unit,
//   flagging each depth; publish the root and nodes 0, 1 of every coarser depth; fetch
//   the next unit's nodes (one wave); step (6), the near field (four waves).  Meanwhile
//   the last worker wave does step (2) above the units (the leftmost unit below an
//   ancestor reduces the nodes under it, three levels per exchange, and publishes it),
//   then, once the near field is done, the far-field blocks of the unit's ancestors
//   (step (3), top table), and the downward chain from level 0 to the unit root
//   (step (4)).  Workers synchronise through LDS counters, streamers poll LDS flags;
//   there is no hardware barrier between the first and the last phase.
//   Then all waves: step (4) inside the unit, steps (5) and (7), and the output.
// A wait that never completes (another kernel holding CUs forever) gives up after
// kSpinLimit polls and sets a status bit; the launch then ends with a wrong result
// instead of hanging.  The host keeps single-launch kernels of different streams from
// overlapping, so every workgroup of a launch becomes resident.
#include <mutex>

#include "l2c_device.h"

namespace l2c {

__device__ __forceinline__ void store_coherent(double *p, double v)
{
    __hip_atomic_store(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

__device__ __forceinline__ double load_coherent(const double *p)
{
    return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

// Wait until every store this wave has issued is complete (s_waitcnt vmcnt(0)); the
// fence keeps the compiler from moving later memory operations above it.
__device__ __forceinline__ void wave_stores_done()
{
    __builtin_amdgcn_s_waitcnt(0x0f70);
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "workgroup");
}

__device__ __forceinline__ void set_flag(unsigned *f, unsigned epoch)
{
    __hip_atomic_store(f, epoch, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

// Lane 0 polls the flag until it equals epoch (bounded); the wave continues afterwards.
__device__ __forceinline__ void wave_wait_flag(const unsigned *f, unsigned epoch, int *status)
{
    if ((threadIdx.x & 63) == 0) {
        bool ok = false;
        for (int it = 0; it < kSpinLimit; ++it) {
            if (__hip_atomic_load(f, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) == epoch) {
                ok = true;
                break;
            }
            __builtin_amdgcn_s_sleep(1);
        }
        if (!ok) atomicOr(status, 1);
    }
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "workgroup");
}

// LDS written by some lanes of a wave and then read by other lanes of the same wave:
// LDS executes a wave's operations in order; this keeps the compiler from reordering.
__device__ __forceinline__ void wave_lds_sync() { __builtin_amdgcn_fence(__ATOMIC_ACQ_REL, "wavefront"); }

// Wait until this wave's LDS operations are complete (s_waitcnt lgkmcnt(0)).
__device__ __forceinline__ void wave_lds_done()
{
    __builtin_amdgcn_s_waitcnt(0xc07f);
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "workgroup");
}

// Barrier of the worker waves only (LDS counter; target is this wave's running count).
__device__ __forceinline__ void worker_sync(unsigned *cnt, unsigned &target, int *status)
{
    wave_lds_done();
    target += kWorkWaves;
    if ((threadIdx.x & 63) == 0) {
        __hip_atomic_fetch_add(cnt, 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
        int it = 0;
        while (__hip_atomic_load(cnt, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP) < target) {
            __builtin_amdgcn_s_sleep(1);
            if (++it == kSpinLimit) {
                atomicOr(status, 2);
                break;
            }
        }
    }
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "workgroup");
}

__device__ __forceinline__ void lds_flag_set(unsigned *f, unsigned v)
{
    __hip_atomic_store(f, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
}

__device__ __forceinline__ unsigned lds_flag_get(const unsigned *f)
{
    return __hip_atomic_load(f, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
}

// Forces v to be computed here: instruction selection otherwise moves pure arithmetic
// next to its final use, past the scheduling barriers that bound register lifetimes.
__device__ __forceinline__ void pin(double &v) { asm volatile("" : "+v"(v)); }

// One group of step (3) for a streaming wave: 64 slots x 3 rows, held in the ring t0..t2
// (row r of every slot); with REFILL the same rows of group nxt are loaded as soon as
// each row has been used.  Slot (j, k) = row k of the three submatrices of block j
// (depth d, index i): c(2i)[k] = Ahat(.,0)[k,:] w(2i+2) + Ahat(.,1)[k,:] w(2i+3),
// c(2i+1)[k] = Ahat(.,2)[k,:] w(2i+3), both parities.
template <int M, bool REFILL>
__device__ __forceinline__ void stream_group(int grp, int nxt, const double2 *sub, const double *wl, double *cown,
                                             double *dummy, int kd, int nslots, int lane, const unsigned *rdy,
                                             const unsigned *nbr,
                                             double2 (&t0)[M / 2], double2 (&t1)[M / 2], double2 (&t2)[M / 2])
{
    constexpr int NCH = 3 * M / 2, NC3 = M / 2, NS = lds_ns<M>();
    const int slot = grp * 64 + lane;
    const bool valid = slot < nslots;
    const int j = valid ? slot / M : 0, k = valid ? slot - j * M : 0;
    int d, i;
    slot_depth(j, kd, d, i);
    int dlo, ilo;                                     // coarsest depth in the group
    slot_depth(min(grp * 64 + 63, nslots - 1) / M, kd, dlo, ilo);
    for (int it = 0; it < kSpinLimit; ++it) {
        if (lds_flag_get(rdy) <= (unsigned)dlo && (dlo == kd || lds_flag_get(nbr) != 0)) break;
        __builtin_amdgcn_s_sleep(1);
    }
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "workgroup");
    const double *wa = wl + (fused_wofs(d) + 2 * i + 2) * NS;   // w(2i+2); w(2i+3) follows
    // one parity at a time (M column values in registers next to the 3-row ring)
    double c00 = 0.0, c01 = 0.0, c10 = 0.0, c11 = 0.0;
#pragma unroll
    for (int sg = 0; sg < 2; ++sg) {
        double wx[M];
#pragma unroll
        for (int l = 0; l < M; ++l) wx[l] = wa[sg * M + l];
        double a0 = 0.0;
#pragma unroll
        for (int c = 0; c < NC3; ++c) a0 = fma(t0[c].y, wx[2 * c + 1], fma(t0[c].x, wx[2 * c], a0));
        pin(a0);
        if (sg == 0) c00 = a0;
        else c01 = a0;
        __builtin_amdgcn_sched_barrier(0);        // one parity's column values at a time
    }
    // the scheduler must not hoist a refill above the last use of the registers it replaces
    __builtin_amdgcn_sched_barrier(0);
    if (REFILL) {
#pragma unroll
        for (int c = 0; c < NC3; ++c) t0[c] = sub[(nxt * NCH + c) * 64];
    }
    __builtin_amdgcn_sched_barrier(0);
#pragma unroll
    for (int sg = 0; sg < 2; ++sg) {
        double wy[M];
#pragma unroll
        for (int l = 0; l < M; ++l) wy[l] = wa[NS + sg * M + l];
        double a1 = 0.0, a2 = 0.0;
#pragma unroll
        for (int c = 0; c < NC3; ++c) {
            a1 = fma(t1[c].y, wy[2 * c + 1], fma(t1[c].x, wy[2 * c], a1));
            a2 = fma(t2[c].y, wy[2 * c + 1], fma(t2[c].x, wy[2 * c], a2));
        }
        pin(a1);
        pin(a2);
        if (sg == 0) {
            c00 += a1;
            c10 = a2;
        } else {
            c01 += a1;
            c11 = a2;
        }
        __builtin_amdgcn_sched_barrier(0);
    }
    __builtin_amdgcn_sched_barrier(0);
    if (REFILL) {
#pragma unroll
        for (int c = 0; c < NC3; ++c) t1[c] = sub[(nxt * NCH + NC3 + c) * 64];
#pragma unroll
        for (int c = 0; c < NC3; ++c) t2[c] = sub[(nxt * NCH + 2 * NC3 + c) * 64];
    }
    // unconditional stores (lanes past the last slot write a dummy node pair): a guarded
    // store would let the compiler sink the products into the branch, behind the refills
    double *co = valid ? cown + ((1 << d) - 2 + 2 * i) * NS + k : dummy;
    co[0] = c00;
    co[M] = c01;
    co[NS] = c10;
    co[NS + M] = c11;
}

template <int M>
__global__ __launch_bounds__(kFusedThreads) void k_fused(ExecArgs a)
{
    constexpr int R = kFusedRows;
    constexpr int NCH = 3 * M / 2;                    // 16-byte chunks of a slot (3 rows of M doubles)
    constexpr int NC3 = M / 2;                        // chunks of one row (a "third")
    constexpr int M2 = 2 * M;
    constexpr int NS = lds_ns<M>();
    constexpr int NTH = kFusedThreads, NSW = kStreamWaves, NWT = kWorkThreads;
    extern __shared__ double lds[];
    L2C_TS(3, 0);
    const Geometry &G = a.geo;
    const int s = G.s, L = G.L, kd = G.kd, G0 = G.groot, dir = a.dir;
    const int nodes = 1 << kd;
    const int own = 2 * nodes - 2;
    const int U = 1 << (G0 + 2);                      // units of an item = nodes of level G0
    const int X = blockIdx.x;                         // this unit
    const int64_t item = blockIdx.y;
    const int64_t u0 = (int64_t)X << kd;              // first finest node
    const int64_t P = int64_t(1) << (L + 1);
    const int gpad = fused_gpad(s);
    const int GS = s + gpad;
    const int GXL = s * (nodes + 2) + R;              // logical per-parity input length
    const int GX = (int)fused_gx(s, kd);
    const int qpad = fused_qpad(s);
    const int QS = 2 * s + qpad;
    const int nQ = (int)fused_nq(s, kd);
    const int nP = 2 * s + 2 * R;
    const int tid = threadIdx.x;
    const int lane = tid & 63, wv = wave_id();
    const bool streamer = wv < NSW;
    const int wt = tid - 64 * NSW;                    // worker thread index
    const int ww = wv - NSW;                          // worker wave index

    double *Bl = lds;                                 // M*M
    double *Tl = Bl + M * M;                          // 2 s M
    double *gp = Tl + 2 * s * M;                      // near-field area: 2 GX input, nQ Q, nP P
    double *Ql = gp + 2 * GX;
    double *Pl = Ql + nQ;
    double *wl = gp + fused_near_area(L, M, s, kd);   // fused_wofs(kd + 1) nodes
    double *cown = wl + fused_wofs(kd + 1) * NS;      // own depths 1..kd at node 2^d - 2
    double *cR = cown + own * NS;                     // c at the unit root (ancestor chain)
    double *w7 = cR + NS;                             // top wave: z [2 x 2M], canc [(G0+1) x 2M]
    double *dummy = w7 + 4 * M + (G0 + 1) * M2;       // 2 NS: stores of out-of-range slots
    unsigned *sync = reinterpret_cast<unsigned *>(dummy + 2 * NS);
    unsigned *wcnt = sync, *rdy = sync + 1, *nbr = sync + 2, *ndone = sync + 3, *qdone = sync + 4;

    const double *in = a.in + item * a.n;
    double *wg = a.w + item * G.NT * M2;              // published nodes, workspace layout
    unsigned *fl = a.flags + item * G.NF;
    const int64_t jb = u0 * 2 * s;                    // first row of the unit
    const int nslots = (nodes - 1) * M;
    const double2 *sub = reinterpret_cast<const double2 *>(a.ahat_bot) + (int64_t)X * G.sub_groups * NCH * 64 + lane;

    unsigned wtarget = 0;
    const int nch = (s + R - 1) / R;
    const int nwork = nodes * 2 * nch;                // near-field items, <= NWT (geometry)
    double acc[R];
#pragma unroll
    for (int r = 0; r < R; ++r) acc[r] = 0.0;
    if (streamer) {
        // ---- streamers: the first group goes in flight after the workers' staging loads
        //      (issued first, they would queue behind it), then step (3)
        __syncthreads();                              // with the workers' barrier after staging
        double2 t0[NC3], t1[NC3], t2[NC3];
        if (wv < G.sub_groups) {
#pragma unroll
            for (int c = 0; c < NC3; ++c) t0[c] = sub[(wv * NCH + c) * 64];
#pragma unroll
            for (int c = 0; c < NC3; ++c) t1[c] = sub[(wv * NCH + NC3 + c) * 64];
#pragma unroll
            for (int c = 0; c < NC3; ++c) t2[c] = sub[(wv * NCH + 2 * NC3 + c) * 64];
        }
        int grp = wv;
#pragma unroll 1
        for (; grp + NSW < G.sub_groups; grp += NSW)
            stream_group<M, true>(grp, grp + NSW, sub, wl, cown, dummy, kd, nslots, lane, rdy, nbr, t0, t1, t2);
        if (grp < G.sub_groups) stream_group<M, false>(grp, 0, sub, wl, cown, dummy, kd, nslots, lane, rdy, nbr, t0, t1, t2);
        L2C_TS(3, 8);
    } else {
        // ---- workers: stage input (both parities, zero past n; cheb2leg u = c .* f), T, B(0),
        //      P and the Q table
        constexpr int UG = kFusedStageG, UT = kFusedStageT, UB = (M * M + NWT - 1) / NWT;
        double vg[UG], vt[UT], vb[UB];
        const int cntg = 2 * GXL;
#pragma unroll
        for (int u = 0; u < UG; ++u) {
            const int e = u * NWT + wt;
            const int sig = e >= GXL, x = e - sig * GXL;
            const int64_t j = jb + 2 * (int64_t)x + sig;
            vg[u] = (e < cntg && x < s * (nodes + 2) && j < a.n) ? in[j] : 0.0;
        }
#pragma unroll
        for (int u = 0; u < UT; ++u) {
            const int e = u * NWT + wt;
            vt[u] = e < 2 * s * M ? a.T[e] : 0.0;
        }
#pragma unroll
        for (int u = 0; u < UB; ++u) {
            const int e = u * NWT + wt;
            vb[u] = e < M * M ? a.B0[e] : 0.0;
        }
        const double vp = wt < nP ? a.Ptab[wt + kPLead - (R - 1)] : 0.0;
        if (wt < nP) Pl[wt] = vp;
#pragma unroll
        for (int u = 0; u < UT; ++u) {
            const int e = u * NWT + wt;
            if (e < 2 * s * M) Tl[e] = vt[u];
        }
#pragma unroll
        for (int u = 0; u < UB; ++u) {
            const int e = u * NWT + wt;
            if (e < M * M) Bl[e] = vb[u];
        }
#pragma unroll
        for (int u = 0; u < UG; ++u) {
            const int e = u * NWT + wt;
            if (e < cntg) {
                const int sig = e >= GXL, x = e - sig * GXL;
                const int64_t j = jb + 2 * (int64_t)x + sig;
                gp[sig * GX + x + (x / s) * gpad] = (dir == 1 && j == 0) ? 2.0 * vg[u] : vg[u];
            }
        }
        if (wt == 0) {
            wcnt[0] = 0;
            rdy[0] = (unsigned)kd + 1;                // no depth ready yet
            nbr[0] = 0;
            ndone[0] = 0;
            qdone[0] = 0;
        }
        __syncthreads();                              // with the streamers' barrier below
        L2C_TS(3, 1);
        // ---- step (3), own blocks.  Slot (j, k) of a group = row k of the three submatrices of
        //      block j (depth d, index i): c(2i)[k] = Ahat(.,0)[k,:] w(2i+2) + Ahat(.,1)[k,:] w(2i+3),
        //      c(2i+1)[k] = Ahat(.,2)[k,:] w(2i+3), both parities.  Rows r = 0, 1, 2 of the next
        //      group are loaded as soon as the same row of this group has been used.
        // ---- step (1): w_k(t, sigma) = sum_m T_k(X_m^sigma) f[2s t + 2m + sigma] (Eq. (wMM))
        //      for the unit's finest nodes and the next unit's first two (its finest-depth
        //      neighbours).  Worker wave -> (sigma, third of k), so a T value is the same for
        //      the whole wave (LDS broadcast); lane -> nodes lane and lane + H, H = half the
        //      node count rounded up, so every T value read feeds two products.  The last
        //      third repeats k = M-1 in its spare slots (no branches in the loop).
        {
            constexpr int KT = (M + 2) / 3;
            const int sig = ww & 1, kb = (ww >> 1) * KT;
            const double *Ts = Tl + sig * s * M;
            int kc[KT];
#pragma unroll
            for (int kk = 0; kk < KT; ++kk) kc[kk] = kb + kk < M ? kb + kk : M - 1;
            const int nall = nodes + 2, H = (nall + 1) >> 1;
            for (int n0 = lane; n0 < H; n0 += 64) {
                const int n1 = n0 + H < nall ? n0 + H : n0;     // odd count: the last lane repeats
                double a0[KT], a1[KT];
#pragma unroll
                for (int kk = 0; kk < KT; ++kk) a0[kk] = a1[kk] = 0.0;
                const double *f0 = gp + sig * GX + n0 * GS, *f1 = gp + sig * GX + n1 * GS;
#pragma unroll 4
                for (int m = 0; m < s; ++m) {
                    const double x0 = f0[m], x1 = f1[m];
#pragma unroll
                    for (int kk = 0; kk < KT; ++kk) {
                        const double t = Ts[m * M + kc[kk]];
                        a0[kk] = fma(t, x0, a0[kk]);
                        a1[kk] = fma(t, x1, a1[kk]);
                    }
                }
                double *w0 = wl + (fused_wofs(kd) + n0) * NS + sig * M;   // nodes >= 2^kd: neighbour slots
                double *w1 = wl + (fused_wofs(kd) + n1) * NS + sig * M;
#pragma unroll
                for (int kk = 0; kk < KT; ++kk)
                    if (kb + kk < M) {
                        w0[kb + kk] = a0[kk];
                        w1[kb + kk] = a1[kk];
                    }
            }
        }
        worker_sync(wcnt, wtarget, a.status);
        if (wt == 0) lds_flag_set(rdy, (unsigned)kd);
        L2C_TS(3, 2);
        // cheb2leg near field reads g_j = j u_j: scale the staged input (step (1) has read u)
        if (dir == 1) {
            for (int e = wt; e < 2 * GX; e += NWT) {
                const int sig = e >= GX, q = e - sig * GX;
                const int nd = q / GS, r = q - nd * GS;
                if (r < s) gp[e] *= (double)(jb + 2 * (int64_t)(nd * s + r) + sig);
            }
        }
        // ---- step (2) inside the unit: depth d from depth d+1 (thread <-> (pair, n)); each
        //      finished depth is flagged for the streamers
        {
            constexpr int QSTEP = NWT / M;
            const int n = wt % M, q0 = wt / M;
            const bool qn_ok = wt < M * QSTEP;
            double brow[M];
#pragma unroll
            for (int kk = 0; kk < M; ++kk) brow[kk] = Bl[(qn_ok ? n : 0) * M + kk];
            for (int d = kd - 1; d >= 0; --d) {
                if (qn_ok)
                    up_level_qn<M>(wl + fused_wofs(d + 1) * NS, wl + fused_wofs(d) * NS, 1 << d, brow, n, q0, QSTEP);
                worker_sync(wcnt, wtarget, a.status);
                if (wt == 0) lds_flag_set(rdy, (unsigned)d);
            }
        }
        L2C_TS(3, 12);
        // publish the root (level G0, node X) and nodes 0, 1 of depths 1..kd-1 (level G0 + d,
        // nodes X 2^d, X 2^d + 1), then raise the unit's flag
        {
            const int cnt = (2 * kd - 1) * M2;
            for (int e = wt; e < cnt; e += NWT) {
                const int q = e / M2, r = e - q * M2;
                const int d = q == 0 ? 0 : (q + 1) >> 1, k = q == 0 ? 0 : (q - 1) & 1;
                store_coherent(wg + (node_offset(G0 + d) + ((int64_t)X << d) + k) * M2 + r,
                               wl[(fused_wofs(d) + k) * NS + r]);
            }
            wave_stores_done();
            worker_sync(wcnt, wtarget, a.status);
            if (wt == 0) set_flag(fl + node_offset(G0) + X, a.epoch);
        }
        L2C_TS(3, 3);
        // ---- near-field Q table (off the path to the published root), by the near waves
        if (ww < kNearWaves) {
            // Q in runs of 8 consecutive S: the first value from Eq. (tau), then the exact ratio
            // Q_{S+1}/Q_S: (2S+1)/(2S+2) for leg2cheb (Eq. (Lambdaint)), 2S/(2S+3) for cheb2leg
            {
                const int QL = 2 * s * nodes + 3 * s + 2 * R;
                for (int run = wt; run * 8 < QL; run += 64 * kNearWaves) {
                    const int x0 = run * 8;
                    int node = x0 / (2 * s), c = x0 - node * 2 * s;
                    int64_t S = jb + x0;
                    double q = near_Q(dir, S);
    #pragma unroll
                    for (int i = 0; i < 8; ++i) {
                        if (x0 + i < QL) Ql[node * QS + c] = q;
                        const double Sd = (double)S;
                        q = dir == 0 ? q * ((2.0 * Sd + 1.0) / (2.0 * Sd + 2.0))
                                     : (S == 0 ? near_Q(dir, 1) : q * ((2.0 * Sd) / (2.0 * Sd + 3.0)));
                        ++S;
                        if (++c == 2 * s) {
                            c = 0;
                            ++node;
                        }
                    }
                }
            }
            // the near waves' own barrier: Q complete before any of them reads it
            wave_lds_done();
            if (lane == 0) {
                __hip_atomic_fetch_add(qdone, 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
                int it = 0;
                while (lds_flag_get(qdone) < (unsigned)kNearWaves) {
                    __builtin_amdgcn_s_sleep(1);
                    if (++it == kSpinLimit) {
                        atomicOr(a.status, 2);
                        break;
                    }
                }
            }
            __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "workgroup");
        }
        // ---- nodes 0, 1 of the next unit at depths 1..kd-1 (one worker wave; the streamers
        //      wait for this only when they reach those depths)
        if (ww == kWorkWaves - 2) {
            const int cnt = 2 * (kd - 1) * M2;
            const bool have = X + 1 < U;
            if (have) wave_wait_flag(fl + node_offset(G0) + X + 1, a.epoch, a.status);
            for (int e = lane; e < cnt; e += 64) {
                const int q = e / M2, r = e - q * M2;
                const int d = (q >> 1) + 1, k = q & 1;
                const double v =
                    have ? load_coherent(wg + (node_offset(G0 + d) + ((int64_t)(X + 1) << d) + k) * M2 + r) : 0.0;
                wl[(fused_wofs(d) + (1 << d) + k) * NS + r] = v;
            }
            wave_lds_done();
            if (lane == 0) lds_flag_set(nbr, 1u);
        }
        // ---- step (6): near field.  Item (node nd, parity sig, rows m0 .. m0+R-1): row m sums
        //      over m' in [m, 2s): P[m'-m] Q[2s u + sig + m + m'] g[2s u + 2m' + sig], with P, Q
        //      and g entering through circular register windows; the sums stay in registers
        //      until the leaf evaluation.
        if (ww < kNearWaves && wt < nwork) {
            const int nd = wt % nodes, x = wt / nodes;
            const int sig = x & 1, m0 = (x >> 1) * R;
            const double *gs = gp + sig * GX + nd * GS;
            const double *qs = Ql + nd * QS;
            const double *ps = Pl + (R - 1) - m0;
            double pb[R], qb[R];
#pragma unroll
            for (int r = 0; r < R; ++r) pb[r] = 0.0;
            // window slots are compile-time: slot t of a step holds m' = mb + t (m0 is a multiple of R)
#pragma unroll
            for (int r = 0; r < R - 1; ++r) {
                const int c = sig + 2 * m0 + r;
                qb[r] = qs[c + (c >= 2 * s ? qpad : 0)];
            }
            const int steps = ((2 * s - m0) + R - 1) / R;
            for (int st = 0; st < steps; ++st) {
                const int mb = m0 + st * R;
                const bool tail = mb + R > 2 * s;
#pragma unroll
                for (int t = 0; t < R; ++t) {
                    const int mp = mb + t;
                    pb[t] = ps[mp];
                    const int c = sig + m0 + mp + R - 1;
                    qb[(t + R - 1) % R] = qs[c + (c >= 2 * s ? qpad : 0)];
                    double gv = gs[mp + (mp >= s ? gpad : 0) + (mp >= 2 * s ? gpad : 0)];
                    if (tail && mp >= 2 * s) gv = 0.0;
#pragma unroll
                    for (int r = 0; r < R; ++r) acc[r] = fma(pb[(t - r + R) % R] * qb[(t + r) % R], gv, acc[r]);
                }
            }
        }
        if (ww < kNearWaves) {
            wave_lds_done();                          // the near-field area is free once all have counted
            if (lane == 0) __hip_atomic_fetch_add(ndone, 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
        }
        L2C_TS(3, 4);
        if (ww == kWorkWaves - 1) {
        // ---- top wave; lane (sg, nn) <-> parity and mode
        const bool act = lane < M2;
        const int sg = lane >= M ? 1 : 0, nn = act ? lane - sg * M : 0;
        double *zb = w7;                              // z0 [2M], z1 [2M]
        double *canc = w7 + 2 * M2;                   // (G0 + 1) x 2M
        // step (2) above the units.  Unit X with kown = min(G0, trailing zeros of X) >= 1 is
        // the leftmost unit below its ancestors at levels G0-1 .. G0-kown and publishes
        // them.  It reduces kHopLevels levels per exchange: it waits for the other
        // 2^kHopLevels - 1 nodes of the input level below its next ancestor (published by
        // their own leftmost units), reduces them in the (now free) near-field area, and
        // publishes the new nodes.  With groot <= 6 that is at most two exchanges.
        {
            constexpr int kHopLevels = 3;
            const int kown = X == 0 ? G0 : min(G0, __ffs(X) - 1);
            double brow[M];
#pragma unroll
            for (int kk = 0; kk < M; ++kk) brow[kk] = Bl[nn * M + kk];
            double cur = act ? wl[lane] : 0.0;                  // this unit's node at the input level
            for (int jdone = 0; jdone < kown;) {
                const int jn = min(kown, jdone + kHopLevels);
                const int gin = G0 - jdone;                      // input level
                const int nin = 1 << (jn - jdone);               // input nodes t0 .. t0 + nin - 1
                const int64_t t0 = (int64_t)X >> jdone;
                double *src = Tl, *dst = Tl + nin * NS;          // ping-pong node buffers (T area)
                {
                    bool done = lane >= nin - 1;                 // lane i waits for node t0 + 1 + i
                    for (int it = 0; it < kSpinLimit; ++it) {
                        if (!done)
                            done = __hip_atomic_load(fl + node_offset(gin) + t0 + 1 + lane, __ATOMIC_RELAXED,
                                                     __HIP_MEMORY_SCOPE_AGENT) == a.epoch;
                        if (__all(done)) break;
                        __builtin_amdgcn_s_sleep(1);
                    }
                    if (!done) atomicOr(a.status, 1);
                    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "workgroup");
                }
                {
                    // nin <= 8 nodes of 2M values: UL loads per lane
                    constexpr int UL = (8 * M2 + 63) / 64;
                    double v[UL];
#pragma unroll
                    for (int u = 0; u < UL; ++u) {
                        const int idx = u * 64 + lane;
                        const int r = idx / M2, e = idx - r * M2;
                        v[u] = (idx < nin * M2 && r > 0) ? load_coherent(wg + (node_offset(gin) + t0 + r) * M2 + e) : 0.0;
                    }
#pragma unroll
                    for (int u = 0; u < UL; ++u) {
                        const int idx = u * 64 + lane;
                        const int r = idx / M2, e = idx - r * M2;
                        if (idx < nin * M2 && r > 0) src[r * NS + e] = v[u];
                    }
                    if (act) src[lane] = cur;
                }
                wave_lds_sync();
                for (int j = jdone + 1; j <= jn; ++j) {
                    const int pn = nin >> (j - jdone);
                    for (int pp = 0; pp < pn; ++pp) {
                        const double *x = src + (2 * pp) * NS + sg * M;
                        const double v = up_pair<M>(brow, x, x + NS, nn);
                        if (act) dst[pp * NS + lane] = v;
                    }
                    wave_lds_sync();
                    cur = act ? dst[lane] : 0.0;
                    if (act) store_coherent(wg + (node_offset(G0 - j) + (X >> j)) * M2 + lane, cur);
                    double *t = src;
                    src = dst;
                    dst = t;
                }
                wave_stores_done();
                if (lane == 0)
                    for (int j = jdone + 1; j <= jn; ++j) set_flag(fl + node_offset(G0 - j) + (X >> j), a.epoch);
                jdone = jn;
                wave_lds_sync();
            }
        }
        // T back into its area (the leaf evaluation needs it) and the ancestors' submatrices
        // (step (3) below) in one batch of loads; then wait until the near field has
        // released the near-field area.  Slot sl = 2g + h of level g holds submatrix r = 2p
        // (h = 0, column node a_g + 2) or r = 1 (h = 1, p = 0 only, column node a_g + 3).
        const int nsl = 2 * (G0 + 1);
        auto slot_ok = [&](int sl) -> bool {
            const int g = sl >> 1;
            const int64_t an = (int64_t)X >> (G0 - g);
            return an < (int64_t(1) << (g + 2)) - 2 && ((sl & 1) == 0 || (an & 1) == 0);
        };
        auto slot_node = [&](int sl) -> int64_t {
            const int g = sl >> 1;
            return node_offset(g) + ((int64_t)X >> (G0 - g)) + 2 + (sl & 1);
        };
        constexpr int UAT = (14 * M * M + 63) / 64;   // groot <= 6: at most 14 slots
        constexpr int UTT = (2 * 33 * M + 63) / 64;   // 2 s M, s <= 33
        double va[UAT];
        {
            double vt[UTT];
#pragma unroll
            for (int u = 0; u < UTT; ++u) {
                const int e = u * 64 + lane;
                vt[u] = e < 2 * s * M ? a.T[e] : 0.0;
            }
#pragma unroll
            for (int u = 0; u < UAT; ++u) {
                const int idx = u * 64 + lane;
                const int sl = idx / (M * M), e = idx - sl * (M * M);
                double x = 0.0;
                if (idx < nsl * M * M && slot_ok(sl)) {
                    const int g = sl >> 1;
                    const int64_t an = (int64_t)X >> (G0 - g);
                    const int r = (sl & 1) ? 1 : 2 * (int)(an & 1);
                    x = a.ahat_top[((level_block_offset(g) + (an >> 1)) * 3 + r) * M * M + e];
                }
                va[u] = x;
            }
#pragma unroll
            for (int u = 0; u < UTT; ++u) {
                const int e = u * 64 + lane;
                if (e < 2 * s * M) Tl[e] = vt[u];
            }
            if (lane == 0) {
                int it = 0;
                while (lds_flag_get(ndone) < (unsigned)kNearWaves) {
                    __builtin_amdgcn_s_sleep(1);
                    if (++it == kSpinLimit) {
                        atomicOr(a.status, 2);
                        break;
                    }
                }
            }
            __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "workgroup");
        }
        // step (3) for the ancestors a_g = X >> (G0 - g), g = 0..G0 (top table), from LDS once
        // every column node is flagged and loaded
        {
            double *colw = gp;                             // nsl x 2M
            double *atop = gp + nsl * M2;                  // nsl x M x M
#pragma unroll
            for (int u = 0; u < UAT; ++u) {
                const int idx = u * 64 + lane;
                if (idx < nsl * M * M) atop[idx] = va[u];
            }
            // every column node flagged (lane sl polls slot sl)
            {
                bool done = lane >= nsl || !slot_ok(lane);
                for (int it = 0; it < kSpinLimit; ++it) {
                    if (!done)
                        done = __hip_atomic_load(fl + slot_node(lane), __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) ==
                               a.epoch;
                    if (__all(done)) break;
                    __builtin_amdgcn_s_sleep(1);
                }
                if (!done) atomicOr(a.status, 1);
                __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "workgroup");
            }
            for (int base = 0; base < nsl * M2; base += 8 * 64) {
                double v[8];
#pragma unroll
                for (int u = 0; u < 8; ++u) {
                    const int idx = base + u * 64 + lane;
                    const int sl = idx / M2, e = idx - sl * M2;
                    v[u] = (idx < nsl * M2 && slot_ok(sl)) ? load_coherent(wg + slot_node(sl) * M2 + e) : 0.0;
                }
#pragma unroll
                for (int u = 0; u < 8; ++u) {
                    const int idx = base + u * 64 + lane;
                    if (idx < nsl * M2) colw[idx] = v[u];
                }
            }
            wave_lds_sync();
            for (int g = 0; g <= G0; ++g) {
                const double *A0 = atop + (2 * g) * M * M + nn * M, *A1 = A0 + M * M;
                const double *x0 = colw + (2 * g) * M2 + sg * M, *x1 = x0 + M2;
                double c0 = 0.0, c1 = 0.0;
#pragma unroll
                for (int l = 0; l < M; ++l) {
                    c0 = fma(A0[l], x0[l], c0);
                    c1 = fma(A1[l], x1[l], c1);
                }
                if (act) canc[g * M2 + lane] = c0 + c1;
            }
        }
        wave_lds_sync();
        // step (4) along the chain: c(a_g) += B(p)^T c(a_{g-1}), p = a_g & 1
        {
            double bcol[M];
#pragma unroll
            for (int k = 0; k < M; ++k) bcol[k] = Bl[k * M + nn];
            double cc = act ? canc[lane] : 0.0;
            for (int g = 1; g <= G0; ++g) {
                const int p = (int)((X >> (G0 - g)) & 1);
                if (act) zb[lane] = cc;
                wave_lds_sync();
                double acc2 = 0.0;
#pragma unroll
                for (int k = 0; k < M; ++k) {
                    const double v = zb[sg * M + k];
                    acc2 = fma(bcol[k], (p && (k & 1)) ? -v : v, acc2);
                }
                wave_lds_sync();
                cc = (act ? canc[g * M2 + lane] : 0.0) + ((p && (nn & 1)) ? -acc2 : acc2);
            }
            if (act) cR[lane] = cc;
        }
        }
    }
    __syncthreads();
    L2C_TS(3, 5);

    // ---- step (4) inside the unit: depth d from depth d-1 (depth 0 = the root's cR)
    {
        constexpr int QSTEP = NTH / M;
        const int n = tid % M, q0 = tid / M;
        const bool qn_ok = tid < M * QSTEP;
        double bcol[M];
#pragma unroll
        for (int k = 0; k < M; ++k) bcol[k] = Bl[k * M + (qn_ok ? n : 0)];
        for (int d = 1; d <= kd; ++d) {
            const int cn = 1 << d;
            const double *parb = d == 1 ? cR : cown + ((cn >> 1) - 2) * NS;
            if (2 * cn <= QSTEP) {
                if (qn_ok) down_level_qn<M>(parb, cown + (cn - 2) * NS, cn, -1, bcol, n, q0, QSTEP);
            } else {
                down_level<M>(parb, cown + (cn - 2) * NS, cn, -1, Bl);
            }
            __syncthreads();
        }
    }
    const double *cfine = cown + (nodes - 2) * NS;
    L2C_TS(3, 6);

    // ---- steps (5) and (7): z = sum_k T_k(X_m^sig) c(u)[sig][k] (row nodes u < P - 2)
    //      + rs * near; leg2cheb divides by c_i pi/2
    double *out = a.out + item * a.n;
    if (!streamer && ww < kNearWaves && wt < nwork) {
        auto eval = [&](int nd, int sig, int m0) {
            const bool far = u0 + nd < P - 2;
            double cc[M];
            const double *cs = cfine + nd * NS + sig * M;
#pragma unroll
            for (int k = 0; k < M; ++k) cc[k] = cs[k];
#pragma unroll
            for (int r = 0; r < R; ++r) {
                const int m = m0 + r;
                if (m < s) {
                    double z = 0.0;
                    if (far) {
                        const double *tt = Tl + (sig * s + m) * M;
#pragma unroll
                        for (int k = 0; k < M; ++k) z = fma(tt[k], cc[k], z);
                    }
                    const int64_t i = jb + nd * 2 * s + 2 * m + sig;
                    double v = acc[r];
                    if (dir == 1) {
                        v *= 2.0 * (double)i + 1.0;
                        if (i == 0) v += in[0];      // K_00 u_0 = u_0 / 2 = f_0
                    }
                    v += z;
                    if (dir == 0) v /= (i == 0 ? kPi : 0.5 * kPi);
                    if (i < a.n) out[i] = v;
                }
            }
        };
        if (nodes == 64) {
            // a wave holds one (parity, row block) for 64 nodes: T rows are wave-uniform
            const int x = __builtin_amdgcn_readfirstlane(ww);
            eval(lane, x & 1, (x >> 1) * R);
        } else {
            const int x = wt / nodes;
            eval(wt % nodes, x & 1, (x >> 1) * R);
        }
    }
    L2C_TS(3, 7);
}

// ------------------------------------------------------------------------------------
bool fused_supported(int M) { return 2 * M <= 64; }

static size_t fused_lds_bytes(const Geometry &G)
{
    return sizeof(double) * (size_t)fused_lds_doubles(G.L, G.M, G.s, G.kd);
}

template <int M>
static const void *fused_fn()
{
    return (const void *)k_fused<M>;
}

static const void *fused_kernel(int M)
{
    switch (M) {
#define L2C_CASE(MM) \
    case MM: return fused_fn<MM>();
        L2C_FOR_EACH_RANK(L2C_CASE)
#undef L2C_CASE
    default: return nullptr;
    }
}

// Items per launch such that every workgroup is resident at once (0: path unavailable).
hipError_t fused_max_items(const l2c_plan_s &p, int64_t *items)
{
    *items = 0;
    const Geometry &G = p.geo;
    if (p.L < 2 || G.kd < 1 || !fused_supported(p.M)) return hipSuccess;
    const int nodes = 1 << G.kd, R = kFusedRows;
    if (nodes * 2 * ((G.s + R - 1) / R) > 64 * kNearWaves) return hipSuccess;          // near-field items
    if (12 * (2 * G.M + 1) > 2 * G.s * G.M) return hipSuccess;                         // hop scratch in T area
    if (G.s > 33 || G.groot > 6) return hipSuccess;                                      // top wave's load batches
    if (2 * (G.s * (nodes + 2) + R) > kFusedStageG * kWorkThreads) return hipSuccess;  // input staging
    if (2 * G.s * G.M > kFusedStageT * kWorkThreads) return hipSuccess;                // T staging
    if (2 * G.s + 2 * R > kWorkThreads) return hipSuccess;                             // P staging
    const size_t lds = fused_lds_bytes(G);
    if (lds > (size_t)kMainLds) return hipSuccess;
    const void *fn = fused_kernel(p.M);
    if (!fn) return hipSuccess;
    hipError_t e = hipFuncSetAttribute(fn, hipFuncAttributeMaxDynamicSharedMemorySize, kMainLds);
    if (e != hipSuccess) return e;
    int per_cu = 0, cus = 0;
    e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, fn, kFusedThreads, lds);
    if (e != hipSuccess) return e;
    e = hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, p.device);
    if (e != hipSuccess) return e;
    const int64_t resident = (int64_t)per_cu * cus;
    const int64_t U = int64_t(1) << (G.groot + 2);
    *items = resident / U;
    return hipSuccess;
}

// Single-launch kernels of one device never overlap: a launch on a stream other than the
// previous one waits for the previous launch.
namespace {
struct FusedOrder {
    std::mutex mu;
    hipStream_t last = nullptr;
    hipEvent_t done = nullptr;
    bool any = false;
};
FusedOrder g_order[64];
}  // namespace

template <int M>
static hipError_t run_fused(l2c_plan_s &p, const double *in, double *out, int64_t batch, hipStream_t st)
{
    const Geometry &G = p.geo;
    ExecArgs a;
    a.n = p.n;
    a.dir = p.direction;
    a.geo = G;
    a.T = p.d_T;
    a.B0 = p.d_B;
    a.Ptab = p.d_P;
    a.ahat_top = p.d_top;
    a.ahat_bot = p.d_bot;
    a.w = p.d_w;
    a.flags = p.d_flags;
    a.status = p.d_status;
    const size_t lds = fused_lds_bytes(G);
    const unsigned U = 1u << (G.groot + 2);
    FusedOrder &o = g_order[p.device & 63];
    std::lock_guard<std::mutex> lock(o.mu);
    if (!o.done) {
        hipError_t e = hipEventCreateWithFlags(&o.done, hipEventDisableTiming);
        if (e != hipSuccess) return e;
    }
    if (o.any && o.last != st) {
        hipError_t e = hipStreamWaitEvent(st, o.done, 0);
        if (e != hipSuccess) return e;
    }
    for (int64_t b0 = 0; b0 < batch; b0 += p.fused_items) {
        ExecArgs c = a;
        c.batch = batch - b0 < p.fused_items ? batch - b0 : p.fused_items;
        c.in = in + b0 * p.n;
        c.out = out + b0 * p.n;
        c.epoch = ++p.epoch;
        if (c.epoch == 0) c.epoch = ++p.epoch;    // 0 is the value of never-written flags
        const bool timed = p.ev_before && p.ev_after && b0 == 0;
        if (timed) (void)hipEventRecord(p.ev_before, st);
        hipLaunchKernelGGL(k_fused<M>, dim3(U, (unsigned)c.batch), dim3(kFusedThreads), lds, st, c);
        if (timed) (void)hipEventRecord(p.ev_after, st);
    }
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    e = hipEventRecord(o.done, st);
    o.last = st;
    o.any = true;
    return e;
}

hipError_t launch_fused(l2c_plan_s &p, const double *in, double *out, int64_t batch, hipStream_t st)
{
    switch (p.M) {
#define L2C_CASE(MM) \
    case MM: return run_fused<MM>(p, in, out, batch, st);
        L2C_FOR_EACH_RANK(L2C_CASE)
#undef L2C_CASE
    default: return hipErrorInvalidValue;
    }
}

}  // namespace l2c
