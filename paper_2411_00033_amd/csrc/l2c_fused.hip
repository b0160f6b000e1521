// l2c_fused.hip -- single-launch execution of Alg. 4 (steps (0)-(7)) for gfx950, FP64.
//
// One workgroup per subtree ("unit") of 2^kd finest nodes below node X of level
// groot = L-1-kd, all units of an item resident at once (one workgroup per CU).  A unit
// needs from the rest of the grid only
//   * nodes 0 and 1 of the next unit at every depth (its own far-field blocks reach two
//     nodes past its right edge, Eq. (globalij)); at the finest depth it computes them
//     itself from the input, at coarser depths it reads them, and
//   * the upward vectors of levels 0..groot, which combine every unit's root.
// Both travel through an exchange buffer of two halves, used by alternate launches.  A
// value not yet written holds a signalling NaN that no arithmetic produces, so a reader
// polls the data itself: once no value it loaded is that NaN, it has all of them (64-bit
// device-coherent stores and loads are single-copy atomic).  Each unit resets its own
// nodes in the other half for the next launch.  Nothing else crosses workgroups.
//
// Inside a workgroup the waves specialise.
//   The streamer (wave 0) reads the unit's far-field table (the dominant HBM traffic)
//   once the workers' staging loads are out, one 64-slot group (27.6 KiB at M = 18) in
//   flight: enough to keep HBM busy without queueing requests so deep that every other
//   memory access of the kernel waits behind them.  The table is laid out finest depth
//   first, and a group is multiplied (step (3)) as soon as the workers flag its depths
//   ready.  Workers (waves 1..7) stage the input, B(0), T and the near-field tables;
//   step (1) for the unit's finest nodes (and two of the next unit); step (2) inside the
//   unit, flagging each depth; publish the root and nodes 0, 1 of every coarser depth;
//   fetch the next unit's nodes (one wave); step (6), the near field (six waves).  Meanwhile
//   the last worker wave does step (2) above the units (the leftmost unit below an
//   ancestor at most three levels up reduces the roots under it and publishes it) and
//   collects the tree-top nodes the unit needs; once the near field is done, all worker
//   waves reduce those, form the far-field blocks of the unit's ancestors (step (3), top
//   table), and the last one runs the downward chain from level 0 to the unit root
//   (step (4)).  Workers synchronise through LDS counters, streamers poll LDS flags;
//   there is no hardware barrier between the first and the last phase.
//   Then all waves: step (4) inside the unit, steps (5) and (7), and the output.
// Every wait is bounded on the device's wall clock: one that never completes (another
// kernel holding CUs forever) gives up and sets a status word, and the launch then ends
// with a wrong result instead of hanging; the host reports the word (the next execute of
// the plan returns an error).  The waits for other workgroups have a bound of their own
// that the host can lower, which tests use to force this path.  The host keeps
// single-launch kernels of different streams from overlapping, so every workgroup of a
// launch becomes resident.
#include <mutex>
#include <vector>

#include "l2c_alloc.h"
#include "l2c_device.h"

namespace l2c {

typedef double d4_t __attribute__((ext_vector_type(4)));   // FP64 MFMA accumulator

__device__ __forceinline__ void store_coherent(double *p, double v)
{
    __hip_atomic_store(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

__device__ __forceinline__ double load_coherent(const double *p)
{
    return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

// LDS written by some lanes of a wave and then read by other lanes of the same wave:
// LDS executes a wave's operations in order; this keeps the compiler from reordering.
__device__ __forceinline__ void wave_lds_sync() { __builtin_amdgcn_fence(__ATOMIC_ACQ_REL, "wavefront"); }

// Wait until this wave's LDS operations are complete (s_waitcnt lgkmcnt(0)).  The fence
// orders LDS only: a workgroup-wide fence would also wait for the wave's outstanding global
// stores (exchange nodes on their way to other workgroups), which nothing here depends on.
__device__ __forceinline__ void wave_lds_done()
{
    __builtin_amdgcn_s_waitcnt(0xc07f);
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "workgroup", "local");
}

// The reader's side: LDS written by other waves before their release is visible.
__device__ __forceinline__ void lds_acquire() { __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "workgroup", "local"); }

// Barrier of the worker waves only (LDS counter; target is this wave's running count).
__device__ __forceinline__ void worker_sync(unsigned *cnt, unsigned &target, const ExecArgs &a)
{
    wave_lds_done();
    target += kWorkWaves;
    if ((threadIdx.x & 63) == 0) {
        __hip_atomic_fetch_add(cnt, 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
        WaitClock wc;
        for (int it = 1; __hip_atomic_load(cnt, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP) < target; ++it) {
            __builtin_amdgcn_s_sleep(1);
            if ((it & 15) == 0 && wc.expired(a.wait_ticks)) {
                raise_status(a.status, kStatusWorkers);
                break;
            }
        }
    }
    lds_acquire();
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
__device__ __forceinline__ void stream_group(const ExecArgs &ea, int grp, int nxt, const double2 *sub, const double *wl,
                                             double *cown, double *dummy, int kd, int nslots, int lane,
                                             const unsigned *rdy, const unsigned *nbr,
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
    {
        WaitClock wc;
        for (int it = 1; !(lds_flag_get(rdy) <= (unsigned)dlo && (dlo == kd || lds_flag_get(nbr) != 0)); ++it) {
            __builtin_amdgcn_s_sleep(1);
            if ((it & 15) == 0 && wc.expired(ea.wait_ticks)) {
                raise_status(ea.status, kStatusStream);
                break;
            }
        }
    }
    lds_acquire();
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

// Exchange nodes hold pub_empty() until the current launch writes them (the buffer half
// of the next launch is reset to it during this one); any other value is final.
__device__ __forceinline__ double pub_empty()
{
    return __longlong_as_double((long long)(((unsigned long long)kPubEmptyHalf << 32) | kPubEmptyHalf));
}

__device__ __forceinline__ bool pub_ready(double v)
{
    return __double_as_longlong(v) != (long long)(((unsigned long long)kPubEmptyHalf << 32) | kPubEmptyHalf);
}

// v[u] = p[off(u)] for every u with want(u), loaded again until no such value is empty
// (bounded; a wave-uniform exit).  Entries without want(u) keep their value.
template <int NU, class Want, class Off>
__device__ __forceinline__ void poll_values(double (&v)[NU], const double *p, const Want &want, const Off &off,
                                            const ExecArgs &a)
{
#pragma unroll
    for (int u = 0; u < NU; ++u)
        if (want(u)) v[u] = pub_empty();
    WaitClock wc;
    for (int it = 1;; ++it) {
#pragma unroll
        for (int u = 0; u < NU; ++u)
            if (want(u) && !pub_ready(v[u])) v[u] = load_coherent(p + off(u));
        bool ok = true;
#pragma unroll
        for (int u = 0; u < NU; ++u) ok = ok && (!want(u) || pub_ready(v[u]));
        // a bound of 0 (a test of this error path) gives up at the first poll, always
        if (a.poll_ticks == 0 || (!__all(ok) && (it & 7) == 0 && wc.expired(a.poll_ticks))) {
            raise_status(a.status, kStatusExchange);
            break;
        }
        if (__all(ok)) break;
        __builtin_amdgcn_s_sleep(1);
    }
}

// The far-field blocks of unit X's ancestors a_g = X >> (G0 - g), g = 0..G0 (top table):
// slot sl = 2g + h holds submatrix r = 2 (a_g & 1) with column node a_g + 2 (h = 0), or
// r = 1 with column node a_g + 3 (h = 1, a_g even only); a block exists while its column
// node lies inside level g.  Column nodes at levels g >= gl = G0 - min(3, G0) are exchange
// nodes; below gl the workgroup reduces each from the 2^(gl-g) level-gl nodes under it.
// Item i of the workgroup's list is one exchange node; a slot's items are consecutive.
struct TopSlots {
    int X, G0, H, gl, nsl;
    __host__ __device__ TopSlots(int X_, int G0_) : X(X_), G0(G0_)
    {
        H = G0 < 3 ? G0 : 3;
        gl = G0 - H;
        nsl = 2 * (G0 + 1);
    }
    __host__ __device__ int64_t anc(int g) const { return (int64_t)X >> (G0 - g); }
    __host__ __device__ bool ok(int sl) const
    {
        const int64_t an = anc(sl >> 1);
        return an < (int64_t(1) << ((sl >> 1) + 2)) - 2 && ((sl & 1) == 0 || (an & 1) == 0);
    }
    __host__ __device__ int64_t col(int sl) const { return anc(sl >> 1) + 2 + (sl & 1); }
    __host__ __device__ int cnt(int sl) const { return (sl >> 1) >= gl ? 1 : 1 << (gl - (sl >> 1)); }
};

// The per-unit tree-top table (kTopSchedInts ints, built on the host at plan time; each
// worker wave holds entries 0..63 as one int per lane and reads them by lane shuffles,
// the top wave also entries 64.. (the item nodes, one per lane)):
//   [0, 3)            pairs of reduction round r = 1, 2, 3
//   [3, 45)           round r's pairs: the item of each pair's left child (14 per round)
//   [45, 59)          each slot's first item (-1: no block)
//   [59]              nitem, the tree-top items the unit loads
//   [64, 64 + nitem)  item i's exchange node
constexpr int kSchPairs = 3, kSchBase = kSchPairs + 3 * 14, kSchItems = kSchBase + 14, kSchNodes = 64;
static_assert(kSchItems < kSchNodes && kSchNodes + 36 <= kTopSchedInts, "tree-top table layout");

void top_table_unit(int X, int G0, int *rec)
{
    const TopSlots ts(X, G0);
    for (int i = 0; i < kTopSchedInts; ++i) rec[i] = 0;
    for (int r = 1; r <= 3; ++r) {
        const int step = 1 << r;
        int t = 0, base = 0;
        for (int sl = 0; sl < ts.nsl; ++sl) {
            if (!ts.ok(sl)) continue;
            const int c = ts.cnt(sl);
            if (r <= ts.gl)
                for (int pp = 0; pp + step <= c; pp += step) rec[kSchPairs + 14 * (r - 1) + t++] = base + pp;
            base += c;
        }
        rec[r - 1] = t;
    }
    int base = 0;
    for (int sl = 0; sl < 14; ++sl) {
        const bool ok = sl < ts.nsl && ts.ok(sl);
        rec[kSchBase + sl] = ok ? base : -1;
        base += ok ? ts.cnt(sl) : 0;
    }
    int nitem = 0;
    for (int sl = 0; sl < ts.nsl; ++sl) {
        if (!ts.ok(sl)) continue;
        const int g = sl >> 1;
        for (int i = 0; i < ts.cnt(sl); ++i)
            rec[kSchNodes + nitem++] = g >= ts.gl ? (int)(node_offset(g) + ts.col(sl))
                                                  : (int)(node_offset(ts.gl) + (ts.col(sl) << (ts.gl - g)) + i);
    }
    rec[kSchItems] = nitem;
}

// wave-uniform entry i < 64 of the table held as entry lane of every lane
__device__ __forceinline__ int sched_at(int lo, int i) { return __shfl(lo, i); }

// The top wave of unit X, while the near field runs, up to the point where the workgroup's
// tree-top items sit in LDS (itm, nitem x NS, in the T area, which step (1) no longer needs):
//   1. Nodes 0, 1 of the next unit at depths 1..kd-1 into wl (the streamer waits for them
//      only when it reaches those depths), and step (2) above the units: unit X with
//      k = min(3, G0, trailing zeros of X) >= 1 is the leftmost unit below its ancestors at
//      levels G0-1 .. G0-k; it reduces the roots of units X .. X+2^k-1 in the scratch xs and
//      writes those ancestors to the exchange buffer.  Both inputs come in one poll.
//   2. The items: wait until every one of them is written, loading it in the same polls.
template <int M>
__device__ __forceinline__ void top_gather(const ExecArgs &a, const TopSlots &ts, int kd, int U, int64_t nbase,
                                           double *wl, double *xs, double *itm, const double *Bl, double *pubc,
                                           unsigned *nbr, int sch_lo, int lane)
{
    constexpr int M2 = 2 * M, NS = lds_ns<M>();
    const int X = ts.X, G0 = ts.G0;
    const bool act = lane < M2;
    const int sg = lane >= M ? 1 : 0, nn = act ? lane - sg * M : 0;
    // item i's exchange node, lane i (used after the first poll)
    const int mine = a.top_sched[(int64_t)X * kTopSchedInts + kSchNodes + lane];
    const int kx = X == 0 ? G0 : min(G0, __ffs(X) - 1);
    const int k = kx < ts.H ? kx : ts.H;
    const int nin = 1 << k;                           // roots X .. X + nin - 1 (k = 0: none)
    {
        constexpr int UN = (12 * M2 + 63) / 64;       // next unit's nodes, kd <= 7
        constexpr int UL = (8 * M2 + 63) / 64;        // roots
        const int cntn = X + 1 < U ? 2 * (kd - 1) * M2 : 0;
        const int nb1 = (int)((nbase + 2 * (kd - 1)) * M2), rb = (int)((node_offset(G0) + X) * M2);
        double v[UN + UL];
#pragma unroll
        for (int u = 0; u < UN + UL; ++u) {
            const int idx = (u - UN) * 64 + lane;
            v[u] = (u >= UN && idx < M2) ? wl[idx] : 0.0;   // root X is this unit's
        }
        poll_values(
            v, pubc,
            [&](int u) {
                const int idx = (u < UN ? u : u - UN) * 64 + lane;
                return u < UN ? idx < cntn : (k >= 1 && idx >= M2 && idx < nin * M2);
            },
            [&](int u) { return u < UN ? nb1 + u * 64 + lane : rb + (u - UN) * 64 + lane; }, a);
        L2C_TS(3, 11);
#pragma unroll
        for (int u = 0; u < UN; ++u) {
            const int e = u * 64 + lane;
            if (e < 2 * (kd - 1) * M2) {
                const int q = e / M2, r = e - q * M2;
                const int d = (q >> 1) + 1, kk = q & 1;
                wl[(fused_wofs(d) + (1 << d) + kk) * NS + r] = v[u];
            }
        }
#pragma unroll
        for (int u = UN; u < UN + UL; ++u) {
            const int idx = (u - UN) * 64 + lane;
            const int r = idx / M2, e = idx - r * M2;
            if (k >= 1 && idx < nin * M2) xs[r * NS + e] = v[u];
        }
        wave_lds_done();
        if (lane == 0) lds_flag_set(nbr, 1u);
    }
    if (k >= 1) {
        double brow[M];
#pragma unroll
        for (int kk = 0; kk < M; ++kk) brow[kk] = Bl[nn * M + kk];
        for (int j = 1; j <= k; ++j) {
            const int step = 1 << j;                  // parents at nodes 0, step, 2 step, ... (in place)
            for (int pp = 0; pp < nin; pp += step) {
                const double *x = xs + pp * NS + sg * M, *y = xs + (pp + (step >> 1)) * NS + sg * M;
                const double v2 = up_pair<M>(brow, x, y, nn);
                if (act) xs[pp * NS + lane] = v2;
                wave_lds_sync();
            }
            if (act) store_coherent(pubc + (node_offset(G0 - j) + (X >> j)) * M2 + lane, xs[lane]);
        }
    }
    L2C_TS(3, 13);
    // 2. items: lane i < nitem holds the exchange node of item i (the unit's table)
    const int nitem = sched_at(sch_lo, kSchItems);
    constexpr int UC = (36 * M2 + 63) / 64;           // at most 36 items (groot <= 6)
    double vc[UC];
    int nid[UC];
#pragma unroll
    for (int u = 0; u < UC; ++u) {
        const int i = (u * 64 + lane) / M2;
        nid[u] = __shfl(mine, i < 63 ? i : 63);
        vc[u] = 0.0;
    }
    poll_values(
        vc, pubc, [&](int u) { return (u * 64 + lane) / M2 < nitem; },
        [&](int u) { return nid[u] * M2 + (u * 64 + lane) % M2; }, a);
    L2C_TS(3, 14);
#pragma unroll
    for (int u = 0; u < UC; ++u) {
        const int idx = u * 64 + lane;
        const int i = idx / M2, e = idx - i * M2;
        if (i < nitem) itm[i * NS + e] = vc[u];
    }
}

// All worker waves, once the items and the schedule are in LDS (after a worker barrier):
//   3. the column nodes below level gl, reduced in place (pairwise, level by level; the
//      pairs of a level are spread over the waves, a barrier between levels); a slot's
//      column node ends up at its first item;
//   4. wave g <= G0: canc_g = the ancestor a_g's far-field blocks times their column
//      nodes (the submatrices ag0, ag1 are this wave's rows nn, loaded beforehand);
//   5. the top wave: the chain of step (4) from level 0 down to the unit root,
//      c(a_g) = canc_g + B(p)^T c(a_{g-1}), p = a_g & 1, into cR.
template <int M>
__device__ __forceinline__ void top_combine(const ExecArgs &a, const TopSlots &ts, double *itm, int sch_lo,
                                            const double (&ag0)[M], const double (&ag1)[M], double *canc,
                                            double *zb, double *cR, const double *Bl, unsigned *wcnt,
                                            unsigned &wtarget, int ww, bool top, int lane)
{
    constexpr int M2 = 2 * M, NS = lds_ns<M>();
    const bool act = lane < M2;
    const int sg = lane >= M ? 1 : 0, nn = act ? lane - sg * M : 0;
    if (ts.gl > 0) {
        double brow[M];
#pragma unroll
        for (int kk = 0; kk < M; ++kk) brow[kk] = Bl[nn * M + kk];
        for (int r = 1; r <= ts.gl; ++r) {
            const int np = sched_at(sch_lo, r - 1), half = (1 << (r - 1)) * NS;
            for (int t = ww; t < np; t += kWorkWaves) {
                const int xi = sched_at(sch_lo, kSchPairs + 14 * (r - 1) + t);
                const double *x = itm + xi * NS + sg * M;
                const double v = up_pair<M>(brow, x, x + half, nn);
                if (act) itm[xi * NS + lane] = v;
            }
            worker_sync(wcnt, wtarget, a);
        }
    }
    L2C_TS(3, 21);
    if (ww <= ts.G0) {
        const int g = ww;
        double c0 = 0.0, c1 = 0.0;
        const int b0 = sched_at(sch_lo, kSchBase + 2 * g), b1 = sched_at(sch_lo, kSchBase + 2 * g + 1);
        const bool ok0 = b0 >= 0, ok1 = b1 >= 0;
        const double *x0 = itm + (ok0 ? b0 : 0) * NS + sg * M;
        const double *x1 = itm + (ok1 ? b1 : 0) * NS + sg * M;
        double xv0[M], xv1[M];
#pragma unroll
        for (int l = 0; l < M; ++l) {
            xv0[l] = x0[l];
            xv1[l] = x1[l];
        }
        ops_first<2 * M>();
        double d0[2] = {0.0, 0.0}, d1[2] = {0.0, 0.0};
#pragma unroll
        for (int l = 0; l < M; ++l) {
            d0[l & 1] = fma(ag0[l], xv0[l], d0[l & 1]);
            d1[l & 1] = fma(ag1[l], xv1[l], d1[l & 1]);
        }
        if (ok0) c0 = d0[0] + d0[1];
        if (ok1) c1 = d1[0] + d1[1];
        if (act) canc[g * M2 + lane] = c0 + c1;
    }
    worker_sync(wcnt, wtarget, a);
    L2C_TS(3, 22);
    if (top) {
        double bcol[M];
#pragma unroll
        for (int k = 0; k < M; ++k) bcol[k] = Bl[k * M + nn];
        double cc = act ? canc[lane] : 0.0;
        for (int g = 1; g <= ts.G0; ++g) {
            const int p = (int)(ts.anc(g) & 1);
            if (act) zb[lane] = cc;
            wave_lds_sync();
            double zv[M];
#pragma unroll
            for (int k = 0; k < M; ++k) zv[k] = zb[sg * M + k];
            ops_first<M>();
            double q0 = 0.0, q1 = 0.0, q2 = 0.0;       // three chains (latency)
#pragma unroll
            for (int k = 0; k < M; ++k) {
                const double v = zv[k];
                const double t = (p && (k & 1)) ? -v : v;
                if (k % 3 == 0) q0 = fma(bcol[k], t, q0);
                else if (k % 3 == 1) q1 = fma(bcol[k], t, q1);
                else q2 = fma(bcol[k], t, q2);
            }
            const double acc2 = (q0 + q1) + q2;
            wave_lds_sync();
            cc = (act ? canc[g * M2 + lane] : 0.0) + ((p && (nn & 1)) ? -acc2 : acc2);
        }
        if (act) cR[lane] = cc;
    }
}

// Rows nn of ancestor a_g's two top-table submatrices (zero where the block does not exist).
template <int M>
__device__ __forceinline__ void load_anc_rows(const ExecArgs &a, const TopSlots &ts, int g, int lane, double (&ag0)[M],
                                              double (&ag1)[M])
{
    const bool act = lane < 2 * M;
    const int nn = act ? (lane >= M ? lane - M : lane) : 0;
    const bool ok0 = g <= ts.G0 && ts.ok(2 * g), ok1 = g <= ts.G0 && ts.ok(2 * g + 1);
    const int64_t an = ts.anc(g <= ts.G0 ? g : 0);
    const double *A = a.ahat_top + (level_block_offset(g <= ts.G0 ? g : 0) + (an >> 1)) * 3 * M * M + nn * M;
    const int r0 = 2 * (int)(an & 1);
#pragma unroll
    for (int l = 0; l < M; ++l) {
        ag0[l] = ok0 ? A[r0 * M * M + l] : 0.0;
        ag1[l] = ok1 ? A[M * M + l] : 0.0;
    }
}

// Step (6) for one item (node, parity sig, rows m0 .. m0+R-1): row m sums over m' in
// [m, 2s): P[m'-m] Q[2s u + sig + m + m'] g[2s u + 2m' + sig], with P, Q and g entering
// through circular register windows (slot t of a step holds m' = mb + t; m0 is a multiple
// of R).  Each step's operands are loaded before its products.  GPAD, QPAD: the pads of
// the node strides of g (between nodes) and Q (one, at 2s), known at compile time so that
// the index arithmetic vanishes where they are zero.
template <int R, int GPAD, int QPAD, bool TAIL>
__device__ __forceinline__ void near_step(double (&acc)[R], double (&pb)[R], double (&qb)[R], const double *gs,
                                          const double *qs, const double *ps, int s, int sig, int m0, int st)
{
    const int mb = m0 + st * R, cb = sig + m0 + mb + R - 1;
    double pn[R], qn[R], gn[R];
#pragma unroll
    for (int t = 0; t < R; ++t) {
        const int mp = mb + t, c = cb + t;
        pn[t] = ps[mp];
        qn[t] = qs[c + (QPAD && c >= 2 * s ? 1 : 0)];
        gn[t] = gs[mp + (GPAD ? (mp >= s ? 1 : 0) + (mp >= 2 * s ? 1 : 0) : 0)];
    }
    ops_first<3 * R>();
#pragma unroll
    for (int t = 0; t < R; ++t) {
        pb[t] = pn[t];
        qb[(t + R - 1) % R] = qn[t];
        const double gv = (TAIL && mb + t >= 2 * s) ? 0.0 : gn[t];
#pragma unroll
        for (int r = 0; r < R; ++r) acc[r] = fma(pb[(t - r + R) % R] * qb[(t + r) % R], gv, acc[r]);
    }
}

template <int R, int GPAD, int QPAD>
__device__ __forceinline__ void near_item(double (&acc)[R], const double *gs, const double *qs, const double *ps,
                                          int s, int sig, int m0)
{
    double pb[R], qb[R];
#pragma unroll
    for (int r = 0; r < R; ++r) pb[r] = 0.0;
#pragma unroll
    for (int r = 0; r < R - 1; ++r) {
        const int c = sig + 2 * m0 + r;
        qb[r] = qs[c + (QPAD && c >= 2 * s ? 1 : 0)];
    }
    // only the last step reaches past m' = 2s (the rows end there): the others take no
    // per-element bound
    const int steps = ((2 * s - m0) + R - 1) / R;
    for (int st = 0; st < steps - 1; ++st) near_step<R, GPAD, QPAD, false>(acc, pb, qb, gs, qs, ps, s, sig, m0, st);
    near_step<R, GPAD, QPAD, true>(acc, pb, qb, gs, qs, ps, s, sig, m0, steps - 1);
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
    // the top wave shares a SIMD with the streamer (waves w and w + 4 pair up), so the
    // near-field waves, which keep the FP64 pipes busy, do not slow its latency-bound chain
    const bool top = wv == kTopWave, near = !streamer && !top;
    // near-field wave index; item blocks of 6, 5, 4 window steps (x = nw >> 1) are paired on
    // the three SIMDs as (0, 4), (1, 5), (2, 3): 10 steps each
    const int nw = top ? kNearWaves : wv < kTopWave ? wv - NSW : (wv == 7 ? 3 : wv - NSW);
    const int ntid = nw * 64 + lane;

    double *Bl = lds;                                 // M*M
    double *Tl = Bl + M * M;                          // 2 s M (the top wave's items in between)
    double *gp = Tl + fused_t_area(L, M, s, kd);      // near-field area: 2 GX input, nQ Q, nP P
    double *Ql = gp + 2 * GX;
    double *Pl = Ql + nQ;
    double *wl = gp + fused_near_area(L, M, s, kd);   // fused_wofs(kd + 1) nodes
    double *cown = wl + fused_wofs(kd + 1) * NS;      // own depths 1..kd at node 2^d - 2
    double *cR = cown + own * NS;                     // c at the unit root (ancestor chain)
    double *w7 = cR + NS;                             // top wave: exchange scratch, then z and canc
    double *dummy = w7 + fused_w7(M, G0);             // 2 NS: stores of out-of-range slots
    unsigned *sync = reinterpret_cast<unsigned *>(dummy + 2 * NS);
    unsigned *wcnt = sync, *rdy = sync + 1, *nbr = sync + 2, *qdone = sync + 4;

    const int64_t n_it = a.item_n ? a.item_n[item] : a.n;
    const double *in = a.item_in ? a.item_in[item] : a.in + item * a.n;
    // exchange nodes: this launch's half, and the next launch's (reset to empty here)
    double *pubc = a.pub + ((int64_t)(a.epoch & 1u) * a.pub_items + item) * G.NX * M2;
    double *pubn = a.pub + (int64_t)((a.epoch + 1u) & 1u) * a.pub_items * G.NX * M2;
    const int64_t nbase = G.NF + (int64_t)X * 2 * (kd - 1);   // this unit's nodes 0, 1 of depths 1..kd-1
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
        L2C_TS(3, 17);
        int grp = wv;
#pragma unroll 1
        for (; grp + NSW < G.sub_groups; grp += NSW) {
            stream_group<M, true>(a, grp, grp + NSW, sub, wl, cown, dummy, kd, nslots, lane, rdy, nbr, t0, t1, t2);
            if (grp == wv) L2C_TS(3, 15);
        }
        if (grp < G.sub_groups) stream_group<M, false>(a, grp, 0, sub, wl, cown, dummy, kd, nslots, lane, rdy, nbr, t0, t1, t2);
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
            vg[u] = (e < cntg && x < s * (nodes + 2) && j < n_it) ? in[j] : 0.0;
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
        //      neighbours): per parity the product W (node x k) = F (node x m) T (m x k), on the
        //      FP64 matrix cores in 16 x 16 tiles, m in steps of 4 (zero padded); lane l
        //      supplies A[l % 16][l / 16] and B[l / 16][l % 16] and receives D[4q + l / 16][l % 16].
        {
            // modes 17..20 (M = 17..20) are a small remainder: the matrix cores take modes
            // 0..15 (one 16-mode tile instead of two mostly empty ones) and the vector units the
            // rest, on the waves that hold one tile fewer
            constexpr int KV = (M > 16 && M <= 20) ? M - 16 : 0;       // modes on the vector units
            constexpr int KTL = (M - KV + 15) / 16;                      // mode tiles
            const int nall = nodes + 2, ntl = (nall + 15) / 16, tiles = 2 * ntl * KTL;
            const int li = lane & 15, lk = lane >> 4;
            for (int t = ww; t < tiles; t += kWorkWaves) {
                const int kt = t % KTL, rest = t / KTL, ntile = rest % ntl, sig = rest / ntl;
                const int na = ntile * 16 + li, kb = kt * 16 + li;
                const bool arow = na < nall, bcol = kb < M - KV;
                const double *fa = gp + sig * GX + (arow ? na : 0) * GS;
                const double *tb = Tl + sig * s * M + (bcol ? kb : 0);
                double av[8], bv[8];                              // s <= 32: at most 8 steps
#pragma unroll
                for (int st = 0; st < 8; ++st) {
                    const int m = 4 * st + lk, mc = m < s ? m : s - 1;
                    av[st] = fa[mc];
                    bv[st] = tb[mc * M];
                }
                ops_first<16>();
                d4_t d = {0.0, 0.0, 0.0, 0.0};
#pragma unroll
                for (int st = 0; st < 8; ++st) {
                    if (4 * st < s) {
                        const bool min = 4 * st + lk < s;
                        d = __builtin_amdgcn_mfma_f64_16x16x4f64((min && arow) ? av[st] : 0.0,
                                                                 (min && bcol) ? bv[st] : 0.0, d, 0, 0, 0);
                    }
                }
#pragma unroll
                for (int q = 0; q < 4; ++q) {
                    const int node = ntile * 16 + 4 * q + lk;     // nodes >= 2^kd: neighbour slots
                    if (node < nall && bcol) wl[(fused_wofs(kd) + node) * NS + sig * M + kb] = d[q];
                }
            }
            if (KV > 0) {
                // output (node, sig, mode 16 + kv), node fastest (the T values are broadcast);
                // the index rotates so that the waves after the last one with an extra tile
                // start first
                const int w0 = tiles % kWorkWaves;
                const int cnt = nall * 2 * KV;
                for (int e = (wt + NWT - 64 * w0) % NWT; e < cnt; e += NWT) {
                    const int node = e % nall, rest = e / nall, kv = rest % KV, sig = rest / KV;
                    const double *fa = gp + sig * GX + node * GS;
                    const double *tb = Tl + sig * s * M + 16 + kv;
                    double acc0 = 0.0, acc1 = 0.0;
                    for (int m0 = 0; m0 < s; m0 += 8) {
                        double fv[8], tv[8];
#pragma unroll
                        for (int i = 0; i < 8; ++i) {
                            const int m = m0 + i, mc = m < s ? m : s - 1;
                            fv[i] = fa[mc];
                            tv[i] = tb[mc * M];
                        }
#pragma unroll
                        for (int i = 0; i < 8; i += 2) {
                            if (m0 + i < s) acc0 = fma(fv[i], tv[i], acc0);
                            if (m0 + i + 1 < s) acc1 = fma(fv[i + 1], tv[i + 1], acc1);
                        }
                    }
                    wl[(fused_wofs(kd) + node) * NS + sig * M + 16 + kv] = acc0 + acc1;
                }
            }
        }
        L2C_TS(3, 16);
        worker_sync(wcnt, wtarget, a);
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
                worker_sync(wcnt, wtarget, a);
                if (wt == 0) lds_flag_set(rdy, (unsigned)d);
            }
        }
        L2C_TS(3, 12);
        // publish the root (level G0, node X) and nodes 0, 1 of depths 1..kd-1 (level G0 + d,
        // nodes X 2^d, X 2^d + 1) as exchange nodes
        {
            const int cnt = (2 * kd - 1) * M2;
            for (int e = wt; e < cnt; e += NWT) {
                const int q = e / M2, r = e - q * M2;
                const int d = q == 0 ? 0 : (q + 1) >> 1, k = q == 0 ? 0 : (q - 1) & 1;
                const int64_t id = q == 0 ? node_offset(G0) + X : nbase + (q - 1);
                store_coherent(pubc + id * M2 + r, wl[(fused_wofs(d) + k) * NS + r]);
            }
        }
        L2C_TS(3, 3);
        // ---- near-field Q table (off the path to the published root), by the near waves
        if (near) {
            // Q in runs of 8 consecutive S: the first value from Eq. (tau), then the exact ratio
            // Q_{S+1}/Q_S: (2S+1)/(2S+2) for leg2cheb (Eq. (Lambdaint)), 2S/(2S+3) for cheb2leg
            {
                const int QL = 2 * s * nodes + 3 * s + 2 * R;
                for (int run = ntid; run * 8 < QL; run += 64 * kNearWaves) {
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
                WaitClock wc;
                for (int it = 1; lds_flag_get(qdone) < (unsigned)kNearWaves; ++it) {
                    __builtin_amdgcn_s_sleep(1);
                    if ((it & 15) == 0 && wc.expired(a.wait_ticks)) {
                        raise_status(a.status, kStatusWorkers);
                        break;
                    }
                }
            }
            lds_acquire();
            L2C_TS(3, 18);
        }
        // ---- step (6): near field.  Item (node nd, parity sig, rows m0 .. m0+R-1): row m sums
        //      over m' in [m, 2s): P[m'-m] Q[2s u + sig + m + m'] g[2s u + 2m' + sig], with P, Q
        //      and g entering through circular register windows; the sums stay in registers
        //      until the leaf evaluation.
        if (near && ntid < nwork) {
            const int nd = ntid % nodes, x = ntid / nodes;
            const int sig = x & 1, m0 = (x >> 1) * R;
            const double *gs = gp + sig * GX + nd * GS;
            const double *qs = Ql + nd * QS;
            const double *ps = Pl + (R - 1) - m0;
            switch (gpad * 2 + qpad) {                    // the pads are wave-uniform
            case 0: near_item<R, 0, 0>(acc, gs, qs, ps, s, sig, m0); break;
            case 1: near_item<R, 0, 1>(acc, gs, qs, ps, s, sig, m0); break;
            case 2: near_item<R, 1, 0>(acc, gs, qs, ps, s, sig, m0); break;
            default: near_item<R, 1, 1>(acc, gs, qs, ps, s, sig, m0); break;
            }
        }
        L2C_TS(3, 4);
        // this unit's exchange nodes in the next launch's half of the buffer: empty again, for
        // items item, item + batch, ... (the next launch may hold more items than this one); by
        // the near waves, off the path to the published root
        if (near) {
            const int kx = X == 0 ? G0 : min(G0, __ffs(X) - 1);
            const int nxq = 2 * (kd - 1), nq = 1 + nxq + (kx < 3 ? kx : 3);
            for (int64_t it = item; it < a.pub_items; it += a.batch) {
                for (int e = ntid; e < nq * M2; e += 64 * kNearWaves) {
                    const int q = e / M2, r = e - q * M2;
                    const int64_t id = q == 0     ? node_offset(G0) + X
                                       : q <= nxq ? nbase + (q - 1)
                                                  : node_offset(G0 - (q - nxq)) + (X >> (q - nxq));
                    store_coherent(pubn + (it * G.NX + id) * M2 + r, pub_empty());
                }
            }
        }
        // ---- steps (2)-(4) above the unit (TopSlots, top_gather, top_combine)
        const TopSlots ts(X, G0);
        // the unit's tree-top table, entry lane in every lane (read by lane shuffles)
        const int sch_lo = a.top_sched[(int64_t)X * kTopSchedInts + lane];
        double ag0[M], ag1[M];
        load_anc_rows<M>(a, ts, ww, lane, ag0, ag1);
        // T again, for step (5): the near waves load it now and write it once the column
        // nodes in the T area have been used
        constexpr int UTR = (kFusedStageT * kWorkThreads + 64 * kNearWaves - 1) / (64 * kNearWaves);
        double vtr[UTR];
#pragma unroll
        for (int u = 0; u < UTR; ++u) {
            const int e = u * 64 * kNearWaves + ntid;
            vtr[u] = (near && e < 2 * s * M) ? a.T[e] : 0.0;
        }
        if (top) {
            top_gather<M>(a, ts, kd, U, nbase, wl, w7, Tl, Bl, pubc, nbr, sch_lo, lane);
            L2C_TS(3, 9);
        }
        worker_sync(wcnt, wtarget, a);         // items and schedule in LDS; near field done
        L2C_TS(3, 20);
        // the near part of the unit's output rows (step (7)'s row scale rs for cheb2leg, and
        // its K_00 term) into the near-field area, now free: node stride 2s+1
        if (near && ntid < nwork) {
            const int x = ntid / nodes, nd = ntid % nodes, sig = x & 1, m0 = (x >> 1) * R;
#pragma unroll
            for (int r = 0; r < R; ++r) {
                const int m = m0 + r;
                if (m < s) {
                    double v = acc[r];
                    if (dir == 1) {
                        const int64_t i = jb + nd * 2 * s + 2 * m + sig;
                        v *= 2.0 * (double)i + 1.0;
                        if (i == 0) v += in[0];      // K_00 u_0 = u_0 / 2 = f_0
                    }
                    gp[nd * (2 * s + 1) + 2 * m + sig] = v;
                }
            }
        }
        top_combine<M>(a, ts, Tl, sch_lo, ag0, ag1, w7 + 2 * M2, w7, cR, Bl, wcnt, wtarget,
                       ww, top, lane);
        if (top) L2C_TS(3, 10);
        if (near) {
#pragma unroll
            for (int u = 0; u < UTR; ++u) {
                const int e = u * 64 * kNearWaves + ntid;
                if (e < 2 * s * M) Tl[e] = vtr[u];
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

    // ---- steps (5) and (7): z = rs * near + sum_k T_k(X_m^sig) c(u)[sig][k] (row nodes
    //      u < P - 2); leg2cheb divides by c_i pi/2.  The unit's rows are assembled in LDS
    //      (the near-field area, free by now; node stride 2s+1 against bank conflicts; with
    //      small s and many nodes the rows reach past the input part into the Q table, dead
    //      by then), then written out in contiguous wave-wide stores.
    double *out = a.item_out ? a.item_out[item] : a.out + item * a.n;
    double *ob = gp;
    const int OS = 2 * s + 1;
    // (the near part is already in ob, written after the near field)
    // far part, step (5): per parity, Z (rows x nodes) = T (rows x M) C (M x nodes) on the
    // FP64 matrix cores, 16 x 16 tiles, k in steps of 4 (zero padded); lane l supplies
    // A[l % 16][l / 16] and B[l / 16][l % 16] and receives D[4q + l / 16][l % 16], q < 4.
    {
        const int lmt = s > 16 ? 1 : 0, lnt = kd > 4 ? kd - 4 : 0;   // row and node tiles: 2^lmt, 2^lnt
        const int tiles = 2 << (lmt + lnt);
        const int li = lane & 15, lk = lane >> 4;
        for (int t = wv; t < tiles; t += NTH / 64) {
            const int tn = t & ((1 << lnt) - 1), tm = (t >> lnt) & lmt, sig = t >> (lnt + lmt);
            const int ma = tm * 16 + li;                  // A row of this lane
            const int nb = tn * 16 + li;                  // B column of this lane
            const bool arow = ma < s, bcol = nb < nodes && u0 + nb < P - 2;
            const double *ta = Tl + (sig * s + (arow ? ma : 0)) * M;
            const double *cb = cfine + (bcol ? nb : 0) * NS + sig * M;
            // operands and the near parts of the tile first (clamped addresses, no branches)
            constexpr int KS = (M + 3) / 4;
            double av[KS], bv[KS], ov[4];
#pragma unroll
            for (int ks = 0; ks < KS; ++ks) {
                const int k = 4 * ks + lk, kc = k < M ? k : M - 1;
                av[ks] = ta[kc];
                bv[ks] = cb[kc];
            }
#pragma unroll
            for (int q = 0; q < 4; ++q) {
                const int m = tm * 16 + 4 * q + lk, nd = tn * 16 + li;
                ov[q] = ob[(nd < nodes ? nd : 0) * OS + 2 * (m < s ? m : 0) + sig];
            }
            ops_first<2 * KS + 4>();
            d4_t d = {0.0, 0.0, 0.0, 0.0};
#pragma unroll
            for (int ks = 0; ks < KS; ++ks) {
                const bool kin = 4 * ks + lk < M;
                d = __builtin_amdgcn_mfma_f64_16x16x4f64((arow && kin) ? av[ks] : 0.0, (bcol && kin) ? bv[ks] : 0.0, d,
                                                         0, 0, 0);
            }
#pragma unroll
            for (int q = 0; q < 4; ++q) {
                const int m = tm * 16 + 4 * q + lk, nd = tn * 16 + li;
                if (m < s && nd < nodes) {
                    const bool i0 = X == 0 && nd == 0 && m == 0 && sig == 0;   // global row 0
                    double v = ov[q] + d[q];
                    if (dir == 0) v *= (i0 ? 1.0 / kPi : 2.0 / kPi);
                    ob[nd * OS + 2 * m + sig] = v;
                }
            }
        }
    }
    __syncthreads();
    {
        // wave wv copies nodes wv, wv + 8, ... (2s <= 64 rows each, one per lane)
        constexpr int CN = 8;                         // nodes per wave per round (kd <= 7: 128 nodes)
        for (int nb = wv; nb < nodes; nb += CN * (NTH / 64)) {
            double v[CN];
#pragma unroll
            for (int c = 0; c < CN; ++c) {
                const int nd = nb + c * (NTH / 64);
                v[c] = (nd < nodes && lane < 2 * s) ? ob[nd * OS + lane] : 0.0;
            }
#pragma unroll
            for (int c = 0; c < CN; ++c) {
                const int nd = nb + c * (NTH / 64);
                const int64_t i = jb + (int64_t)nd * 2 * s + lane;
                if (nd < nodes && lane < 2 * s && i < n_it) out[i] = v[c];
            }
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

hipError_t fused_top_table(const l2c_plan_s &p, int **dst)
{
    *dst = nullptr;
    const int G0 = p.geo.groot, U = 1 << (G0 + 2);
    std::vector<int> tab((size_t)U * kTopSchedInts);
    for (int X = 0; X < U; ++X) top_table_unit(X, G0, tab.data() + (size_t)X * kTopSchedInts);
    hipError_t e = dev_alloc(dst, tab.size() * sizeof(int));
    if (e != hipSuccess) return e;
    return hipMemcpy(*dst, tab.data(), tab.size() * sizeof(int), hipMemcpyHostToDevice);
}

// Items per launch such that every workgroup is resident at once (0: path unavailable).
hipError_t fused_max_items(const l2c_plan_s &p, int64_t *items)
{
    *items = 0;
    const Geometry &G = p.geo;
    if (p.L < 2 || G.kd < 1 || !fused_supported(p.M)) return hipSuccess;
    const int nodes = 1 << G.kd, R = kFusedRows;
    if (nodes * 2 * ((G.s + R - 1) / R) > 64 * kNearWaves) return hipSuccess;          // near-field items
    if (G.groot > 6 || G.kd > 7) return hipSuccess;                                      // register batches
    if (2 * G.s > 64) return hipSuccess;                                                 // output copy: a row per lane
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
// previous one waits for everything enqueued so far on the previous one (an event recorded
// there at the switch), so a run of launches on one stream records no event.
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
static hipError_t run_fused(l2c_plan_s &p, const double *in, double *out, int64_t batch, hipStream_t st,
                            const ItemArrays *ia)
{
    const Geometry &G = p.geo;
    ExecArgs a;
    a.n = p.n;
    a.item_n = nullptr;
    a.item_in = nullptr;
    a.item_out = nullptr;
    a.dir = p.direction;
    a.geo = G;
    a.T = p.d_T;
    a.B0 = p.d_B;
    a.Ptab = p.d_P;
    a.ahat_top = p.d_top;
    a.ahat_bot = p.d_bot;
    a.w = p.d_w;
    a.pub = p.d_pub;
    a.top_sched = p.d_topsch;
    a.pub_items = p.fused_items;
    a.status = p.d_status;
    const uint64_t khz = (uint64_t)(p.clock_khz > 0 ? p.clock_khz : 100000);
    a.wait_ticks = (uint64_t)kWaitUs * khz / 1000u;
    a.poll_ticks = (uint64_t)p.poll_us * khz / 1000u;
    const size_t lds = fused_lds_bytes(G);
    const unsigned U = 1u << (G.groot + 2);
    FusedOrder &o = g_order[p.device & 63];
    std::lock_guard<std::mutex> lock(o.mu);
    if (!o.done) {
        hipError_t e = hipEventCreateWithFlags(&o.done, hipEventDisableTiming);
        if (e != hipSuccess) return e;
    }
    if (o.any && o.last != st) {
        hipError_t e = hipEventRecord(o.done, o.last);
        if (e == hipSuccess) e = hipStreamWaitEvent(st, o.done, 0);
        if (e != hipSuccess) return e;
    }
    for (int64_t b0 = 0; b0 < batch; b0 += p.fused_items) {
        ExecArgs c = a;
        c.batch = batch - b0 < p.fused_items ? batch - b0 : p.fused_items;
        c.in = in ? in + b0 * p.n : nullptr;     // null: a ragged batch (item arrays)
        c.out = out ? out + b0 * p.n : nullptr;
        if (ia) {
            c.item_n = ia->n + b0;
            c.item_in = ia->in + b0;
            c.item_out = ia->out + b0;
        }
        c.epoch = ++p.epoch;
        const bool timed = p.ev_before && p.ev_after && b0 == 0;
        if (timed) (void)hipEventRecord(p.ev_before, st);
        hipLaunchKernelGGL(k_fused<M>, dim3(U, (unsigned)c.batch), dim3(kFusedThreads), lds, st, c);
        if (timed) (void)hipEventRecord(p.ev_after, st);
    }
    const hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    o.last = st;
    o.any = true;
    return hipSuccess;
}

hipError_t launch_fused(l2c_plan_s &p, const double *in, double *out, int64_t batch, hipStream_t st,
                        const ItemArrays *ia)
{
    switch (p.M) {
#define L2C_CASE(MM) \
    case MM: return run_fused<MM>(p, in, out, batch, st, ia);
        L2C_FOR_EACH_RANK(L2C_CASE)
#undef L2C_CASE
    default: return hipErrorInvalidValue;
    }
}

}  // namespace l2c

#ifdef L2C_PHASE_TIMING
// Instrumented builds only: copy (and optionally clear) this file's phase table (kernel 3
// is k_fused; phases in the order of L2C_TS above).
extern "C" int l2c_debug_phase_ts(unsigned long long *dst, int64_t count, int clear)
{
    const size_t bytes = sizeof(unsigned long long) * (size_t)kPhaseKernels * kPhaseUnits * kPhaseSlots;
    if (count * (int64_t)sizeof(unsigned long long) != (int64_t)bytes) return -1;
    if (dst && hipMemcpyFromSymbol(dst, HIP_SYMBOL(l2c_phase_ts), bytes, 0, hipMemcpyDeviceToHost) != hipSuccess)
        return -3;
    if (clear) {
        static unsigned long long zero[kPhaseKernels * kPhaseUnits * kPhaseSlots];
        if (hipMemcpyToSymbol(HIP_SYMBOL(l2c_phase_ts), zero, bytes, 0, hipMemcpyHostToDevice) != hipSuccess)
            return -3;
    }
    return 0;
}
#endif
