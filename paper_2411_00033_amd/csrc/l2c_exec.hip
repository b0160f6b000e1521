// l2c_exec.hip -- execution kernels of the modal multipole Legendre <-> Chebyshev
// transform (arXiv 2411.00033, Alg. 4) for gfx950, FP64.
//
// One execute is three launches (plus one more k_top pass per 6 extra levels) on the
// caller's stream:
//   k_up    steps (0)-(2): stage the input (zero padding, c .* f for cheb2leg), contract
//           every finest node with T(sigma) (Eq. (wMM)) and run the upward pass
//           (Eq. (wtk), with the even/odd-diagonal split of App. A2) inside a subtree
//           of 2^ku finest nodes; writes w for every level of the subtree.
//   k_top   step (2) above the k_up subtree roots, 6 levels per pass, in LDS.
//   k_main  steps (3)-(7) for a subtree of 2^kd finest nodes: the far-field products
//           of its own blocks (streamed once from the subtree-major table: the
//           dominant HBM traffic) and of its ancestors (top table, shared in L2), the
//           downward spreading of step (4) from level 0, the leaf evaluation of
//           Eq. (step5), the near-diagonal direct part of step (6), the scaling of
//           step (7), and the output.  Nothing but w crosses kernel boundaries.
// Plans with L = 0, and short transforms, use k_direct (Alg. 1 for every row).
#include <mutex>

#include "l2c_device.h"

namespace l2c {

// ------------------------------------------------------------------------------------
// k_up: one workgroup per (subtree of 2^ku finest nodes, item).
// LDS: f chunk [nodes][D] (odd D = 2s + 1: lanes reading consecutive nodes hit distinct
//      banks), T, B(0), every w level of the subtree.
template <int M>
__global__ __launch_bounds__(kThreads) void k_up(ExecArgs a)
{
    extern __shared__ double lds[];
    L2C_TS(0, 0);
    const Geometry &G = a.geo;
    const int s = G.s, L = G.L, ku = G.ku;
    const int nodes = 1 << ku;
    const int64_t item = blockIdx.y;
    const int64_t t0 = (int64_t)blockIdx.x << ku;    // first finest node of the subtree
    const int D = 2 * s + 1;                          // odd row stride: distinct banks
    double *fl = lds;                                 // nodes * D
    double *Tl = fl + nodes * D;                      // 2 * s * M
    double *Bl = Tl + 2 * s * M;                      // M * M
    double *lv = Bl + M * M;                          // (2 nodes - 1) nodes: every subtree level
    const int tid = threadIdx.x;
    const int lane = tid & 63, wv = wave_id();

    // stage the input: zero past n; cheb2leg uses u = c .* f (u_0 = 2 f_0), Sec. 4.1
    const int64_t n_it = a.item_n ? a.item_n[item] : a.n;
    const double *in = a.item_in ? a.item_in[item] : a.in + item * a.n;
    const int64_t base = t0 * 2 * s;
    {
        constexpr int U = 8;
        const int cnt = nodes * 2 * s;
        for (int b0 = 0; b0 < cnt; b0 += U * kThreads) {
            double v[U];
#pragma unroll
            for (int u = 0; u < U; ++u) {
                const int e = b0 + u * kThreads + tid;
                const int64_t gi = base + e;
                v[u] = (e < cnt && gi < n_it) ? in[gi] : 0.0;
            }
#pragma unroll
            for (int u = 0; u < U; ++u) {
                const int e = b0 + u * kThreads + tid;
                if (e < cnt) {
                    const int nd = e / (2 * s);
                    fl[nd * D + (e - nd * 2 * s)] = (a.dir == 1 && base + e == 0) ? 2.0 * v[u] : v[u];
                }
            }
        }
    }
    stage_lds<5>(Tl, a.T, 2 * s * M);
    stage_lds<2>(Bl, a.B0, M * M);
    __syncthreads();
    L2C_TS(0, 1);

    // step (1): w_k(t, sigma) = sum_m T_k(X_m^sigma) f[2s t + 2m + sigma]  (Eq. (wMM)).
    // Wave -> (sigma, half of k); lane -> node; the T values of a step are the same for
    // every lane of the wave (LDS broadcast).
    {
        constexpr int KH = M / 2;
        const int sig = wv & 1, kb = (wv >> 1) * KH;
        const double *Ts = Tl + (size_t)sig * s * M + kb;
        for (int nd = lane; nd < nodes; nd += 64) {
            double acc[KH];
#pragma unroll
            for (int k = 0; k < KH; ++k) acc[k] = 0.0;
            const double *fr = fl + nd * D + sig;
            for (int m = 0; m < s; ++m) {
                const double fv = fr[2 * m];
#pragma unroll
                for (int k = 0; k < KH; ++k) acc[k] = fma(Ts[m * M + k], fv, acc[k]);
            }
            double *wo = lv + nd * lds_ns<M>() + sig * M + kb;
#pragma unroll
            for (int k = 0; k < KH; ++k) wo[k] = acc[k];
        }
    }
    __syncthreads();
    L2C_TS(0, 2);

    // step (2) inside the subtree, then every level to the workspace
    subtree_up<M>(lv, nodes, ku, Bl);
    double *wg = a.w + item * G.NT * 2 * M;
    for (int d = 0; d <= ku; ++d)
        nodes_lds_to_global<M, 4, kThreads>(wg + (node_offset(L - 1 - d) + (t0 >> d)) * 2 * M,
                                            lv + (2 * nodes - 2 * (nodes >> d)) * lds_ns<M>(), nodes >> d);
    L2C_TS(0, 3);
}

// ------------------------------------------------------------------------------------
// k_top: step (2) for kt levels above level gin; one workgroup per 2^kt nodes of gin.
template <int M>
__global__ __launch_bounds__(kThreads) void k_top(ExecArgs a, int gin, int kt)
{
    extern __shared__ double lds[];
    L2C_TS(1, 0);
    const int nodes = 1 << kt;
    const int64_t item = blockIdx.y;
    const int64_t t0 = (int64_t)blockIdx.x << kt;
    double *Bl = lds;                          // M * M
    double *lv = Bl + M * M;                   // (2 nodes - 1) nodes
    double *wg = a.w + item * a.geo.NT * 2 * M;
    nodes_global_to_lds<M, 10, kThreads>(lv, wg + (node_offset(gin) + t0) * 2 * M, nodes);
    stage_lds<2>(Bl, a.B0, M * M);
    __syncthreads();
    L2C_TS(1, 1);
    subtree_up<M>(lv, nodes, kt, Bl);
    for (int d = 1; d <= kt; ++d)
        nodes_lds_to_global<M, 4, kThreads>(wg + (node_offset(gin - d) + (t0 >> d)) * 2 * M,
                                            lv + (2 * nodes - 2 * (nodes >> d)) * lds_ns<M>(), nodes >> d);
    L2C_TS(1, 2);
}

// ------------------------------------------------------------------------------------
// k_main: one workgroup per (subtree root R at level groot, item); one workgroup per CU.
// Order of work: the staging loads (own column-node w, input) are issued, then the
// wave's first Ahat group; the near-field tables are computed while both arrive.  The
// near field (input only) runs while the Ahat stream arrives; then the ancestors' far
// field (top table in L2), the own far field (Ahat stream, next group refilled while the
// current one is used), the downward pass, and the leaf evaluation, which writes the
// output rows directly.
//
// Near-field work item = (node nd, parity sig, R rows starting at m0); item wi maps to
// nd = wi mod nodes, so with 64 nodes a wave holds one (sig, m0) and 64 nodes.  To keep
// these 64 lanes on distinct LDS banks the per-parity input and the Q table are stored
// with one pad double after every s (g, when s is even) or 2s (Q) entries.
template <int M>
__global__ __launch_bounds__(kMainThreads) void k_main(ExecArgs a)
{
    constexpr int R = kNearRows;
    constexpr int NCH = 3 * M / 2;
    constexpr int M2 = 2 * M;                          // node stride in the workspace
    constexpr int NS = lds_ns<M>();                    // node stride in LDS
    extern __shared__ double lds[];
    L2C_TS(2, 0);
    const Geometry &G = a.geo;
    const int s = G.s, L = G.L, kd = G.kd, groot = G.groot, dir = a.dir;
    const int nodes = 1 << kd;                        // finest nodes of the subtree
    const int own = 2 * nodes - 2;                    // own row / column nodes, depths 1..kd
    const int64_t item = blockIdx.y;
    const int64_t Rn = blockIdx.x;                    // subtree root, level groot
    const int64_t u0 = Rn << kd;                      // first finest row node
    // a subtree whose rows all lie past its item's length (in a ragged batch, items shorter
    // than the group's padded length) writes nothing: the workgroup ends before any barrier
    if (u0 * 2 * s >= (a.item_n ? a.item_n[item] : a.n)) return;
    const int64_t P = int64_t(1) << (L + 1);
    const int gpad = near_gpad(s);                    // g: node stride s + gpad
    const int GS = s + gpad;
    const int GXL = s * (nodes + 1) + R;              // logical per-parity g length
    const int GX = (int)near_gx(s, kd);               // padded per-parity g length
    const int qpad = near_qpad(s);                    // Q: node stride 2s + qpad
    const int QS = 2 * s + qpad;
    const int nQ = (int)near_nq(s, kd);
    const int nP = 2 * s + 2 * R;                     // P_d for d = [-(R-1), nP - R + 1)
    const int tid = threadIdx.x;
    const int lane = tid & 63, wv = wave_id();

    double *Bl = lds;                                 // M*M
    double *canc = Bl + M * M;                        // (groot+1) nodes: ancestors, level 0..groot
    double *cown = canc + (groot + 1) * NS;           // own nodes: depth d at node offset 2^d - 2
    double *wl = cown + own * NS;                     // own column nodes
    double *gp = wl + own * NS;                       // 2 * GX, later T (2 s M)
    double *Tl = gp;
    double *Ql = gp + 2 * GX;                         // nQ
    double *Pl = Ql + nQ;                             // nP

    const int64_t n_it = a.item_n ? a.item_n[item] : a.n;
    const double *in = a.item_in ? a.item_in[item] : a.in + item * a.n;
    const double *wgl = a.w + item * G.NT * M2;
    const int64_t jb = u0 * 2 * s;                    // first row of the subtree

    // ---- staging loads: own column-node w and the near-field input (registers)
    constexpr int UW = kMainStageW, UG = kMainStageG;
    double vw[UW], vg[UG];
    const int cntw = own * M2, cntg = 2 * GXL;
#pragma unroll
    for (int u = 0; u < UW; ++u) {
        // own column-node w: depth d holds column nodes (R << d) + 2 + [0, 2^d) of level
        // groot + d; flat node q = (2^d - 2) + t.  Nodes past the end of a level are zero.
        const int e = u * kMainThreads + tid;
        vw[u] = 0.0;
        if (e < cntw) {
            const int q = e / M2, r = e - q * M2;
            const int d = 31 - __clz(q + 2);
            const int64_t t = (Rn << d) + 2 + (q - ((1 << d) - 2));
            const int g = groot + d;
            if (t < (int64_t(1) << (g + 2))) vw[u] = wgl[(node_offset(g) + t) * M2 + r];
        }
    }
#pragma unroll
    for (int u = 0; u < UG; ++u) {
        const int e = u * kMainThreads + tid;              // e = sig * GXL + x
        const int sig = e >= GXL, x = e - sig * GXL;
        const int64_t j = jb + 2 * (int64_t)x + sig;
        vg[u] = (e < cntg && x < s * (nodes + 1) && j < n_it) ? in[j] : 0.0;
    }
    // ---- the wave's first far-field group goes in flight behind them
    const int nslots = (nodes - 1) * M;
    const double2 *sub = reinterpret_cast<const double2 *>(a.ahat_bot) + Rn * G.sub_groups * NCH * 64 + lane;
    double2 ar[NCH];
    if (!a.cfar && wv < G.sub_groups) {
#pragma unroll
        for (int ch = 0; ch < NCH; ++ch) ar[ch] = sub[(wv * NCH + ch) * 64];
    }
    // ---- near-field tables (arithmetic only) while the loads are in flight
    // Q in runs of 8 consecutive S: the first value from Eq. (tau), then the exact ratio
    // Q_{S+1}/Q_S, (2S+1)/(2S+2) for leg2cheb (Eq. (Lambdaint)) and 2S/(2S+3) for cheb2leg.
    {
        const int QL = 2 * s * nodes + 3 * s + 2 * R;   // logical entries read
        for (int run = tid; run * 8 < QL; run += kMainThreads) {
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
    for (int e = tid; e < nP; e += kMainThreads) Pl[e] = a.Ptab[e + kPLead - (R - 1)];
    stage_lds<1, kMainThreads>(Bl, a.B0, M * M);
    for (int e = tid; e < 2 * GX; e += kMainThreads) gp[e] = 0.0;
    __syncthreads();
#pragma unroll
    for (int u = 0; u < UW; ++u) {
        const int e = u * kMainThreads + tid;
        if (e < cntw) wl[(e / M2) * NS + e % M2] = vw[u];
    }
#pragma unroll
    for (int u = 0; u < UG; ++u) {
        const int e = u * kMainThreads + tid;
        if (e < cntg) {
            const int sig = e >= GXL, x = e - sig * GXL;
            const int64_t j = jb + 2 * (int64_t)x + sig;
            gp[sig * GX + x + (x / s) * gpad] = dir == 1 ? vg[u] * (double)j : vg[u];   // g_j = j u_j
        }
    }
    __syncthreads();
    L2C_TS(2, 1);

    // ---- step (6): near field.  Row m of the node's s rows of one parity sums over
    //      m' in [m, 2s): P[m'-m] Q[2s u + sig + m + m'] g[2s u + 2m' + sig].  P, Q and g
    //      enter through circular register windows (3 LDS reads per step for R rows);
    //      the sums stay in registers until the leaf evaluation.
    const int nch = (s + R - 1) / R;
    const int nwork = nodes * 2 * nch;               // <= kNearItems * kMainThreads (geometry)
    double acc[kNearItems][R];
#pragma unroll
    for (int it = 0; it < kNearItems; ++it) {
#pragma unroll
        for (int r = 0; r < R; ++r) acc[it][r] = 0.0;
        const int wi = lane + 64 * (wv + (kMainThreads / 64) * it);
        if (wi >= nwork) continue;
        const int nd = wi % nodes, x = wi / nodes;
        const int sig = x & 1, m0 = (x >> 1) * R;
        const double *gs = gp + sig * GX + nd * GS;      // g at m': gs[m' + (m' / s) gpad]
        const double *qs = Ql + nd * QS;                 // Q at c = sig + m0 + r + m': qs[c + (c >= 2s) qpad]
        const double *ps = Pl + (R - 1) - m0;            // P for row m0 + r at m': ps[m' - r]
        double pb[R], qb[R];
#pragma unroll
        for (int r = 0; r < R; ++r) pb[r] = 0.0;         // P at negative offsets
#pragma unroll
        for (int r = 0; r < R - 1; ++r) {
            const int c = sig + 2 * m0 + r;              // m' = m0
            qb[(m0 + r) % R] = qs[c + (c >= 2 * s ? qpad : 0)];
        }
        const int steps = ((2 * s - m0) + R - 1) / R;
        for (int st = 0; st < steps; ++st) {
            const int mb = m0 + st * R;
            const bool tail = mb + R > 2 * s;
#pragma unroll
            for (int t = 0; t < R; ++t) {
                const int mp = mb + t;                    // m' ; mp % R == t
                pb[t] = ps[mp];
                const int c = sig + m0 + mp + R - 1;
                qb[(t + R - 1) % R] = qs[c + (c >= 2 * s ? qpad : 0)];
                double gv = gs[mp + (mp >= s ? gpad : 0) + (mp >= 2 * s ? gpad : 0)];
                if (tail && mp >= 2 * s) gv = 0.0;
#pragma unroll
                for (int r = 0; r < R; ++r)
                    acc[it][r] = fma(pb[(t - r + R) % R] * qb[(t + r) % R], gv, acc[it][r]);
            }
        }
    }
    L2C_TS(2, 2);

    // ---- step (3), ancestors a_g = R >> (groot - g), g = 0..groot, from the top table
    for (int e = tid; e < (groot + 1) * M; e += kMainThreads) {
        const int g = e / M, k = e - g * M;
        const int64_t an = Rn >> (groot - g);
        double c0 = 0.0, c1 = 0.0;
        if (an < (int64_t(1) << (g + 2)) - 2) {
            const int64_t b = an >> 1;
            const double *Ab = a.ahat_top + (level_block_offset(g) + b) * 3 * M * M;
            const double *wc = wgl + (node_offset(g) + an + 2) * M2;   // w(a+2), w(a+3)
            if ((an & 1) == 0) {
                const double *A0r = Ab + k * M, *A1r = Ab + M * M + k * M;
#pragma unroll 3
                for (int l = 0; l < M; ++l) {
                    c0 = fma(A0r[l], wc[l], c0);
                    c1 = fma(A0r[l], wc[M + l], c1);
                    c0 = fma(A1r[l], wc[M2 + l], c0);
                    c1 = fma(A1r[l], wc[M2 + M + l], c1);
                }
            } else {
                const double *A2r = Ab + 2 * M * M + k * M;
#pragma unroll 3
                for (int l = 0; l < M; ++l) {
                    c0 = fma(A2r[l], wc[l], c0);
                    c1 = fma(A2r[l], wc[M + l], c1);
                }
            }
        }
        canc[g * NS + k] = c0;
        canc[g * NS + M + k] = c1;
    }
    L2C_TS(2, 3);

    // ---- step (3), own blocks: wave <-> groups of 64 slots; lane (j, k) produces
    //      c(2i)[k] = Ahat(.,0)[k,:] w(2i+2) + Ahat(.,1)[k,:] w(2i+3),  c(2i+1)[k] = Ahat(.,2)[k,:] w(2i+3)
    //      for both parities (i = block index within its depth).  The wave's first group
    //      was put in flight at the start; later groups are loaded when reached.
    if (a.cfar) {
        // the far-field part of the own blocks, computed by k_regen (the blocks regenerated
        // from the kernel samples instead of read from a stored table)
        const double *cf = a.cfar + (item * (P >> kd) + Rn) * own * M2;
        for (int e = tid; e < own * M2; e += kMainThreads) cown[(e / M2) * NS + e % M2] = cf[e];
    }
    for (int grp = wv; !a.cfar && grp < G.sub_groups; grp += kMainThreads / 64) {
        if (grp != wv) {
#pragma unroll
            for (int c2 = 0; c2 < NCH; ++c2) ar[c2] = sub[(grp * NCH + c2) * 64];
        }
        const int slot = grp * 64 + lane;
        const bool valid = slot < nslots;
        const int j = valid ? slot / M : 0, k = valid ? slot - j * M : 0;
        int d, i;                                        // depth and block index within it
        slot_depth(j, kd, d, i);
        const double *wt = wl + ((1 << d) - 2 + 2 * i) * NS;   // w(2i+2), then w(2i+3)
        double c00 = 0, c01 = 0, c10 = 0, c11 = 0;
#pragma unroll
        for (int c2 = 0; c2 < NCH; ++c2) {
            const double a0 = ar[c2].x, a1 = ar[c2].y;
#pragma unroll
            for (int h = 0; h < 2; ++h) {
                const int el = 2 * c2 + h, r = el / M, l = el - r * M;
                const double av = h ? a1 : a0;
                if (r == 0) {
                    c00 = fma(av, wt[l], c00);
                    c01 = fma(av, wt[M + l], c01);
                } else if (r == 1) {
                    c00 = fma(av, wt[NS + l], c00);
                    c01 = fma(av, wt[NS + M + l], c01);
                } else {
                    c10 = fma(av, wt[NS + l], c10);
                    c11 = fma(av, wt[NS + M + l], c11);
                }
            }
        }
        if (valid) {
            double *co = cown + ((1 << d) - 2 + 2 * i) * NS + k;
            co[0] = c00;
            co[M] = c01;
            co[NS] = c10;
            co[NS + M] = c11;
        }
    }
    __syncthreads();
    L2C_TS(2, 4);

    // ---- step (4): the chain of ancestors, c(a_g) += B(p)^T c(a_{g-1}), p = a_g & 1,
    //      then the subtree depths d = 1..kd from depth d-1 (depth 0 = R); T moves into
    //      the (now dead) near-field input area meanwhile
    stage_lds<3, kMainThreads>(Tl, a.T, 2 * s * M);
    {
        constexpr int QSTEP = kMainThreads / M;
        const int n = tid % M, q0 = tid / M;
        const bool qn_ok = tid < M * QSTEP;
        double bcol[M];
#pragma unroll
        for (int k = 0; k < M; ++k) bcol[k] = Bl[k * M + (qn_ok ? n : 0)];
        for (int g = 1; g <= groot; ++g) {
            if (qn_ok)
                down_level_qn<M>(canc + (g - 1) * NS, canc + g * NS, 1, (int)((Rn >> (groot - g)) & 1), bcol, n, q0,
                                 QSTEP);
            __syncthreads();
        }
        for (int d = 1; d <= kd; ++d) {
            const int cn = 1 << d;
            const double *parb = d == 1 ? canc + groot * NS : cown + ((cn >> 1) - 2) * NS;
            if (2 * cn <= QSTEP) {
                if (qn_ok) down_level_qn<M>(parb, cown + (cn - 2) * NS, cn, -1, bcol, n, q0, QSTEP);
            } else {
                down_level<M>(parb, cown + (cn - 2) * NS, cn, -1, Bl);
            }
            __syncthreads();
        }
    }
    if (groot == 0 && kd == 0) __syncthreads();
    const double *cfine = kd > 0 ? cown + (nodes - 2) * NS : canc + groot * NS;
    L2C_TS(2, 5);

    // ---- steps (5) and (7) for the thread's rows: z = sum_k T_k(X_m^sig) c(u)[sig][k]
    //      (row nodes u < P - 2) + rs * near; leg2cheb divides by c_i pi/2
    double *out = a.item_out ? a.item_out[item] : a.out + item * a.n;
#pragma unroll
    for (int it = 0; it < kNearItems; ++it) {
        const int wi = lane + 64 * (wv + (kMainThreads / 64) * it);
        if (wi >= nwork) continue;
        const int nd = wi % nodes, x = wi / nodes;
        const int sig = x & 1, m0 = (x >> 1) * R;
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
                double v = acc[it][r];
                if (dir == 1) {
                    v *= 2.0 * (double)i + 1.0;
                    if (i == 0) v += in[0];      // K_00 u_0 = u_0 / 2 = f_0
                }
                v += z;
                if (dir == 0) v *= (i == 0 ? 1.0 / kPi : 2.0 / kPi);
                if (i < n_it) out[i] = v;
            }
        }
    }
    L2C_TS(2, 6);
}

// ------------------------------------------------------------------------------------
// k_direct: Alg. 1, each output row as one sum over its band j >= i, j - i even, with the
// factorisation a_ij = rs_i P_{(j-i)/2} Q_{(i+j)/2} g_j of the near field applied to the
// whole row.  Used by plans with L = 0 and, up to kDirectMaxN, by short transforms,
// where a multipole launch is pure latency.
// Workgroup (row block rb, parity sg) of one item: rows i = 2 i' + sg, i' in
// [16 rb, 16 rb + 16); 16 lanes per row take j' = i' + lane, i' + lane + 16, ...
// (j = 2 j' + sg) and a butterfly over the 16 lanes adds their partial sums.  The
// block's g, P and Q are staged in LDS first: with c = j' - 16 rb, g[c] = g_{2j'+sg},
// P[c] = P_c, Q[c] = Q_{32 rb + sg + c}, and row r of the block reads P[c - r] Q[c + r] g[c].
// P and Q come from the plan's tables (k_direct_tables), built once with the same device
// functions that the near field uses.
constexpr int kDirRows = 16;

int64_t direct_table_len(int64_t n) { return (n + 1) / 2 + n + 17; }

__global__ void k_direct_tables(double *tab, int64_t n, int dir)
{
    const int64_t HP = (n + 1) / 2;
    const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (e < HP) tab[e] = near_P(dir, e);
    else if (e < HP + n + 17) tab[e] = near_Q(dir, e - HP);
}

hipError_t direct_build(const l2c_plan_s &p, double *tab, hipStream_t st)
{
    const int64_t len = direct_table_len(p.n);
    hipLaunchKernelGGL(k_direct_tables, dim3((unsigned)((len + 255) / 256)), dim3(256), 0, st, tab, p.n, p.direction);
    return hipGetLastError();
}

__global__ __launch_bounds__(kThreads) void k_direct(const double *in, double *out, int64_t nmax, int dir,
                                                     const int64_t *item_n, const double *const *item_in,
                                                     double *const *item_out, const double *tab)
{
    extern __shared__ double lds[];
    const int64_t HPm = (nmax + 1) / 2;
    double *gl = lds, *Pl = gl + HPm, *Ql = Pl + HPm;   // HPm, HPm and HPm + kDirRows doubles
    const int sg = blockIdx.x & 1;
    const int64_t i0 = (int64_t)(blockIdx.x >> 1) * kDirRows;
    const int64_t item = blockIdx.y;
    const int64_t n = item_n ? item_n[item] : nmax;     // ragged batch: this item's length (<= nmax)
    const int64_t H = (n - sg + 1) / 2;                 // rows (and columns) of parity sg
    if (i0 >= H) return;
    const double *x = item_in ? item_in[item] : in + item * nmax;
    double *y = item_out ? item_out[item] : out + item * nmax;
    const int64_t C = H - i0;                           // columns j' in [i0, H)
    const double *Pt = tab, *Qt = tab + HPm + 2 * i0 + sg;   // Q_S for S < nmax + 17
    for (int64_t c = threadIdx.x; c < C + kDirRows; c += kThreads) {
        if (c < C) {
            const int64_t j = 2 * (i0 + c) + sg;
            double v = x[j];
            if (dir == 1) v *= (double)j;
            gl[c] = v;
            Pl[c] = Pt[c];
        }
        Ql[c] = Qt[c];
    }
    __syncthreads();
    const int r = threadIdx.x >> 4, k = threadIdx.x & 15;
    const int64_t ip = i0 + r;
    double acc = 0.0;
    if (ip < H)
        for (int64_t c = r + k; c < C; c += 16) acc = fma(Pl[c - r] * Ql[c + r], gl[c], acc);
#pragma unroll
    for (int m = 8; m >= 1; m >>= 1) acc += __shfl_xor(acc, m, 16);
    if (k == 0 && ip < H) {
        const int64_t i = 2 * ip + sg;
        if (dir == 1) {
            acc *= 2.0 * (double)i + 1.0;
            if (i == 0) acc += x[0];   // K_00 u_0 = f_0
        } else {
            acc /= (i == 0 ? kPi : 0.5 * kPi);
        }
        y[i] = acc;
    }
}

static hipError_t direct_attrs();

hipError_t launch_direct(const l2c_plan_s &p, const double *in, double *out, int64_t batch, hipStream_t st,
                         const ItemArrays *ia)
{
    if (!p.d_dir) return hipErrorInvalidValue;
    const int64_t HPm = (p.n + 1) / 2;
    const size_t lds = sizeof(double) * (size_t)(3 * HPm + kDirRows);
    if (lds > 64 * 1024) {
        const hipError_t attr_err = direct_attrs();
        if (attr_err != hipSuccess) return attr_err;
    }
    const unsigned blocks = (unsigned)(2 * ((HPm + kDirRows - 1) / kDirRows));
    for (int64_t b0 = 0; b0 < batch; b0 += kMaxItemsPerLaunch) {
        const int64_t nb = batch - b0 < kMaxItemsPerLaunch ? batch - b0 : kMaxItemsPerLaunch;
        const bool timed = p.ev_before && p.ev_after && b0 == 0;
        if (timed) (void)hipEventRecord(p.ev_before, st);
        hipLaunchKernelGGL(k_direct, dim3(blocks, (unsigned)nb), dim3(kThreads), lds, st,
                           ia ? nullptr : in + b0 * p.n, ia ? nullptr : out + b0 * p.n, p.n, p.direction,
                           ia ? ia->n + b0 : nullptr, ia ? ia->in + b0 : nullptr, ia ? ia->out + b0 : nullptr,
                           (const double *)p.d_dir);
        if (timed) (void)hipEventRecord(p.ev_after, st);
        const hipError_t e = hipGetLastError();
        if (e != hipSuccess) return e;
    }
    return hipSuccess;
}

// ------------------------------------------------------------------------------------
static size_t up_lds_bytes(const Geometry &G)
{
    const int nodes = 1 << G.ku;
    const int D = 2 * G.s + 1;
    return sizeof(double) * ((size_t)nodes * D + 2 * (size_t)G.s * G.M + (size_t)G.M * G.M +
                             (size_t)(2 * nodes - 1) * (2 * G.M + 1));
}

static size_t top_lds_bytes(const Geometry &G, int kt)
{
    const int nodes = 1 << kt;
    return sizeof(double) * ((size_t)G.M * G.M + (size_t)(2 * nodes - 1) * (2 * G.M + 1));
}

static size_t main_lds_bytes(const Geometry &G)
{
    return sizeof(double) * (size_t)main_lds_doubles(G.L, G.M, G.s, G.kd);
}

// Allow the full 160 KiB LDS of a gfx950 CU for k_up<M> and k_main<M> (once per process and
// rank; the result is kept).  Plans call it when they are made, so that an execute captured
// into a graph makes no such call.
template <int M>
static hipError_t main_attrs()
{
    static std::once_flag attr_once;
    static hipError_t attr_err = hipSuccess;
    std::call_once(attr_once, [] {
        attr_err = hipFuncSetAttribute((const void *)k_up<M>, hipFuncAttributeMaxDynamicSharedMemorySize, 160 * 1024);
        if (attr_err == hipSuccess)
            attr_err =
                hipFuncSetAttribute((const void *)k_main<M>, hipFuncAttributeMaxDynamicSharedMemorySize, 160 * 1024);
    });
    return attr_err;
}

static hipError_t direct_attrs()
{
    static std::once_flag attr_once;
    static hipError_t attr_err = hipSuccess;
    std::call_once(attr_once, [] {
        attr_err = hipFuncSetAttribute((const void *)k_direct, hipFuncAttributeMaxDynamicSharedMemorySize, 160 * 1024);
    });
    return attr_err;
}

hipError_t prepare_launches(const l2c_plan_s &p)
{
    hipError_t e = direct_attrs();
    if (e != hipSuccess || p.L == 0) return e;
    switch (p.M) {
#define L2C_CASE(MM) \
    case MM: return main_attrs<MM>();
        L2C_FOR_EACH_RANK(L2C_CASE)
#undef L2C_CASE
    default: return hipErrorInvalidValue;
    }
}

template <int M>
static hipError_t run(const l2c_plan_s &p, const double *in, double *out, int64_t batch, hipStream_t st,
                      const ItemArrays *ia, double *w)
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
    const int64_t P = int64_t(1) << (G.L + 1);
    const size_t up_lds = up_lds_bytes(G), main_lds = main_lds_bytes(G);
    const hipError_t attr_err = main_attrs<M>();
    if (attr_err != hipSuccess) return attr_err;
    for (int64_t b0 = 0; b0 < batch; b0 += kMaxItemsPerLaunch) {
        ExecArgs c = a;
        c.batch = batch - b0 < kMaxItemsPerLaunch ? batch - b0 : kMaxItemsPerLaunch;
        c.in = in ? in + b0 * p.n : nullptr;     // null: a ragged batch (item arrays)
        c.out = out ? out + b0 * p.n : nullptr;
        if (ia) {
            c.item_n = ia->n + b0;
            c.item_in = ia->in + b0;
            c.item_out = ia->out + b0;
        }
        c.w = w + b0 * G.NT * 2 * M;
        const unsigned items = (unsigned)c.batch;
        hipLaunchKernelGGL(k_up<M>, dim3((unsigned)(P >> G.ku), items), dim3(kThreads), up_lds, st, c);
        for (int gin = G.L - 1 - G.ku; gin > 0;) {
            const int kt = gin < G.kt ? gin : G.kt;
            const unsigned wgs = (unsigned)((int64_t(1) << (gin + 2)) >> kt);
            hipLaunchKernelGGL(k_top<M>, dim3(wgs, items), dim3(kThreads), top_lds_bytes(G, kt), st, c, gin, kt);
            gin -= kt;
        }
        if (p.regen) {
            // the own blocks' far-field products, their submatrices recomputed from the samples
            double *cf = p.d_cf + b0 * regen_cf_per_item(G);
            const hipError_t e = launch_regen(p, c, cf, st);
            if (e != hipSuccess) return e;
            c.cfar = cf;
        }
        const bool timed = p.ev_before && p.ev_after && b0 == 0;
        if (timed) (void)hipEventRecord(p.ev_before, st);
        hipLaunchKernelGGL(k_main<M>, dim3((unsigned)(P >> G.kd), items), dim3(kMainThreads), main_lds, st, c);
        if (timed) (void)hipEventRecord(p.ev_after, st);
    }
    return hipGetLastError();
}

hipError_t launch_execute(const l2c_plan_s &p, const double *in, double *out, int64_t batch, hipStream_t st,
                          const ItemArrays *ia)
{
    if (p.L == 0) return launch_direct(p, in, out, batch, st, ia);
    switch (p.M) {
#define L2C_CASE(MM) \
    case MM: return run<MM>(p, in, out, batch, st, ia, p.d_w);
        L2C_FOR_EACH_RANK(L2C_CASE)
#undef L2C_CASE
    default: return hipErrorInvalidValue;
    }
}

// ------------------------------------------------------------------------------------
// Workspace of leg2cheb_execute_noalloc: the upward vectors w of the three-launch path in
// a fixed device array instead of the plan's workspace, for callers that cannot allocate.
// Each device holds its own copy for the life of the process.  Nothing in it needs to
// start at zero (k_up and k_top write every node that k_main reads), and calls that
// overlap on one device race for it.
static __device__ __align__(256) double scratch[kNoallocScratchBytes / sizeof(double)];

namespace {
std::mutex g_scratch_mu;
double *g_scratch_ptr[64] = {};   // device address of scratch, per device
}  // namespace

// The device address of scratch on `device` (the current device), resolved once per device.
hipError_t noalloc_scratch(int device, double **ptr)
{
    *ptr = nullptr;
    if (device < 0 || device >= 64) return hipErrorInvalidDevice;
    std::lock_guard<std::mutex> lock(g_scratch_mu);
    if (!g_scratch_ptr[device]) {
        double *q = nullptr;
        const hipError_t e = hipGetSymbolAddress((void **)&q, HIP_SYMBOL(scratch));
        if (e != hipSuccess) return e;
        if (!q) return hipErrorInvalidSymbol;
        g_scratch_ptr[device] = q;
    }
    *ptr = g_scratch_ptr[device];
    return hipSuccess;
}

hipError_t launch_execute_scratch(const l2c_plan_s &p, const double *in, double *out, int64_t batch, hipStream_t st,
                                  double *w)
{
    if (p.L == 0 || !w) return hipErrorInvalidValue;
    switch (p.M) {
#define L2C_CASE(MM) \
    case MM: return run<MM>(p, in, out, batch, st, nullptr, w);
        L2C_FOR_EACH_RANK(L2C_CASE)
#undef L2C_CASE
    default: return hipErrorInvalidValue;
    }
}

}  // namespace l2c
