// l2c_exec.hip -- execution kernels of the modal multipole Legendre <-> Chebyshev
// transform (arXiv 2411.00033, Alg. 4) for gfx950, FP64.
//
// One execute is four launches on the caller's stream:
//   k_up    steps (0)+(1)+(2): stage the input (zero padding, c .* f for cheb2leg),
//           contract each finest node with T(sigma) (Eq. (wMM)) and run the upward
//           pass (Eq. (wtk), with the even/odd-diagonal split of App. A2) inside a
//           subtree of 2^ku finest nodes; writes w for every level of the subtree.
//   k_top   step (2) for the levels above the subtree roots (one workgroup per item).
//   k_far   step (3): every far-field product c(g,b,p) = sum_q Ahat(g,b,r) w(g,b,q)
//           of every level, streaming the Ahat table once per launch (the dominant
//           HBM traffic); Ahat rows stay in registers and are applied to up to
//           kFarItems batch items.
//   k_down  steps (4)-(7): per subtree of 2^kd finest nodes, spread c down from level
//           0 (each workgroup walks its own chain of ancestors), evaluate
//           z = T(sigma) c at the finest level (Eq. (step5)), add the near-diagonal
//           direct part (step (6)), scale (step (7)) and write the output.
// Plans with L = 0 use k_direct (Alg. 1 for every row).
#include "l2c_internal.h"
#include "l2c_math.h"

namespace l2c {

__device__ __forceinline__ int wave_id() { return __builtin_amdgcn_readfirstlane(threadIdx.x >> 6); }

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

// ------------------------------------------------------------------------------------
// k_up: one workgroup per (subtree of 2^ku finest nodes, item).
// LDS: f chunk [nodes][D] (D >= 2s, row stride padded against bank conflicts),
//      w for every subtree level, B(0).
template <int M>
__global__ __launch_bounds__(kThreads) void k_up(ExecArgs a)
{
    extern __shared__ double lds[];
    const int s = a.s, L = a.L, ku = a.ku;
    const int nodes = 1 << ku;
    const int64_t item = blockIdx.y;
    const int64_t t0 = (int64_t)blockIdx.x << ku;    // first finest node of the subtree
    const int D = (s & 1) ? 2 * s : 2 * s + 2;        // D = 2 (mod 4) doubles
    double *fl = lds;                                 // nodes * D
    double *wl = fl + nodes * D;                      // sum_d 2^(ku-d) nodes * 2M
    double *Bl = wl + (2 * nodes - 1) * 2 * M;        // M * M
    const int tid = threadIdx.x;

    for (int e = tid; e < M * M; e += kThreads) Bl[e] = a.B0[e];
    // stage the input: zero past n; cheb2leg uses u = c .* f (u_0 = 2 f_0), Sec. 4.1
    const double *in = a.in + item * a.n;
    const int64_t base = t0 * 2 * s;
    for (int e = tid; e < nodes * 2 * s; e += kThreads) {
        const int nd = e / (2 * s), m = e - nd * 2 * s;
        const int64_t gi = base + e;
        double v = gi < a.n ? in[gi] : 0.0;
        if (a.dir == 1 && gi == 0) v *= 2.0;
        fl[nd * D + m] = v;
    }
    __syncthreads();

    // step (1): w_k(t, sigma) = sum_m T_k(X_m^sigma) f[2s t + 2m + sigma]  (Eq. (wMM)).
    // Wave -> (sigma, half of k); lane -> node; T is wave-uniform (scalar loads).
    {
        constexpr int KH = M / 2;
        const int wv = wave_id();
        const int sig = wv & 1, kb = (wv >> 1) * KH;
        const double *Ts = a.T + (size_t)sig * s * M + kb;
        for (int nd = tid & 63; nd < nodes; nd += 64) {
            double acc[KH];
#pragma unroll
            for (int k = 0; k < KH; ++k) acc[k] = 0.0;
            const double *fr = fl + nd * D + sig;
            for (int m = 0; m < s; ++m) {
                const double fv = fr[2 * m];
#pragma unroll
                for (int k = 0; k < KH; ++k) acc[k] = fma(Ts[m * M + k], fv, acc[k]);
            }
            double *wo = wl + nd * 2 * M + sig * M + kb;
#pragma unroll
            for (int k = 0; k < KH; ++k) wo[k] = acc[k];
        }
    }
    __syncthreads();

    // step (2) inside the subtree: w(parent) = B(0) w(2T) + B(1) w(2T+1) (Eq. (wtk)).
    // B(1) = B(0) with odd diagonals negated (App. A2): with z0 = w(2T)+w(2T+1),
    // z1 = w(2T)-w(2T+1), out_n = sum_{k<=n} b_nk z_{(n-k) mod 2, k}.
    {
        double *child = wl;
        int cn = nodes;
        for (int d = 1; d <= ku; ++d) {
            double *par = child + cn * 2 * M;
            const int pn = cn >> 1;
            for (int e = tid; e < pn * 2 * M; e += kThreads) {
                const int pnode = e / (2 * M), r = e - pnode * 2 * M;
                const int sig = r / M, nn = r - sig * M;
                const double *wa = child + (2 * pnode) * 2 * M + sig * M;
                const double *wb = wa + 2 * M;
                double acc = 0.0;
                for (int k = 0; k <= nn; ++k) {
                    const double zk = ((nn - k) & 1) ? wa[k] - wb[k] : wa[k] + wb[k];
                    acc = fma(Bl[nn * M + k], zk, acc);
                }
                par[e] = acc;
            }
            __syncthreads();
            child = par;
            cn = pn;
        }
    }

    // write w of every subtree level to the workspace
    {
        double *wg = a.w + item * a.NT * 2 * M;
        const double *src = wl;
        int cn = nodes;
        for (int d = 0; d <= ku; ++d) {
            const int g = L - 1 - d;
            double *dst = wg + (node_offset(g) + (t0 >> d)) * 2 * M;
            for (int e = tid; e < cn * 2 * M; e += kThreads) dst[e] = src[e];
            src += cn * 2 * M;
            cn >>= 1;
        }
    }
}

// ------------------------------------------------------------------------------------
// k_top: step (2) for levels g0-1 .. 0 (g0 = level of the k_up subtree roots).
template <int M>
__global__ __launch_bounds__(1024) void k_top(ExecArgs a, int g0)
{
    __shared__ double Bl[M * M];
    const int64_t item = blockIdx.x;
    for (int e = threadIdx.x; e < M * M; e += blockDim.x) Bl[e] = a.B0[e];
    __syncthreads();
    double *wg = a.w + item * a.NT * 2 * M;
    for (int g = g0 - 1; g >= 0; --g) {
        const int pn = 1 << (g + 2);
        const double *child = wg + node_offset(g + 1) * 2 * M;
        double *par = wg + node_offset(g) * 2 * M;
        for (int e = threadIdx.x; e < pn * 2 * M; e += blockDim.x) {
            const int pnode = e / (2 * M), r = e - pnode * 2 * M;
            const int sig = r / M, nn = r - sig * M;
            const double *wa = child + (2 * pnode) * 2 * M + sig * M;
            const double *wb = wa + 2 * M;
            double acc = 0.0;
            for (int k = 0; k <= nn; ++k) {
                const double zk = ((nn - k) & 1) ? wa[k] - wb[k] : wa[k] + wb[k];
                acc = fma(Bl[nn * M + k], zk, acc);
            }
            par[e] = acc;
        }
        __syncthreads();
    }
}

// ------------------------------------------------------------------------------------
// k_far: step (3) for all levels.  Wave <-> 64 slots of the far-field table; lane
// (b, k) computes, for both parities,
//     c(2b)[k]   = Ahat(b,0)[k,:] w(2b+2) + Ahat(b,1)[k,:] w(2b+3)
//     c(2b+1)[k] = Ahat(b,2)[k,:] w(2b+3)
// (row node 2b+p, column node 2b+q+2, r = p + q(q+1)/2).  The 3M doubles of a slot are
// loaded once (coalesced 16-byte chunks) and applied to kFarItems items.
template <int M>
__global__ __launch_bounds__(kThreads) void k_far(ExecArgs a, FarLayout lay)
{
    constexpr int NCH = 3 * M / 2;
    const int64_t grp = (int64_t)blockIdx.x * (kThreads / 64) + wave_id();
    if (grp >= lay.group_off[lay.L]) return;
    int g = 0;
    while (grp >= lay.group_off[g + 1]) ++g;
    const int lane = threadIdx.x & 63;
    const int64_t slot = (grp - lay.group_off[g]) * 64 + lane;
    const int64_t b = slot / M;
    const int k = (int)(slot - b * M);
    const int64_t nblk = (int64_t(1) << (g + 1)) - 1;

    double2 ar[NCH];
    const double2 *src = reinterpret_cast<const double2 *>(a.ahat) + grp * NCH * 64 + lane;
#pragma unroll
    for (int ch = 0; ch < NCH; ++ch) ar[ch] = src[ch * 64];
    if (b >= nblk) return;

    const double *A0 = reinterpret_cast<const double *>(ar);
    const int64_t rown = node_offset(g) + 2 * b;   // row node 2b; column nodes 2b+2, 2b+3
    const int64_t it0 = (int64_t)blockIdx.y * kFarItems;
    const int64_t it1 = min(it0 + (int64_t)kFarItems, a.batch);
    for (int64_t it = it0; it < it1; ++it) {
        const double *wt = a.w + (it * a.NT + rown + 2) * 2 * M;   // w(2b+2), then w(2b+3)
        double c00 = 0, c01 = 0, c10 = 0, c11 = 0;                 // c(row p)[sigma]
#pragma unroll
        for (int l = 0; l < M; ++l) {
            const double w20 = wt[l], w21 = wt[M + l];
            const double w30 = wt[2 * M + l], w31 = wt[3 * M + l];
            c00 = fma(A0[l], w20, c00);
            c01 = fma(A0[l], w21, c01);
            c00 = fma(A0[M + l], w30, c00);
            c01 = fma(A0[M + l], w31, c01);
            c10 = fma(A0[2 * M + l], w30, c10);
            c11 = fma(A0[2 * M + l], w31, c11);
        }
        double *co = a.c + (it * a.NT + rown) * 2 * M + k;
        co[0] = c00;
        co[M] = c01;
        co[2 * M] = c10;
        co[3 * M] = c11;
    }
}

// ------------------------------------------------------------------------------------
// k_down: one workgroup per (subtree of 2^kd finest nodes, item).
template <int M>
__global__ __launch_bounds__(kThreads) void k_down(ExecArgs a)
{
    constexpr int R = kNearRows;
    extern __shared__ double lds[];
    const int s = a.s, L = a.L, kd = a.kd, dir = a.dir;
    const int nodes = 1 << kd;
    const int64_t item = blockIdx.y;
    const int64_t u0 = (int64_t)blockIdx.x << kd;    // first finest row node
    const int64_t P = int64_t(1) << (L + 1);          // finest nodes
    const int groot = L - 1 - kd;                     // level of the subtree root
    const int GS = 2 * s + R;                         // per (node, parity) g segment
    const int nQ = 2 * s * nodes + s + 2 * R;         // Q_S for S = 2s u0 + [0, nQ)
    const int nP = 2 * s + 2 * R;                     // P_d for d = [-(R-1), nP - R + 1)
    const int tid = threadIdx.x;

    double *Bl = lds;                                 // M*M
    double *Tl = Bl + M * M;                          // 2*s*M
    double *cl = Tl + 2 * s * M;                      // (2*nodes) * 2M: chain + subtree levels
    double *gl = cl + 2 * nodes * 2 * M;              // nodes * 2 * GS
    double *Ql = gl + nodes * 2 * GS;                 // nQ
    double *Pl = Ql + nQ;                             // nP
    double *zl = Pl + nP;                             // nodes * 2s

    for (int e = tid; e < M * M; e += kThreads) Bl[e] = a.B0[e];
    for (int e = tid; e < 2 * s * M; e += kThreads) Tl[e] = a.T[e];
    // g_j for j in node u and u+1, split by parity: gl[(u*2+sig)*GS + m'] = g[2s u + 2m' + sig]
    const double *in = a.in + item * a.n;
    const int64_t jb = u0 * 2 * s;
    for (int e = tid; e < nodes * 2 * GS; e += kThreads) {
        const int seg = e / GS, mp = e - seg * GS;
        const int nd = seg >> 1, sig = seg & 1;
        double v = 0.0;
        if (mp < 2 * s) {
            const int64_t j = jb + (int64_t)nd * 2 * s + 2 * mp + sig;
            if (j < a.n) {
                v = in[j];
                if (dir == 1) v *= (double)j;  // g_j = j u_j (u_j = f_j for j >= 1; g_0 = 0)
            }
        }
        gl[e] = v;
    }
    for (int e = tid; e < nQ; e += kThreads) Ql[e] = near_Q(dir, jb + e);
    for (int e = tid; e < nP; e += kThreads) {
        const int d = e - (R - 1);
        Pl[e] = d < 0 ? 0.0 : near_P(dir, d);
    }

    // steps (4): chain of ancestors, level 0 .. groot, then the subtree levels.
    // c_acc(child) = c_far(child) + B(p)^T c_acc(parent), p = child & 1; with
    // B(1) = B(0) with odd diagonals negated: (B(p)^T c)_n = sum_{k>=n} b_kn (+-1)^(k-n) c_k.
    const double *cfar = a.c + item * a.NT * 2 * M;
    double *chain = cl;                               // 2M, the running ancestor
    double *sub = cl + 2 * M;                         // subtree levels 1..kd (2^d nodes each)
    for (int g = 0; g <= groot; ++g) {
        const int64_t node = u0 >> (kd + groot - g);
        const bool has = node < (int64_t(1) << (g + 2)) - 2;
        double v = 0.0;
        if (tid < 2 * M) {
            const int sig = tid / M, nn = tid - sig * M;
            if (has) v = cfar[(node_offset(g) + node) * 2 * M + tid];
            if (g > 0) {
                const int p = (int)(node & 1);
                const double *cp = chain + sig * M;
                double acc = 0.0;
                for (int k = nn; k < M; ++k) {
                    const double bv = Bl[k * M + nn];
                    acc = fma((p && ((k - nn) & 1)) ? -bv : bv, cp[k], acc);
                }
                v += acc;
            }
        }
        __syncthreads();
        if (tid < 2 * M) chain[tid] = v;
        __syncthreads();
    }
    {
        const double *par = chain;
        double *cur = sub;
        for (int d = 1; d <= kd; ++d) {
            const int g = groot + d;
            const int cn = 1 << d;
            const int64_t first = u0 >> (kd - d);
            for (int e = tid; e < cn * 2 * M; e += kThreads) {
                const int v = e / (2 * M), r = e - v * 2 * M;
                const int sig = r / M, nn = r - sig * M;
                const int64_t node = first + v;
                double acc = 0.0;
                if (node < (int64_t(1) << (g + 2)) - 2) acc = cfar[(node_offset(g) + node) * 2 * M + r];
                const int p = v & 1;
                const double *cp = par + (v >> 1) * 2 * M + sig * M;
                for (int k = nn; k < M; ++k) {
                    const double bv = Bl[k * M + nn];
                    acc = fma((p && ((k - nn) & 1)) ? -bv : bv, cp[k], acc);
                }
                cur[e] = acc;
            }
            __syncthreads();
            par = cur;
            cur += cn * 2 * M;
        }
    }
    // the finest-level c of the subtree: level kd of `sub`, i.e. after 2 + 4 + ... + 2^(kd-1) nodes
    const double *cfine = kd > 0 ? sub + ((1 << kd) - 2) * 2 * M : chain;

    // step (5): z(u)[2m + sig] = sum_k T_k(X_m^sig) c(u)[sig][k] for row nodes u < P - 2
    for (int e = tid; e < nodes * 2 * s; e += kThreads) {
        const int nd = e / (2 * s), rr = e - nd * 2 * s;
        const int m = rr >> 1, sig = rr & 1;
        double acc = 0.0;
        if (u0 + nd < P - 2) {
            const double *cc = cfine + nd * 2 * M + sig * M;
            const double *tt = Tl + (sig * s + m) * M;
#pragma unroll
            for (int k = 0; k < M; ++k) acc = fma(tt[k], cc[k], acc);
        }
        zl[e] = acc;
    }
    __syncthreads();

    // step (6): near field.  Thread <-> (node, parity, R consecutive same-parity rows);
    // row m (of the node's s rows of this parity) sums over m' in [m, 2s):
    //   P[m'-m] Q[2s u + sig + m + m'] g[2s u + 2m' + sig].
    // P, Q and g enter through small circular windows so each step costs 3 LDS reads
    // for R rows.
    const int nch = (s + R - 1) / R;
    for (int wi = tid; wi < nodes * 2 * nch; wi += kThreads) {
        const int ch = wi % nch;
        const int seg = wi / nch;
        const int nd = seg >> 1, sig = seg & 1;
        const int m0 = ch * R;
        const double *gs = gl + seg * GS;
        const double *qs = Ql + nd * 2 * s + sig + m0;   // Q index for row m0 + r at m': qs[r + m']
        const double *ps = Pl + (R - 1) - m0;            // P index for row m0 + r at m': ps[m' - r]
        double acc[R], pb[R], qb[R];
#pragma unroll
        for (int r = 0; r < R; ++r) {
            acc[r] = 0.0;
            pb[r] = 0.0;  // P at negative offsets
        }
#pragma unroll
        for (int r = 0; r < R - 1; ++r) qb[(m0 + r) % R] = qs[m0 + r];
        const int steps = ((2 * s - m0) + R - 1) / R;
        for (int st = 0; st < steps; ++st) {
            const int mb = m0 + st * R;
#pragma unroll
            for (int t = 0; t < R; ++t) {
                const int mp = mb + t;                    // m' ; mp % R == t
                pb[t] = ps[mp];                           // P[m' - m0]
                qb[(t + R - 1) % R] = qs[mp + R - 1];     // Q for row R-1
                const double gv = gs[mp];
#pragma unroll
                for (int r = 0; r < R; ++r)
                    acc[r] = fma(pb[(t - r + R) % R] * qb[(t + r) % R], gv, acc[r]);
            }
        }
        // step (7) pieces: row scales, diagonal special case; accumulate into z
#pragma unroll
        for (int r = 0; r < R; ++r) {
            const int m = m0 + r;
            if (m < s) {
                const int zi = nd * 2 * s + 2 * m + sig;
                const int64_t i = jb + zi;
                double v = acc[r];
                if (dir == 1) {
                    v *= 2.0 * (double)i + 1.0;
                    if (i == 0) v += in[0];      // K_00 u_0 = u_0 / 2 = f_0
                }
                zl[zi] += v;
            }
        }
    }
    __syncthreads();

    // step (7): leg2cheb divides by c_i pi/2; write out the valid part
    double *out = a.out + item * a.n;
    for (int e = tid; e < nodes * 2 * s; e += kThreads) {
        const int64_t i = jb + e;
        if (i < a.n) {
            double v = zl[e];
            if (dir == 0) v /= (i == 0 ? kPi : 0.5 * kPi);
            out[i] = v;
        }
    }
}

// ------------------------------------------------------------------------------------
// k_direct: plans with L = 0 (n <= leaf): the whole product directly (Alg. 1 per row).
__global__ __launch_bounds__(kThreads) void k_direct(const double *in, double *out, int64_t n, int dir)
{
    extern __shared__ double lds[];
    double *gl = lds;          // n
    double *Ql = gl + n;       // n
    double *Pl = Ql + n;       // n
    const int64_t item = blockIdx.x;
    const double *x = in + item * n;
    for (int64_t e = threadIdx.x; e < n; e += kThreads) {
        double v = x[e];
        if (dir == 1) v *= (double)e;
        gl[e] = v;
        Ql[e] = near_Q(dir, e);
        Pl[e] = near_P(dir, e);
    }
    __syncthreads();
    for (int64_t i = threadIdx.x; i < n; i += kThreads) {
        double acc = 0.0;
        for (int64_t j = i; j < n; j += 2) acc = fma(Pl[(j - i) / 2] * Ql[(i + j) / 2], gl[j], acc);
        if (dir == 1) {
            acc *= 2.0 * (double)i + 1.0;
            if (i == 0) acc += x[0];
        } else {
            acc /= (i == 0 ? kPi : 0.5 * kPi);
        }
        out[item * n + i] = acc;
    }
}

// ------------------------------------------------------------------------------------
static size_t up_lds_bytes(int s, int M, int ku)
{
    const int nodes = 1 << ku;
    const int D = (s & 1) ? 2 * s : 2 * s + 2;
    return sizeof(double) * ((size_t)nodes * D + (size_t)(2 * nodes - 1) * 2 * M + (size_t)M * M);
}

static size_t down_lds_bytes(int s, int M, int kd)
{
    const int R = kNearRows, nodes = 1 << kd;
    const size_t GS = 2 * s + R;
    const size_t nQ = 2 * (size_t)s * nodes + s + 2 * R;
    const size_t nP = 2 * s + 2 * R;
    return sizeof(double) * ((size_t)M * M + 2 * (size_t)s * M + (size_t)2 * nodes * 2 * M +
                             (size_t)nodes * 2 * GS + nQ + nP + (size_t)nodes * 2 * s);
}

template <int M>
static hipError_t run(const l2c_plan_s &p, const double *in, double *out, int64_t batch, hipStream_t st)
{
    ExecArgs a;
    a.in = in;
    a.out = out;
    a.n = p.n;
    a.n_pad = p.n_pad;
    a.batch = batch;
    a.L = p.L;
    a.s = p.s;
    a.M = M;
    a.dir = p.direction;
    a.ku = p.L - 1 < kUpDepth ? p.L - 1 : kUpDepth;
    a.kd = p.L - 1 < kDownDepth ? p.L - 1 : kDownDepth;
    a.T = p.d_T;
    a.B0 = p.d_B;
    a.ahat = p.d_ahat;
    a.w = p.d_w;
    a.c = p.d_c;
    a.NT = p.NT;
    const int64_t P = int64_t(1) << (p.L + 1);
    const size_t up_lds = up_lds_bytes(p.s, M, a.ku), down_lds = down_lds_bytes(p.s, M, a.kd);
    static bool attr_set = false;   // allow the full 160 KiB LDS of a gfx950 CU
    if (!attr_set) {
        (void)hipFuncSetAttribute((const void *)k_up<M>, hipFuncAttributeMaxDynamicSharedMemorySize, 160 * 1024);
        (void)hipFuncSetAttribute((const void *)k_down<M>, hipFuncAttributeMaxDynamicSharedMemorySize, 160 * 1024);
        attr_set = true;
    }

    // grid.y carries the item index; at most kMaxItemsPerLaunch items per launch
    const int g0 = p.L - 1 - a.ku;
    const int64_t groups = p.far.group_off[p.L];
    for (int64_t b0 = 0; b0 < batch; b0 += kMaxItemsPerLaunch) {
        ExecArgs c = a;
        c.batch = batch - b0 < kMaxItemsPerLaunch ? batch - b0 : kMaxItemsPerLaunch;
        c.in = in + b0 * p.n;
        c.out = out + b0 * p.n;
        c.w = p.d_w + b0 * p.NT * 2 * M;
        c.c = p.d_c + b0 * p.NT * 2 * M;
        const unsigned items = (unsigned)c.batch;
        hipLaunchKernelGGL(k_up<M>, dim3((unsigned)(P >> a.ku), items), dim3(kThreads), up_lds, st, c);
        if (g0 > 0) hipLaunchKernelGGL(k_top<M>, dim3(items), dim3(1024), 0, st, c, g0);
        const unsigned fx = (unsigned)((groups + 3) / 4);
        const unsigned fy = (unsigned)((c.batch + kFarItems - 1) / kFarItems);
        const bool timed = p.ev_before && p.ev_after && b0 == 0;
        if (timed) (void)hipEventRecord(p.ev_before, st);
        hipLaunchKernelGGL(k_far<M>, dim3(fx, fy), dim3(kThreads), 0, st, c, p.far);
        if (timed) (void)hipEventRecord(p.ev_after, st);
        hipLaunchKernelGGL(k_down<M>, dim3((unsigned)(P >> a.kd), items), dim3(kThreads), down_lds, st, c);
    }
    return hipGetLastError();
}

hipError_t launch_execute(const l2c_plan_s &p, const double *in, double *out, int64_t batch, hipStream_t st)
{
    if (p.L == 0) {
        if (p.ev_before && p.ev_after) (void)hipEventRecord(p.ev_before, st);
        hipLaunchKernelGGL(k_direct, dim3((unsigned)batch), dim3(kThreads), 3 * sizeof(double) * p.n, st,
                           in, out, p.n, p.direction);
        if (p.ev_before && p.ev_after) (void)hipEventRecord(p.ev_after, st);
        return hipGetLastError();
    }
    switch (p.M) {
#define L2C_CASE(MM) \
    case MM: return run<MM>(p, in, out, batch, st);
        L2C_FOR_EACH_RANK(L2C_CASE)
#undef L2C_CASE
    default: return hipErrorInvalidValue;
    }
}

}  // namespace l2c
