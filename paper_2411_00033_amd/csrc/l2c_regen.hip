// l2c_regen.hip -- far-field blocks recomputed in every execute instead of read from a
// stored table (plans made with L2C_TABLES_REGEN), for gfx950, FP64.
//
// A far-field submatrix is the 2-D DCT-II of the kernel sampled at the Chebyshev-Gauss
// points of its square (Eq. (aklmore)): Ahat = D S D^T, with D[k][m] = sc_k cos(k (m+1/2)
// pi / M), sc_0 = 1/M, sc_k = 2/M.  Its product with an upward vector is applied in that
// factored form, c = D (S (D^T w)), so the submatrix itself is never formed (3 M^2 instead
// of 2 M^3 + M^2 multiply-adds per submatrix and parity pair).  The samples factor as in
// Sec. 4.3: S[m][n] = Lambda((y-x)/2) Lambda((x+y)/2) for leg2cheb (Eq. (Aij)), and for
// cheb2leg the reverse kernel of Eq. (Lxymod), a rational factor times
// Lambda((y-x)/2) / Lambda((x+y)/2).  The first factor depends only on the level and on
// the submatrix's offset from the diagonal (2 h or 3 h, Eq. (globalij)): every plan keeps it
// as a table of 2 L M x M blocks (k_build_lminus; the plan's own k_build_ahat samples from
// it too).  The second is evaluated per sample in the execute.
//
// k_regen computes, for every block below the subtree roots of level groot (the blocks
// whose table the single-launch and three-launch paths stream), the far-field part of
// step (3) for its two row nodes, c(2b) = Ahat(.,0) w(2b+2) + Ahat(.,1) w(2b+3) and
// c(2b+1) = Ahat(.,2) w(2b+3), both parities, from the upward vectors k_up and k_top left
// in the workspace.  It writes them in k_main's order (per subtree, depth d at node
// 2^d - 2), and k_main reads them in place of its stream.  The blocks of levels
// 0..groot stay in the plan's (small) top table.
#include "l2c_alloc.h"
#include "l2c_device.h"

namespace l2c {

constexpr int kRegenThreads = 64;    // one wave per workgroup
constexpr int kRegenBlocks = 4;      // far-field blocks per workgroup (in sequence)

// Lambda((y - x)/2) for the submatrices of level g at offset dl h from the diagonal
// (dl = 2 + di), sample (m, n): table [g][di][m][n], g = 0..L-1.
template <int M>
__global__ void k_build_lminus(double *lm, Geometry G, const double *XG)
{
    const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (e >= (int64_t)G.L * 2 * M * M) return;
    const int mn = (int)(e % (M * M)), t = (int)(e / (M * M));
    const int di = t & 1, g = t >> 1;
    const int m = mn / M, n = mn % M;
    const double h = (double)((int64_t)G.s << (G.L - g - 1));
    lm[e] = lambda_real((2.0 + di) * h + 0.5 * h * (XG[n] - XG[m]));
}

// The series of Eq. (tau) in t = 1/x^2, and of its reciprocal (coefficients of 1/tau from
// those of tau by series division: 1/64, -19/2^13, 631/2^19, -174317/2^27); both accurate to
// about an ulp for x > 20.
__device__ __forceinline__ double tau_poly(double t)
{
    double p = 180323.0 / 134217728.0;
    p = fma(p, t, -671.0 / 524288.0);
    p = fma(p, t, 21.0 / 8192.0);
    p = fma(p, t, -1.0 / 64.0);
    return fma(p, t, 1.0);
}

__device__ __forceinline__ double inv_tau_poly(double t)
{
    double p = -174317.0 / 134217728.0;
    p = fma(p, t, 631.0 / 524288.0);
    p = fma(p, t, -19.0 / 8192.0);
    p = fma(p, t, 1.0 / 64.0);
    return fma(p, t, 1.0);
}

// 1/x and 1/sqrt(x) (x > 0, normal) from the hardware estimates and two Newton steps each
// (quadratic convergence; a few ulp), cheaper than the correctly rounded library sequences.
__device__ __forceinline__ double recip(double x)
{
    double r = __builtin_amdgcn_rcp(x);
    r = fma(r, fma(-x, r, 1.0), r);
    return fma(r, fma(-x, r, 1.0), r);
}

__device__ __forceinline__ double rsqrt_nr(double x)
{
    double y = __builtin_amdgcn_rsq(x);
    y = fma(0.5 * y, fma(-x * y, y, 1.0), y);
    return fma(0.5 * y, fma(-x * y, y, 1.0), y);
}

// Pair index pr of (m, n), m <= n, in row-major order of the upper triangle -> m.
template <int M>
__device__ __forceinline__ int pair_row(int pr)
{
    int m = 0;
    while (pr >= M - m) {
        pr -= M - m;
        ++m;
    }
    return m;
}

template <int M>
__global__ __launch_bounds__(kRegenThreads) void k_regen(ExecArgs a, const double *lm, const double *Dm,
                                                          const double *XG, double *cf)
{
    constexpr int MM = M * M, M2 = 2 * M, NPAIR = M * (M + 1) / 2;
    __shared__ double Dl[MM];
    __shared__ double Xl[M];
    __shared__ unsigned char Pm[NPAIR], Pn[NPAIR];   // pair index -> (m, n), m <= n
    __shared__ double Ph[NPAIR];                     // (X_m + X_n + 2) / 2 of the pair
    __shared__ double S[3 * MM];      // the three submatrices' samples, [r][m][n]
    __shared__ double W[2 * M2];      // w(2b+2), w(2b+3): [q][sigma][l]
    __shared__ double Uv[2 * M2];     // u = D^T w
    __shared__ double V[2 * M2];      // v = S u: [row node 2b or 2b+1][sigma][m]
    const Geometry &G = a.geo;
    const int kd = G.kd, groot = G.groot, L = G.L, s = G.s, dir = a.dir;
    const int nown = (1 << kd) - 1;                  // blocks per subtree
    const int own = 2 * (1 << kd) - 2;               // row nodes per subtree
    const int64_t U = int64_t(1) << (groot + 2);     // subtrees of an item
    const int64_t item = blockIdx.y;
    const int lane = threadIdx.x;
    // the scaled DCT matrix of Eq. (aklmore): Dl[k][m] = sc_k cos(k (m + 1/2) pi / M), sc_0 = 1/M,
    // sc_k = 2/M (D^T w reads it by columns, D v by rows)
    for (int e = lane; e < MM; e += kRegenThreads) Dl[e] = Dm[e] * ((e < M ? 1.0 : 2.0) / M);
    for (int pr = lane; pr < NPAIR; pr += kRegenThreads) {
        const int m = pair_row<M>(pr);
        Pm[pr] = (unsigned char)m;
        Pn[pr] = (unsigned char)(pr - (m * (2 * M - m + 1)) / 2 + m);
    }
    for (int e = lane; e < M; e += kRegenThreads) Xl[e] = XG[e];
    __syncthreads();
    for (int pr = lane; pr < NPAIR; pr += kRegenThreads) Ph[pr] = 0.5 * (Xl[Pm[pr]] + Xl[Pn[pr]] + 2.0);
    const double *wit = a.w + item * G.NT * M2;
    for (int bb = 0; bb < kRegenBlocks; ++bb) {
        const int64_t gblk = (int64_t)blockIdx.x * kRegenBlocks + bb;
        if (gblk >= U * nown) break;                 // uniform over the workgroup
        const int64_t Rn = gblk / nown;
        const int j = (int)(gblk - Rn * nown);
        int d, i;
        slot_depth(j, kd, d, i);
        const int g = groot + d;
        const int64_t b = (Rn << (d - 1)) + i;       // block b of level g
        double *co = cf + ((item * U + Rn) * own + (1 << d) - 2 + 2 * i) * M2;   // c(2i), c(2i+1)
        if (b >= (int64_t(1) << (g + 1)) - 1) {      // past the level's last block (Eq. (Nb))
            for (int e = lane; e < 2 * M2; e += kRegenThreads) co[e] = 0.0;
            continue;
        }
        __syncthreads();                             // the previous block's reads of W, S, V are done
        const double *wg = wit + (node_offset(g) + 2 * b + 2) * M2;   // w(2b+2), then w(2b+3)
        for (int e = lane; e < 2 * M2; e += kRegenThreads) W[e] = wg[e];
        // samples: x = i0 + h (X_m + 1), y = j0 + h (X_n + 1) with the corner of Eq. (globalij).
        // The factor in (x+y)/2 depends on X_m + X_n only: one evaluation per pair m <= n
        // serves samples (m, n) and (n, m) (M (M+1)/2 pairs per submatrix).
        const double h = (double)((int64_t)s << (L - g - 1));
        const double *lmg = lm + (int64_t)g * 2 * MM;
        for (int r = 0; r < 3; ++r) {                  // the submatrix: p, q and its row bases are uniform
            const int p = r == 2 ? 1 : 0, q = r == 0 ? 0 : 1;          // r = p + q (q + 1) / 2
            const double *lmr = lmg + (q + 2 - p - 2) * MM;             // offset (q + 2 - p) h
            const double zb = h * (double)(4 * b + p + q + 2);
            const double i0 = 2.0 * h * (double)(2 * b + p), j0 = 2.0 * h * (double)(2 * b + q + 2);
            double *Sr = S + r * MM;
#pragma unroll 2
            for (int pr = lane; pr < NPAIR; pr += kRegenThreads) {
                const int m = Pm[pr], n = Pn[pr];
                const double zp = zb + h * Ph[pr];
                // Lambda(zp) = tau(x) / sqrt(x), x = zp + 1/4 (Eq. (tau), zp >= 20): with rx = 1/x
                // and sr = 1/sqrt(x), tau(rx^2) sr; its reciprocal from the reciprocal series,
                // x sr / tau
                const bool big = zp >= 20.0;
                const double x = zp + 0.25, rx = recip(x), sr = rsqrt_nr(x), tt = rx * rx;
                if (dir == 0) {
                    const double lp = big ? tau_poly(tt) * sr : lambda_real(zp);
                    Sr[m * M + n] = lmr[m * M + n] * lp;
                    Sr[n * M + m] = lmr[n * M + m] * lp;
                } else {
                    // Eq. (Lxymod): 2 (x+1/2) y / ((x+y)(x+y+1)(x-y+1)) Lambda((y-x)/2) /
                    // Lambda((x+y)/2), one division for both samples of the pair
                    const double ilp = big ? inv_tau_poly(tt) * x * sr : 1.0 / lambda_real(zp);
                    const double xm = i0 + h * (Xl[m] + 1.0), yn = j0 + h * (Xl[n] + 1.0);
                    const double xn = i0 + h * (Xl[n] + 1.0), ym = j0 + h * (Xl[m] + 1.0);
                    const double sp = xm + yn;                                // = xn + ym
                    const double d1 = xm - yn + 1.0, d2 = xn - ym + 1.0;
                    const double c2 = ilp * recip(sp * (sp + 1.0) * d1 * d2);
                    Sr[m * M + n] = 2.0 * (xm + 0.5) * yn * d2 * c2 * lmr[m * M + n];
                    Sr[n * M + m] = 2.0 * (xn + 0.5) * ym * d1 * c2 * lmr[n * M + m];
                }
            }
        }
        __syncthreads();
        // The three products below take both parities per lane (one read of D or S serves
        // two multiply-adds): 2M lanes, one pass of the wave.
        // u = D^T w: u[q][sigma][n] = sum_l Dl[l][n] w[q][sigma][l]
        for (int e = lane; e < M2; e += kRegenThreads) {
            const int q = e / M, n = e - q * M;
            double a0 = 0.0, a1 = 0.0;
#pragma unroll
            for (int l = 0; l < M; ++l) {
                const double dv = Dl[l * M + n];
                a0 = fma(dv, W[(2 * q) * M + l], a0);
                a1 = fma(dv, W[(2 * q + 1) * M + l], a1);
            }
            Uv[(2 * q) * M + n] = a0;
            Uv[(2 * q + 1) * M + n] = a1;
        }
        __syncthreads();
        // v = S u: row node 2b takes S(0) u(2b+2) + S(1) u(2b+3), row node 2b+1 takes S(2) u(2b+3)
        for (int e = lane; e < M2; e += kRegenThreads) {
            const int t = e / M, m = e - t * M;
            double a0 = 0.0, a1 = 0.0;
            if (t == 0) {
#pragma unroll
                for (int n = 0; n < M; ++n) {
                    const double s0 = S[m * M + n], s1 = S[MM + m * M + n];
                    a0 = fma(s0, Uv[n], a0);
                    a0 = fma(s1, Uv[M2 + n], a0);
                    a1 = fma(s0, Uv[M + n], a1);
                    a1 = fma(s1, Uv[M2 + M + n], a1);
                }
            } else {
#pragma unroll
                for (int n = 0; n < M; ++n) {
                    const double s2 = S[2 * MM + m * M + n];
                    a0 = fma(s2, Uv[M2 + n], a0);
                    a1 = fma(s2, Uv[M2 + M + n], a1);
                }
            }
            V[t * M2 + m] = a0;
            V[t * M2 + M + m] = a1;
        }
        __syncthreads();
        // c = D v: c[k] = sum_m sc_k cos(k (m + 1/2) pi / M) v[m]
        for (int e = lane; e < M2; e += kRegenThreads) {
            const int t = e / M, k = e - t * M;
            double a0 = 0.0, a1 = 0.0;
#pragma unroll
            for (int m = 0; m < M; ++m) {
                const double dv = Dl[k * M + m];
                a0 = fma(dv, V[(2 * t) * M + m], a0);
                a1 = fma(dv, V[(2 * t + 1) * M + m], a1);
            }
            co[(2 * t) * M + k] = a0;
            co[(2 * t + 1) * M + k] = a1;
        }
    }
}

template <int M>
static hipError_t build_lm(const l2c_plan_s &p, hipStream_t st)
{
    const int64_t total = (int64_t)p.L * 2 * M * M;
    if (total <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_build_lminus<M>, dim3((unsigned)((total + 255) / 256)), dim3(256), 0, st, p.d_lm, p.geo,
                       (const double *)p.d_XG);
    return hipGetLastError();
}

template <int M>
static hipError_t run_regen(const l2c_plan_s &p, const ExecArgs &c, double *cf, hipStream_t st)
{
    const Geometry &G = p.geo;
    const int64_t blocks = (int64_t(1) << (G.groot + 2)) * ((1 << G.kd) - 1);
    if (G.kd < 1 || blocks == 0) return hipSuccess;
    const unsigned wgs = (unsigned)((blocks + kRegenBlocks - 1) / kRegenBlocks);
    hipLaunchKernelGGL(k_regen<M>, dim3(wgs, (unsigned)c.batch), dim3(kRegenThreads), 0, st, c,
                       (const double *)p.d_lm, (const double *)p.d_D, (const double *)p.d_XG, cf);
    return hipGetLastError();
}

hipError_t launch_build_lminus(const l2c_plan_s &p, hipStream_t st)
{
    switch (p.M) {
#define L2C_CASE(MM) \
    case MM: return build_lm<MM>(p, st);
        L2C_FOR_EACH_RANK(L2C_CASE)
#undef L2C_CASE
    default: return hipErrorInvalidValue;
    }
}

hipError_t launch_regen(const l2c_plan_s &p, const ExecArgs &c, double *cf, hipStream_t st)
{
    switch (p.M) {
#define L2C_CASE(MM) \
    case MM: return run_regen<MM>(p, c, cf, st);
        L2C_FOR_EACH_RANK(L2C_CASE)
#undef L2C_CASE
    default: return hipErrorInvalidValue;
    }
}

}  // namespace l2c
