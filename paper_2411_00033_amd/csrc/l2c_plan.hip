// l2c_plan.hip -- device part of the plan stage (arXiv 2411.00033, Secs. 3.2 and 4.3).
//
// k_build_ahat: one wave per block (g, b) of the decomposition, adjacent blocks of a level
// in one workgroup (so that the rows they share in the far-field tables meet in one L2);
// for each of its
// three submatrices r = (p,q) it samples the kernel at the M x M Chebyshev-Gauss
// points of its domain [i, i+2h] x [j, j+2h] (Eq. (aklmore)),
//     x_m = i + h (X_m + 1),  y_n = j + h (X_n + 1),  X_m = cos((m+1/2) pi / M),
// with the leg2cheb kernel A(x,y) = Lambda((y-x)/2) Lambda((y+x)/2) (Sec. 3.2) or the
// cheb2leg kernel of Eq. (Lxymod), and applies the 2-D DCT-II
//     ahat_kl = 4/(c_k c_l M^2) sum_m sum_n K(x_m, y_n) D_km D_ln,  D_km = cos(k (m+1/2) pi / M),
// as two M x M x M products: each lane holds one row of the samples (then one column of
// the partial product) in registers, and the DCT matrix enters as operands that are the
// same for every lane.  All in FP64.  Results go straight into the
// far-field tables that k_main reads (layouts in l2c_internal.h).  For the nodal basis
// (Eq. (AijLag)) the samples K(x_k, y_l) themselves are the far-field blocks.
//
// k_build_small makes the Vandermonde matrices T(sigma) of Eq. (Xs), the near-field factor
// P_d, the Chebyshev-Gauss points and the DCT matrix, also in FP64 on the device.
//
// Two of the paper's planning shortcuts (Sec. 4.3) cut the Lambda evaluations per block
// from 6 M^2 to 3 M (M+1)/2: the factor Lambda((y-x)/2) depends only on the level and the
// submatrix's offset from the diagonal, and comes from a table built once per plan
// (k_build_lminus, l2c_regen.hip); the factor in (x+y)/2 is symmetric in the sample
// indices and is evaluated once per pair m <= n.  (Its other shortcuts, term dropping in
// Eq. (tau) and a radix-2/3 DCT of size 18, save CPU flops that do not bound this kernel.)
#include "l2c_internal.h"
#include "l2c_math.h"

namespace l2c {

constexpr int kAhatWaves = 4;                     // k_build_ahat: blocks (one per wave) per workgroup

// Address (in doubles) of element (r, k, l) of block b of level g in the plan tables.
template <int M>
__device__ __forceinline__ double *ahat_addr(double *top, double *bot, const Geometry &G, int g, int64_t b,
                                             int r, int k, int l)
{
    constexpr int NCH = 3 * M / 2;
    if (g <= G.groot) return top + ((level_block_offset(g) + b) * 3 + r) * M * M + k * M + l;
    const int d = g - G.groot;                      // depth below the subtree root
    const int64_t Rn = b >> (d - 1);                // subtree of the block
    const int64_t j = ((int64_t(1) << G.kd) - (int64_t(1) << d)) + (b - (Rn << (d - 1)));   // finest depth first
    const int64_t slot = j * M + k;
    const int64_t grp = Rn * G.sub_groups + slot / 64;
    const int lane = (int)(slot % 64);
    const int el = r * M + l;
    return bot + ((grp * NCH + el / 2) * 64 + lane) * 2 + (el & 1);
}

template <int M>
__global__ __launch_bounds__(64 * kAhatWaves) void k_build_ahat(double *top, double *bot, Geometry G, int dir,
                                                                const double *XG, const double *__restrict__ Dm,
                                                                int nodal, const double *lm, int64_t nblocks)
{
    constexpr int MM = M * M, NPAIR = M * (M + 1) / 2;
    __shared__ double Sw[kAhatWaves][3 * MM];        // per wave: the samples, then S D^T
    __shared__ double Xl[M];
    __shared__ unsigned char pm[NPAIR], pn[NPAIR];    // pair index -> (m, n), m <= n
    const int tid = threadIdx.x, wave = tid >> 6, lane = tid & 63;
    for (int e = tid; e < M; e += 64 * kAhatWaves) Xl[e] = XG[e];
    for (int e = tid; e < NPAIR; e += 64 * kAhatWaves) {
        int pr = e, m = 0;
        while (pr >= M - m) {
            pr -= M - m;
            ++m;
        }
        pm[e] = (unsigned char)m;
        pn[e] = (unsigned char)(m + pr);
    }
    __syncthreads();
    // one block (level g, block b) per wave; adjacent blocks of a level in one workgroup
    const int64_t blk = (int64_t)blockIdx.x * kAhatWaves + wave;
    const bool act = blk < nblocks;
    int64_t gb = act ? blk : 0;
    int g = 0;
    while (gb >= (int64_t(1) << (g + 1)) - 1) {
        gb -= (int64_t(1) << (g + 1)) - 1;
        ++g;
    }
    const int64_t b = gb;
    const double h = (double)((int64_t)G.s << (G.L - g - 1));
    double *S = Sw[wave];

    // samples (m, n) and (n, m) of submatrix r from one Lambda((x+y)/2); per submatrix, p, q,
    // the factor table's rows and the corner are the same for the whole wave
    if (act) {
        for (int r = 0; r < 3; ++r) {
            const int p = (r == 2) ? 1 : 0, q = (r == 0) ? 0 : 1;   // r = p + q(q+1)/2
            const double i0 = 2.0 * h * (double)(2 * b + p);        // Eq. (globalij)
            const double j0 = 2.0 * h * (double)(2 * b + q + 2);
            const double *lmr = lm + ((int64_t)g * 2 + (q - p)) * MM;   // offset (q + 2 - p) h
            const double zb = h * (double)(4 * b + p + q + 2);
            for (int pr = lane; pr < NPAIR; pr += 64) {
                const int m = pm[pr], n = pn[pr];
                const double zp = zb + 0.5 * h * (Xl[m] + Xl[n] + 2.0);
                double vmn, vnm;
                if (dir == 0) {
                    const double lp = lambda_real(zp);
                    vmn = lmr[m * M + n] * lp;
                    vnm = lmr[n * M + m] * lp;
                } else {
                    // Eq. (Lxymod): 2 (x+1/2) y / ((x+y)(x+y+1)(x-y+1)) Lambda((y-x)/2) / Lambda((x+y)/2)
                    const double ilp = 1.0 / lambda_real(zp);
                    const double xm = i0 + h * (Xl[m] + 1.0), yn = j0 + h * (Xl[n] + 1.0);
                    const double xn = i0 + h * (Xl[n] + 1.0), ym = j0 + h * (Xl[m] + 1.0);
                    const double sp = xm + yn;
                    vmn = 2.0 * (xm + 0.5) * yn / (sp * (sp + 1.0) * (xm - yn + 1.0)) * ilp * lmr[m * M + n];
                    vnm = 2.0 * (xn + 0.5) * ym / (sp * (sp + 1.0) * (xn - ym + 1.0)) * ilp * lmr[n * M + m];
                }
                S[r * MM + m * M + n] = vmn;
                S[r * MM + n * M + m] = vnm;
                if (nodal) {
                    *ahat_addr<M>(top, bot, G, g, b, r, m, n) = vmn;
                    *ahat_addr<M>(top, bot, G, g, b, r, n, m) = vnm;
                }
            }
        }
    }
    if (nodal) return;                                // uniform: no barrier follows
    __syncthreads();
    // U[r][m][l] = sum_n S[r][m][n] D[l][n]: one row (r, m) per lane, held in registers; D is
    // the same for every lane (scalar operands).  Each lane rewrites only its own row.
    if (act) {
        for (int t = lane; t < 3 * M; t += 64) {
            double srow[M];
#pragma unroll
            for (int n = 0; n < M; ++n) srow[n] = S[t * M + n];
#pragma unroll
            for (int l = 0; l < M; ++l) {
                double acc = 0.0;
#pragma unroll
                for (int n = 0; n < M; ++n) acc = fma(srow[n], Dm[l * M + n], acc);
                S[t * M + l] = acc;
            }
        }
    }
    __syncthreads();
    // ahat[r][k][l] = 4/(c_k c_l M^2) sum_m D[k][m] U[r][m][l]: one column (r, l) per lane
    if (act) {
        for (int t = lane; t < 3 * M; t += 64) {
            const int r = t / M, l = t - r * M;
            double ucol[M];
#pragma unroll
            for (int m = 0; m < M; ++m) ucol[m] = S[r * MM + m * M + l];
#pragma unroll
            for (int k = 0; k < M; ++k) {
                double acc = 0.0;
#pragma unroll
                for (int m = 0; m < M; ++m) acc = fma(Dm[k * M + m], ucol[m], acc);
                const double sc = 4.0 / ((k == 0 ? 2.0 : 1.0) * (l == 0 ? 2.0 : 1.0) * M * M);
                *ahat_addr<M>(top, bot, G, g, b, r, k, l) = acc * sc;
            }
        }
    }
}

// Plan tables -> canonical [level][block][r][k][l].
template <int M>
__global__ void k_export_ahat(double *top, double *bot, Geometry G, double *dst, int64_t total)
{
    const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (e >= total) return;
    int64_t blk = e / (3 * M * M);
    const int rem = (int)(e - blk * 3 * M * M);
    const int r = rem / (M * M), k = (rem / M) % M, l = rem % M;
    int g = 0;
    while (blk >= (int64_t(1) << (g + 1)) - 1) {
        blk -= (int64_t(1) << (g + 1)) - 1;
        ++g;
    }
    dst[e] = *ahat_addr<M>(top, bot, G, g, blk, r, k, l);
}

// The plan's small tables, one thread per entry:
//   T[sigma][m][k] = T_k(X), X = -1 + (2m + sigma)/s (Eq. (Xs)), by the three-term recurrence;
//   P[e] = 0 for e < kPLead, then the near-field factor P_d, d = e - kPLead (lambda_d for
//          leg2cheb, lambda_d / (1 - 2d) for cheb2leg, Eq. (Lxymod));
//   XG[m] = cos((m + 1/2) pi / M) and Dm[k][m] = cos(k (m + 1/2) pi / M) (Eq. (aklmore)).
__global__ void k_build_small(double *T, double *P, double *XG, double *Dm, int s, int M, int dir, int plen)
{
    int e = blockIdx.x * blockDim.x + threadIdx.x;
    const int nt = 2 * s * M;
    if (e < nt) {
        const int k = e % M, sm = e / M, m = sm % s, sig = sm / s;
        const double X = -1.0 + (double)(2 * m + sig) / (double)s;
        double t0 = 1.0, t1 = X;
        for (int j = 0; j < k; ++j) {
            const double t2 = 2.0 * X * t1 - t0;
            t0 = t1;
            t1 = t2;
        }
        T[e] = t0;
        return;
    }
    e -= nt;
    if (e < plen) {
        const int d = e - kPLead;
        double v = 0.0;
        if (d >= 0) {
            const double lam = lambda_int(d);
            v = dir == 0 ? lam : lam / (1.0 - 2.0 * (double)d);
        }
        P[e] = v;
        return;
    }
    e -= plen;
    if (e < M) {
        XG[e] = cos((e + 0.5) * kPi / M);
        return;
    }
    e -= M;
    if (e < M * M) {
        const int k = e / M, m = e % M;
        Dm[e] = cos(k * (m + 0.5) * kPi / M);
    }
}

__global__ void k_to_f32(const double *src, float *dst, int64_t n)
{
    const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (e < n) dst[e] = (float)src[e];
}

hipError_t launch_build_small(const l2c_plan_s &p, hipStream_t st)
{
    const int total = 2 * p.s * p.M + (int)p_table_len(p.s) + p.M + p.M * p.M;
    hipLaunchKernelGGL(k_build_small, dim3((total + 255) / 256), dim3(256), 0, st, p.d_T, p.d_P, p.d_XG, p.d_D, p.s,
                       p.M, p.direction, (int)p_table_len(p.s));
    return hipGetLastError();
}

hipError_t launch_to_f32(const double *src, float *dst, int64_t n, hipStream_t st)
{
    if (n <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_to_f32, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, st, src, dst, n);
    return hipGetLastError();
}

template <int M>
static hipError_t build(const l2c_plan_s &p, hipStream_t st)
{
    // plans that regenerate the blocks below the subtree roots store levels 0..groot only
    // (the first blocks of the level-major enumeration)
    const int64_t blocks = p.regen ? level_block_offset(p.geo.groot + 1) : p.nb;
    if (blocks <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_build_ahat<M>, dim3((unsigned)((blocks + kAhatWaves - 1) / kAhatWaves)),
                       dim3(64 * kAhatWaves), 0, st, p.d_top, p.d_bot, p.geo, p.direction, p.d_XG,
                       (const double *)p.d_D, p.basis, (const double *)p.d_lm, blocks);
    return hipGetLastError();
}

template <int M>
static hipError_t xport(const l2c_plan_s &p, double *dst, hipStream_t st)
{
    const int64_t total = p.nc * M * M;
    hipLaunchKernelGGL(k_export_ahat<M>, dim3((unsigned)((total + 255) / 256)), dim3(256), 0, st, p.d_top,
                       p.d_bot, p.geo, dst, total);
    return hipGetLastError();
}

hipError_t launch_build_ahat(const l2c_plan_s &p, hipStream_t st)
{
    switch (p.M) {
#define L2C_CASE(MM) \
    case MM: return build<MM>(p, st);
        L2C_FOR_EACH_RANK(L2C_CASE)
#undef L2C_CASE
    default: return hipErrorInvalidValue;
    }
}

hipError_t launch_export_ahat(const l2c_plan_s &p, double *dst, hipStream_t st)
{
    switch (p.M) {
#define L2C_CASE(MM) \
    case MM: return xport<MM>(p, dst, st);
        L2C_FOR_EACH_RANK(L2C_CASE)
#undef L2C_CASE
    default: return hipErrorInvalidValue;
    }
}

}  // namespace l2c
