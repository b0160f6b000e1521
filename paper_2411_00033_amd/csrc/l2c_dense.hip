// l2c_dense.hip -- batches of short FP64 transforms by the direct product of Alg. 1
// (arXiv 2411.00033) on the FP64 matrix cores.
//
// For n up to kDenseMaxN (4096; up to there this path is faster than the multipole kernels
// on batches, by measurement) the plan stores, per parity sigma, the dense upper-triangular
// matrix D(sigma)[i'][j'] of the coefficients of f_j in z_i (i = 2i' + sigma,
// j = 2j' + sigma; a_ij is zero when j - i is odd):
//   leg2cheb: lambda_{(j-i)/2} lambda_{(i+j)/2} / (c_i pi / 2)          (Eqs. (aij), (AfCf))
//   cheb2leg: (2i+1) P_{(j-i)/2} Q_{(i+j)/2} j for j >= 1, and 1 at (0, 0)  (Eq. (Lxymod) with
//             u = c .* f, regrouped as in the near field)
// An execute is then, per parity, Z(sigma) = F(sigma) D(sigma)^T over the batch: FP64
// 16 x 16 x 4 matrix-core products, each workgroup 64 transforms x 64 outputs per parity,
// K in chunks of 16 staged through LDS (the next chunk loaded while one is multiplied),
// chunks below the diagonal skipped.  At these sizes the direct product needs more flops
// than the multipole method (about 4x at n = 1024) but runs at the matrix cores' rate,
// while the multipole kernels give each small subtree a whole latency-bound workgroup.
#include "l2c_device.h"

namespace l2c {

typedef double d4v __attribute__((ext_vector_type(4)));

__global__ void kd_build(double *D, int64_t n, int64_t HP, int dir)
{
    const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;   // (sigma, i', j')
    if (e >= 2 * HP * HP) return;
    const int sg = (int)(e / (HP * HP));
    const int64_t r = e - sg * HP * HP, ip = r / HP, jp = r - ip * HP;
    const int64_t i = 2 * ip + sg, j = 2 * jp + sg;
    double v = 0.0;
    if (jp >= ip && j < n) {
        const int64_t d = jp - ip, S = ip + jp + sg;
        if (dir == 0) {
            v = near_P(0, d) * near_Q(0, S) * (i == 0 ? 1.0 / kPi : 2.0 / kPi);
        } else {
            v = (i == 0 && j == 0) ? 1.0 : (2.0 * (double)i + 1.0) * near_P(1, d) * near_Q(1, S) * (double)j;
        }
    }
    D[e] = v;
}

constexpr int kDS = 17;   // LDS row stride (doubles): odd, distinct banks across rows

__global__ __launch_bounds__(256) void kd_dense(const double *in, double *out, int64_t n, int64_t batch,
                                                const int64_t *item_n, const double *const *item_in,
                                                double *const *item_out, const double *D, int64_t HP)
{
    __shared__ double Fs[2][64][kDS];
    __shared__ double Ds[2][64][kDS];
    const int tid = threadIdx.x, lane = tid & 63, wv = tid >> 6;
    const int li = lane & 15, lq = lane >> 4;
    const int64_t item0 = (int64_t)blockIdx.x * 64;
    const int64_t ob = blockIdx.y;                 // outputs i' in [64 ob, 64 ob + 64)
    // loader: row tid / 4 of the tile, part tid mod 4
    const int lr = tid >> 2, lp = tid & 3;
    const int64_t lit = item0 + lr;
    const double *rowp = nullptr;
    int64_t rn = 0;
    if (lit < batch) {
        rn = item_n ? item_n[lit] : n;
        rowp = item_in ? item_in[lit] : in + lit * n;
    }
    const int kc0 = 4 * (int)ob, kcN = (int)(HP / 16);   // chunks of 16 j'; j' >= i' >= 64 ob
    // this thread's D rows (one per parity), from column 4 lp on
    const double *drow0 = D + (64 * ob + lr) * HP + 4 * lp, *drow1 = drow0 + HP * HP;
    double fv[8], dv[2][4];
    auto load = [&](int kc) {
        const int64_t j0 = 32 * kc + 8 * lp;         // both parities of j' = 16 kc + 4 lp + e/2
        if (j0 + 8 <= rn) {                           // the whole segment inside the row
#pragma unroll
            for (int e = 0; e < 8; ++e) fv[e] = rowp[j0 + e];
        } else {
#pragma unroll
            for (int e = 0; e < 8; ++e) fv[e] = (j0 + e < rn) ? rowp[j0 + e] : 0.0;
        }
#pragma unroll
        for (int e = 0; e < 4; ++e) {
            dv[0][e] = drow0[16 * kc + e];
            dv[1][e] = drow1[16 * kc + e];
        }
    };
    d4v acc[2][4];
#pragma unroll
    for (int sg = 0; sg < 2; ++sg)
#pragma unroll
        for (int ct = 0; ct < 4; ++ct) acc[sg][ct] = d4v{0.0, 0.0, 0.0, 0.0};
    if (kc0 < kcN) load(kc0);
    for (int kc = kc0; kc < kcN; ++kc) {
        __syncthreads();                            // the previous chunk's reads are done
#pragma unroll
        for (int e = 0; e < 8; ++e) Fs[e & 1][lr][4 * lp + (e >> 1)] = fv[e];
#pragma unroll
        for (int sg = 0; sg < 2; ++sg)
#pragma unroll
            for (int e = 0; e < 4; ++e) Ds[sg][lr][4 * lp + e] = dv[sg][e];
        __syncthreads();
        if (kc + 1 < kcN) load(kc + 1);
        // A = F (16 transforms x 4 j'), B = D^T (4 j' x 16 outputs); lane l supplies
        // A[l % 16][l / 16], B[l / 16][l % 16] and holds D rows 4q + l / 16 (q = register)
#pragma unroll
        for (int st = 0; st < 4; ++st) {
            const int k = 4 * st + lq;
#pragma unroll
            for (int sg = 0; sg < 2; ++sg) {
                const double a = Fs[sg][16 * wv + li][k];
#pragma unroll
                for (int ct = 0; ct < 4; ++ct)
                    acc[sg][ct] = __builtin_amdgcn_mfma_f64_16x16x4f64(a, Ds[sg][16 * ct + li][k], acc[sg][ct], 0, 0, 0);
            }
        }
    }
    // outputs: transform 16 wv + 4 q + l / 16, row i = 2 (64 ob + 16 ct + l % 16) + sigma
#pragma unroll
    for (int q = 0; q < 4; ++q) {
        const int64_t it = item0 + 16 * wv + 4 * q + lq;
        if (it >= batch) continue;
        const int64_t nr = item_n ? item_n[it] : n;
        double *o = item_out ? item_out[it] : out + it * n;
#pragma unroll
        for (int ct = 0; ct < 4; ++ct)
#pragma unroll
            for (int sg = 0; sg < 2; ++sg) {
                const int64_t i = 2 * (64 * ob + 16 * ct + li) + sg;
                if (i < nr) o[i] = acc[sg][ct][q];
            }
    }
}

int64_t dense_hp(int64_t n) { return (((n + 1) / 2 + 63) / 64) * 64; }

hipError_t dense_build(const l2c_plan_s &p, double *D, hipStream_t st)
{
    const int64_t HP = dense_hp(p.n), total = 2 * HP * HP;
    hipLaunchKernelGGL(kd_build, dim3((unsigned)((total + 255) / 256)), dim3(256), 0, st, D, p.n, HP, p.direction);
    return hipGetLastError();
}

hipError_t launch_dense(const l2c_plan_s &p, const double *in, double *out, int64_t batch, hipStream_t st,
                        const ItemArrays *ia)
{
    const int64_t HP = dense_hp(p.n);
    for (int64_t b0 = 0; b0 < batch; b0 += kMaxItemsPerLaunch * 64) {
        const int64_t nb = batch - b0 < kMaxItemsPerLaunch * 64 ? batch - b0 : kMaxItemsPerLaunch * 64;
        const dim3 grid((unsigned)((nb + 63) / 64), (unsigned)(HP / 64));
        const bool timed = p.ev_before && p.ev_after && b0 == 0;
        if (timed) (void)hipEventRecord(p.ev_before, st);
        hipLaunchKernelGGL(kd_dense, grid, dim3(256), 0, st, ia ? nullptr : in + b0 * p.n,
                           ia ? nullptr : out + b0 * p.n, p.n, nb, ia ? ia->n + b0 : nullptr,
                           ia ? ia->in + b0 : nullptr, ia ? ia->out + b0 : nullptr, (const double *)p.d_dense, HP);
        if (timed) (void)hipEventRecord(p.ev_after, st);
        const hipError_t e = hipGetLastError();
        if (e != hipSuccess) return e;
    }
    return hipSuccess;
}

}  // namespace l2c
