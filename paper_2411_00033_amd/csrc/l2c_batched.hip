// l2c_batched.hip -- the batched execution form (precision L2C_FP32): the modal
// multipole transform (arXiv 2411.00033, Alg. 4) for 16 transforms at a time, every
// product of steps (1)-(6) on the gfx950 matrix cores with the batch as the product's
// column dimension.
//
// A "tile" is the 16 x 16 matrix [k][item] of one tree node and parity for the 16
// transforms of a workgroup row (blockIdx.y): the upward vectors w of Eq. (wTf) and
// the far-field coefficients c of Eq. (cfrompq) are tiles.  A tile lives in the
// matrix-core accumulator layout: lane l holds column l mod 16 (the item) and rows
// row(l / 16, r), r = 0..3.  The same four values are exactly the B operand of the
// next 16 x 16 x 4 product when its k-th step takes the rows row(q, kk): every product
// of the method that maps a tile to a tile (B(0), B(1), B(p)^T, Ahat, T(sigma)) is four
// matrix-core instructions on registers, with the A operand arranged to match.
//
//   kb_up    steps (0)-(2): one wave per 2^KU finest nodes; step (1) (Eq. (wMM)) reads
//            the input directly as the B operand (8 consecutive values per lane: both
//            parities of 4 modes), then the upward pass (Eq. (wtk)) runs in registers
//            as a depth-first walk; every w tile goes to the workspace.
//   kb_top   step (2) for KT levels above a level, leaves loaded from the workspace.
//   kb_main  steps (3)-(7): one wave per level-groot subtree of 2^KD finest row nodes.
//            The ancestors' c (levels 0..groot) come first (far-field blocks plus the
//            downward transfer of step (4)); a depth-first walk then produces each
//            finest node's c and evaluates it (Eq. (step5)) together with the near
//            field of step (6) as one accumulator: the near-diagonal band of one node and
//            parity is the dense s x 2s matrix P_{m'-m} Q_{S} (zero below the diagonal)
//            times the input, on the matrix cores, with its factors from LDS.
// The tables (Ahat in the A-operand order, T, B(0), P, Q) and the workspace hold the
// form's precision; inputs and outputs stay FP64 (converted on load, scaled by step (7)
// in FP64 on store).
#include "l2c_device.h"

namespace l2c {

template <typename T>
struct Mx;
template <>
struct Mx<float> {
    typedef float v4 __attribute__((ext_vector_type(4)));
    static __device__ __forceinline__ v4 mma(float a, float b, v4 c)
    {
        return __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c, 0, 0, 0);
    }
    // accumulator register r of lane group q holds row 4q + r
    static __host__ __device__ constexpr int row(int q, int r) { return 4 * q + r; }
};
template <>
struct Mx<double> {
    typedef double v4 __attribute__((ext_vector_type(4)));
    static __device__ __forceinline__ v4 mma(double a, double b, v4 c)
    {
        return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0);
    }
    static __host__ __device__ constexpr int row(int q, int r) { return q + 4 * r; }
};

template <typename T>
struct BTile {
    typename Mx<T>::v4 v[2];   // parity sigma = 0, 1
};

template <typename T>
struct BatArgs {
    const double *in;
    double *out;
    int64_t n;
    const int64_t *item_n;          // ragged batches (see ExecArgs)
    const double *const *item_in;
    double *const *item_out;
    int64_t batch;                  // items of this launch
    int dir, L, s, M;
    int gin;                        // kb_top: level of the loaded nodes
    int64_t NT;                     // workspace nodes per tile
    const T *ahat;                  // [blocks][3][64 lanes][4]: A operands, level-major blocks
    const T *Tm;                    // [2][s][M]
    const T *B0;                    // [M][M]
    const T *Pt;                    // [2s]: P_d
    const T *Qt;                    // [n_pad + 2s]: Q_S
    T *w;                           // [tiles][NT][2][64][4]
};

template <typename T>
__device__ __forceinline__ BTile<T> tile_zero()
{
    BTile<T> t;
    t.v[0] = typename Mx<T>::v4{0, 0, 0, 0};
    t.v[1] = t.v[0];
    return t;
}

template <typename T>
__device__ __forceinline__ T *tile_ptr(const BatArgs<T> &a, int64_t node, int sig, int lane)
{
    return a.w + (((int64_t)blockIdx.y * a.NT + node) * 2 + sig) * 256 + lane * 4;
}

template <typename T>
__device__ __forceinline__ BTile<T> tile_load(const BatArgs<T> &a, int64_t node, int lane)
{
    typedef typename Mx<T>::v4 v4;
    BTile<T> t;
    t.v[0] = *reinterpret_cast<const v4 *>(tile_ptr(a, node, 0, lane));
    t.v[1] = *reinterpret_cast<const v4 *>(tile_ptr(a, node, 1, lane));
    return t;
}

template <typename T>
__device__ __forceinline__ void tile_store(const BatArgs<T> &a, int64_t node, int lane, const BTile<T> &t)
{
    typedef typename Mx<T>::v4 v4;
    *reinterpret_cast<v4 *>(tile_ptr(a, node, 0, lane)) = t.v[0];
    *reinterpret_cast<v4 *>(tile_ptr(a, node, 1, lane)) = t.v[1];
}

// The lane's transform: item blockIdx.y * 16 + lane mod 16 (length 0 past the batch).
struct LaneItem {
    const double *in;
    double *out;
    int64_t n;
};

template <typename T>
__device__ __forceinline__ LaneItem lane_item(const BatArgs<T> &a, int lane)
{
    LaneItem it{nullptr, nullptr, 0};
    const int64_t item = (int64_t)blockIdx.y * 16 + (lane & 15);
    if (item < a.batch) {
        it.n = a.item_n ? a.item_n[item] : a.n;
        it.in = a.item_in ? a.item_in[item] : a.in + item * a.n;
        it.out = a.item_out ? a.item_out[item] : a.out + item * a.n;
    }
    return it;
}

// Eight consecutive input values x[e] = u[j0 + e] (zero past the item's length), with
// u = c .* f for cheb2leg (u_0 = 2 f_0, Sec. 4.1); times j for the near field's g_j = j u_j.
__device__ __forceinline__ void load8(const LaneItem &it, int64_t j0, int dir, bool times_j, double (&x)[8])
{
#pragma unroll
    for (int e = 0; e < 8; ++e) x[e] = (j0 + e < it.n) ? it.in[j0 + e] : 0.0;
    if (dir == 1) {
        if (j0 == 0) x[0] *= 2.0;
        if (times_j) {
#pragma unroll
            for (int e = 0; e < 8; ++e) x[e] *= (double)(j0 + e);
        }
    }
}

// t += Bm t_in for one tile and both parities, Bm given as the four A-operand values of
// the lane (Bm[l mod 16][row(l / 16, kk)]).
template <typename T>
__device__ __forceinline__ void tile_mac(BTile<T> &acc, const T (&am)[4], const BTile<T> &x)
{
#pragma unroll
    for (int sg = 0; sg < 2; ++sg) {
#pragma unroll
        for (int kk = 0; kk < 4; ++kk) acc.v[sg] = Mx<T>::mma(am[kk], x.v[sg][kk], acc.v[sg]);
    }
}

// ------------------------------------------------------------------------------------
// Upward pass.  Leaf tiles come from step (1) (LEAF_STEP1) or from the workspace.
template <typename T, int K, bool LEAF_STEP1>
__device__ __forceinline__ void up_walk(const BatArgs<T> &a, int64_t t0, int gleaf, int lane)
{
    typedef typename Mx<T>::v4 v4;
    const int li = lane & 15, q = lane >> 4;
    const int M = a.M, s = a.s;
    // A operands of the parent transfer: B(0) and B(1) = B(0) with odd diagonals negated
    T b0a[4], b1a[4];
#pragma unroll
    for (int kk = 0; kk < 4; ++kk) {
        const int k = Mx<T>::row(q, kk);
        const T v = (li < M && k < M) ? a.B0[li * M + k] : T(0);
        b0a[kk] = v;
        b1a[kk] = ((li - k) & 1) ? -v : v;
    }
    // A operands of step (1): T(sigma)^T, column m = 16 c + 4 q + kk
    T ta[2][2][4];
#pragma unroll
    for (int sg = 0; sg < 2; ++sg)
#pragma unroll
        for (int c = 0; c < 2; ++c)
#pragma unroll
            for (int kk = 0; kk < 4; ++kk) {
                const int m = 16 * c + 4 * q + kk;
                ta[sg][c][kk] = (LEAF_STEP1 && li < M && m < s) ? a.Tm[(sg * s + m) * M + li] : T(0);
            }
    LaneItem it{nullptr, nullptr, 0};
    if (LEAF_STEP1) it = lane_item(a, lane);

    BTile<T> stk[K > 0 ? K : 1];
    for (int i = 0; i < (1 << K); ++i) {
        const int64_t t = t0 + i;
        BTile<T> cur;
        if (LEAF_STEP1) {
            // step (1): w_k(t, sigma) = sum_m T_k(X_m^sigma) u[2 s t + 2 m + sigma]
            cur = tile_zero<T>();
#pragma unroll
            for (int c = 0; c < 2; ++c) {
                if (16 * c < s) {
                    double x[8];
                    load8(it, 2 * s * t + 32 * c + 8 * q, a.dir, false, x);
#pragma unroll
                    for (int kk = 0; kk < 4; ++kk) {
                        const bool in_node = 16 * c + 4 * q + kk < s;
#pragma unroll
                        for (int sg = 0; sg < 2; ++sg)
                            cur.v[sg] = Mx<T>::mma(ta[sg][c][kk], in_node ? (T)x[2 * kk + sg] : T(0), cur.v[sg]);
                    }
                }
            }
            tile_store(a, node_offset(gleaf) + t, lane, cur);
        } else {
            cur = tile_load(a, node_offset(gleaf) + t, lane);
        }
        // climb while this node is a right child: parent = B(0) left + B(1) right (Eq. (wtk))
        bool done = false;
#pragma unroll
        for (int d = 1; d <= K; ++d) {
            if (!done) {
                if (((i >> (d - 1)) & 1) == 0) {
                    stk[d - 1] = cur;
                    done = true;
                } else {
                    BTile<T> par = tile_zero<T>();
                    tile_mac(par, b0a, stk[d - 1]);
                    tile_mac(par, b1a, cur);
                    cur = par;
                    tile_store(a, node_offset(gleaf - d) + (t >> d), lane, cur);
                }
            }
        }
    }
    (void)sizeof(v4);
}

template <typename T, int KU>
__global__ __launch_bounds__(256) void kb_up(BatArgs<T> a)
{
    const int lane = threadIdx.x & 63;
    const int64_t sub = (int64_t)blockIdx.x * 4 + wave_id();
    const int64_t P = int64_t(1) << (a.L + 1);   // finest nodes
    if ((sub << KU) >= P) return;
    up_walk<T, KU, true>(a, sub << KU, a.L - 1, lane);
}

template <typename T, int KT>
__global__ __launch_bounds__(256) void kb_top(BatArgs<T> a)
{
    const int lane = threadIdx.x & 63;
    const int64_t sub = (int64_t)blockIdx.x * 4 + wave_id();
    if ((sub << KT) >= (int64_t(1) << (a.gin + 2))) return;
    up_walk<T, KT, false>(a, sub << KT, a.gin, lane);
}

// ------------------------------------------------------------------------------------
// Far field of one row node v of level g (step (3), Eq. (cfrompq)): block b = v >> 1,
// c(2b) = Ahat(0) w(2b+2) + Ahat(1) w(2b+3), c(2b+1) = Ahat(2) w(2b+3); zero when the
// block lies past the last one of the level (b >= b_g = 2^(g+1) - 1).
template <typename T>
__device__ __forceinline__ BTile<T> far_tile(const BatArgs<T> &a, int g, int64_t v, int lane)
{
    typedef typename Mx<T>::v4 v4;
    BTile<T> r = tile_zero<T>();
    const int64_t b = v >> 1;
    if (b >= (int64_t(1) << (g + 1)) - 1) return r;
    const int64_t blk = level_block_offset(g) + b;
    const T *ab = a.ahat + (blk * 3 * 64 + lane) * 4;
    if ((v & 1) == 0) {
        const v4 A0 = *reinterpret_cast<const v4 *>(ab);
        const v4 A1 = *reinterpret_cast<const v4 *>(ab + 64 * 4);
        const BTile<T> w2 = tile_load(a, node_offset(g) + v + 2, lane);
        const BTile<T> w3 = tile_load(a, node_offset(g) + v + 3, lane);
        const T a0[4] = {A0[0], A0[1], A0[2], A0[3]}, a1[4] = {A1[0], A1[1], A1[2], A1[3]};
        tile_mac(r, a0, w2);
        tile_mac(r, a1, w3);
    } else {
        const v4 A2 = *reinterpret_cast<const v4 *>(ab + 2 * 64 * 4);
        const BTile<T> w2 = tile_load(a, node_offset(g) + v + 2, lane);
        const T a2[4] = {A2[0], A2[1], A2[2], A2[3]};
        tile_mac(r, a2, w2);
    }
    return r;
}

// Steps (5)-(7) for finest row node u: z = T(sigma) c(u) (row nodes u < P - 2) plus the
// near field, then the scaling of step (7) and the FP64 store.
template <typename T>
__device__ __forceinline__ void leaf_eval(const BatArgs<T> &a, int64_t u, const BTile<T> &cu, const T (&te)[2][2][4],
                                          const T *Pl, T *Ql, const LaneItem &it, int lane)
{
    typedef typename Mx<T>::v4 v4;
    const int li = lane & 15, q = lane >> 4;
    const int s = a.s, dir = a.dir;
    const int64_t P = int64_t(1) << (a.L + 1);
    const int64_t base = 2 * s * u;                      // first row of the node
    // Q_S for S = base + [0, 3s): the node's window, through this wave's LDS area
    for (int e = lane; e < 3 * s; e += 64) Ql[e] = a.Qt[base + e];
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_s_waitcnt(0xc07f);
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
    const int nrt = s > 16 ? 2 : 1;
    v4 acc[2][2];
#pragma unroll
    for (int sg = 0; sg < 2; ++sg)
#pragma unroll
        for (int rt = 0; rt < 2; ++rt) acc[sg][rt] = v4{0, 0, 0, 0};
    // far part (Eq. (step5)): rows m = 16 rt + l mod 16 of T(sigma), modes row(q, kk)
    if (u < P - 2) {
#pragma unroll
        for (int sg = 0; sg < 2; ++sg)
#pragma unroll
            for (int rt = 0; rt < 2; ++rt)
                if (rt < nrt) {
#pragma unroll
                    for (int kk = 0; kk < 4; ++kk) acc[sg][rt] = Mx<T>::mma(te[sg][rt][kk], cu.v[sg][kk], acc[sg][rt]);
                }
    }
    // near field (step (6)): row m, column m' = 16 c + 4 q + kk of parity sigma:
    //   rs_i P_{m'-m} Q_{base + sigma + m + m'} for m <= m' < 2s, times g_{base + 2 m' + sigma}
    const int nc = (2 * s + 15) / 16;
    for (int c = 0; c < nc; ++c) {
        double x[8];
        load8(it, base + 32 * c + 8 * q, dir, true, x);
#pragma unroll
        for (int sg = 0; sg < 2; ++sg) {
#pragma unroll
            for (int rt = 0; rt < 2; ++rt) {
                if (rt < nrt && c >= rt) {
                    const int m = 16 * rt + li;
                    const double rs = dir == 1 ? 2.0 * (double)(base + 2 * m + sg) + 1.0 : 1.0;
#pragma unroll
                    for (int kk = 0; kk < 4; ++kk) {
                        const int mp = 16 * c + 4 * q + kk;
                        const bool nz = m < s && mp >= m && mp < 2 * s;
                        const T pq = nz ? Pl[nz ? mp - m : 0] * Ql[nz ? sg + m + mp : 0] : T(0);
                        acc[sg][rt] = Mx<T>::mma(pq * (T)rs, (T)x[2 * kk + sg], acc[sg][rt]);
                    }
                }
            }
        }
    }
    // step (7) and output: lane holds rows m = 16 rt + row(q, r) of item l mod 16
    if (!it.out) return;
    const double f0 = (dir == 1 && base == 0 && it.n > 0) ? it.in[0] : 0.0;
#pragma unroll
    for (int rt = 0; rt < 2; ++rt) {
        if (rt < nrt) {
#pragma unroll
            for (int r = 0; r < 4; ++r) {
                const int m = 16 * rt + Mx<T>::row(q, r);
#pragma unroll
                for (int sg = 0; sg < 2; ++sg) {
                    const int64_t i = base + 2 * m + sg;
                    if (m < s && i < it.n) {
                        double v = (double)acc[sg][rt][r];
                        if (dir == 0) v *= (i == 0 ? 1.0 / kPi : 2.0 / kPi);
                        else if (i == 0) v += f0;   // K_00 u_0 = u_0 / 2 = f_0
                        it.out[i] = v;
                    }
                }
            }
        }
    }
}

template <typename T, int KD>
__global__ __launch_bounds__(256) void kb_main(BatArgs<T> a)
{
    __shared__ T Pl[64];
    __shared__ T Qs[4][96];
    const int lane = threadIdx.x & 63, wv = wave_id();
    const int li = lane & 15, q = lane >> 4;
    const int s = a.s, M = a.M;
    for (int e = threadIdx.x; e < 2 * s; e += 256) Pl[e] = a.Pt[e];
    __syncthreads();
    const int groot = a.L - 1 - KD;
    const int64_t Rn = (int64_t)blockIdx.x * 4 + wv;
    if (Rn >= (int64_t(1) << (groot + 2))) return;
    const LaneItem it = lane_item(a, lane);

    // A operands: B(p)^T (step (4)) and T(sigma) (Eq. (step5))
    T bt[2][4], te[2][2][4];
#pragma unroll
    for (int kk = 0; kk < 4; ++kk) {
        const int k = Mx<T>::row(q, kk);
        const T v = (li < M && k < M) ? a.B0[k * M + li] : T(0);
        bt[0][kk] = v;
        bt[1][kk] = ((k - li) & 1) ? -v : v;
    }
#pragma unroll
    for (int sg = 0; sg < 2; ++sg)
#pragma unroll
        for (int rt = 0; rt < 2; ++rt)
#pragma unroll
            for (int kk = 0; kk < 4; ++kk) {
                const int m = 16 * rt + li, k = Mx<T>::row(q, kk);
                te[sg][rt][kk] = (m < s && k < M) ? a.Tm[(sg * s + m) * M + k] : T(0);
            }

    // ancestors a_g = Rn >> (groot - g): c(a_0) = far; c(a_g) = far + B(p)^T c(a_{g-1})
    BTile<T> cp = far_tile(a, 0, Rn >> groot, lane);
    for (int g = 1; g <= groot; ++g) {
        const int64_t v = Rn >> (groot - g);
        BTile<T> cv = far_tile(a, g, v, lane);
        tile_mac(cv, bt[v & 1], cp);
        cp = cv;
    }
    // depth-first walk over the subtree: stk[d] = c of the current node at depth d
    BTile<T> stk[KD + 1];
    stk[0] = cp;
    for (int i = 0; i < (1 << KD); ++i) {
        // depths whose node changes at leaf i: d > KD - ctz(i) (all for i = 0)
        const int dmin = i == 0 ? 1 : KD - __builtin_ctz(i) ;
#pragma unroll
        for (int d = 1; d <= KD; ++d) {
            if (d >= dmin) {
                const int64_t v = (Rn << d) + (i >> (KD - d));
                BTile<T> cv = far_tile(a, groot + d, v, lane);
                tile_mac(cv, bt[v & 1], stk[d - 1]);
                stk[d] = cv;
            }
        }
        leaf_eval(a, (Rn << KD) + i, stk[KD], te, Pl, Qs[wv], it, lane);
    }
}

// ------------------------------------------------------------------------------------
// Plan-time helpers: Ahat (FP64 plan tables) -> A-operand order of the form's type;
// Q_S for S < len.
template <typename T, int M>
__global__ void kb_pack_ahat(const double *top, const double *bot, Geometry G, T *dst, int64_t blocks)
{
    const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;   // (blk, r, lane, kk)
    if (e >= blocks * 3 * 256) return;
    const int kk = (int)(e & 3), lane = (int)((e >> 2) & 63);
    const int64_t br = e >> 8;
    const int r = (int)(br % 3);
    int64_t b = br / 3;
    int g = 0;
    while (b >= (int64_t(1) << (g + 1)) - 1) {
        b -= (int64_t(1) << (g + 1)) - 1;
        ++g;
    }
    const int k = lane & 15, l = Mx<T>::row(lane >> 4, kk);
    double v = 0.0;
    if (k < M && l < M) {
        if (g <= G.groot) {
            v = top[((level_block_offset(g) + b) * 3 + r) * M * M + k * M + l];
        } else {
            constexpr int NCH = 3 * M / 2;
            const int d = g - G.groot;
            const int64_t Rn = b >> (d - 1);
            const int64_t j = ((int64_t(1) << G.kd) - (int64_t(1) << d)) + (b - (Rn << (d - 1)));
            const int64_t slot = j * M + k;
            const int64_t grp = Rn * G.sub_groups + slot / 64;
            const int ln = (int)(slot % 64);
            const int el = r * M + l;
            v = bot[((grp * NCH + el / 2) * 64 + ln) * 2 + (el & 1)];
        }
    }
    dst[e] = (T)v;
}

template <typename T>
__global__ void kb_q_table(T *Qt, int64_t len, int dir)
{
    const int64_t S = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (S < len) Qt[S] = (T)near_Q(dir, S);
}

template <typename T, int M>
static hipError_t pack(const l2c_plan_s &p, void *dst, hipStream_t st)
{
    const int64_t blocks = level_block_offset(p.L);
    const int64_t total = blocks * 3 * 256;
    hipLaunchKernelGGL((kb_pack_ahat<T, M>), dim3((unsigned)((total + 255) / 256)), dim3(256), 0, st, p.d_top,
                       p.d_bot, p.geo, (T *)dst, blocks);
    return hipGetLastError();
}

hipError_t batched_build_tables(const l2c_plan_s &p, void *ahat_dst, void *q_dst, int64_t q_len, hipStream_t st)
{
    hipError_t e;
    switch (p.M) {
    case 12: e = pack<float, 12>(p, ahat_dst, st); break;
    case 16: e = pack<float, 16>(p, ahat_dst, st); break;
    default: return hipErrorInvalidValue;
    }
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(kb_q_table<float>, dim3((unsigned)((q_len + 255) / 256)), dim3(256), 0, st, (float *)q_dst,
                       q_len, p.direction);
    return hipGetLastError();
}

// ------------------------------------------------------------------------------------
template <typename T>
static hipError_t run_batched(const l2c_plan_s &p, const double *in, double *out, int64_t batch, hipStream_t st,
                              const ItemArrays *ia)
{
    const int L = p.L;
    const int ku = L - 1 < kBatUpDepth ? L - 1 : kBatUpDepth;
    const int kd = L - 1 < kBatMainDepth ? L - 1 : kBatMainDepth;
    const int64_t Pn = int64_t(1) << (L + 1);
    for (int64_t b0 = 0; b0 < batch; b0 += kBatMaxTiles * 16) {
        const int64_t nb = batch - b0 < kBatMaxTiles * 16 ? batch - b0 : kBatMaxTiles * 16;
        const unsigned tiles = (unsigned)((nb + 15) / 16);
        BatArgs<T> a;
        a.in = ia ? nullptr : in + b0 * p.n;
        a.out = ia ? nullptr : out + b0 * p.n;
        a.n = p.n;
        a.item_n = ia ? ia->n + b0 : nullptr;
        a.item_in = ia ? ia->in + b0 : nullptr;
        a.item_out = ia ? ia->out + b0 : nullptr;
        a.batch = nb;
        a.dir = p.direction;
        a.L = L;
        a.s = p.s;
        a.M = p.M;
        a.gin = 0;
        a.NT = p.geo.NT;
        a.ahat = (const T *)p.d_bA;
        a.Tm = (const T *)p.d_bT;
        a.B0 = (const T *)p.d_bB;
        a.Pt = (const T *)p.d_bP;
        a.Qt = (const T *)p.d_bQ;
        a.w = (T *)p.d_bw;
        {
            const unsigned gx = (unsigned)(((Pn >> ku) + 3) / 4);
            switch (ku) {
#define L2C_UP(KK) \
    case KK: hipLaunchKernelGGL((kb_up<T, KK>), dim3(gx, tiles), dim3(256), 0, st, a); break;
                L2C_UP(0) L2C_UP(1) L2C_UP(2) L2C_UP(3)
#undef L2C_UP
            default: return hipErrorInvalidValue;
            }
        }
        for (int gin = L - 1 - ku; gin > 0;) {
            const int kt = gin < kBatTopDepth ? gin : kBatTopDepth;
            const int gout = gin - kt;
            a.gin = gin;
            const unsigned gx = (unsigned)((((int64_t)1 << (gout + 2)) + 3) / 4);
            switch (kt) {
#define L2C_TOP(KK) \
    case KK: hipLaunchKernelGGL((kb_top<T, KK>), dim3(gx, tiles), dim3(256), 0, st, a); break;
                L2C_TOP(1) L2C_TOP(2) L2C_TOP(3)
#undef L2C_TOP
            default: return hipErrorInvalidValue;
            }
            gin = gout;
        }
        {
            const int groot = L - 1 - kd;
            const unsigned gx = (unsigned)((((int64_t)1 << (groot + 2)) + 3) / 4);
            switch (kd) {
#define L2C_MAIN(KK) \
    case KK: hipLaunchKernelGGL((kb_main<T, KK>), dim3(gx, tiles), dim3(256), 0, st, a); break;
                L2C_MAIN(0) L2C_MAIN(1) L2C_MAIN(2) L2C_MAIN(3)
#undef L2C_MAIN
            default: return hipErrorInvalidValue;
            }
        }
        const hipError_t e = hipGetLastError();
        if (e != hipSuccess) return e;
    }
    return hipSuccess;
}

hipError_t launch_batched(const l2c_plan_s &p, const double *in, double *out, int64_t batch, hipStream_t st,
                          const ItemArrays *ia)
{
    if (p.L < 1 || p.s > 32 || p.M > 16) return hipErrorInvalidValue;
    return run_batched<float>(p, in, out, batch, st, ia);
}

}  // namespace l2c
