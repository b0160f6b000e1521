// l2c_batched.hip -- the batched execution forms (precisions L2C_FP32, L2C_BF16X2 and
// L2C_FP16X2, and the FP64 tile form): the modal multipole transform (arXiv 2411.00033,
// Alg. 4) for 16 transforms at a time, every product of steps (1)-(6) on the gfx950 matrix
// cores with the batch as the product's column dimension.  The far part (steps (1)-(5))
// takes FP32 products, or BF16 or FP16 hi+lo products, with FP32 accumulation; the near
// field of step (6) (the dense near-diagonal leaf blocks, where the largest terms and
// their cancellations sit) and the sum of the two parts are FP64 in every form.
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
//            finest node's c and evaluates it (Eq. (step5)), and adds the near field of
//            step (6): the near-diagonal band of one node and parity is the dense s x 2s
//            matrix P_{m'-m} Q_{S} (zero below the diagonal) times the input, on the FP64
//            matrix cores, with its factors and the staged input from LDS.
// The far-part tables (Ahat in the A-operand order, T, B(0)) and the workspace hold the
// form's precision, the near-field tables (P, Q) FP64; inputs and outputs stay FP64
// (converted on load for the far part, scaled by step (7) in FP64 on store).
#include <type_traits>

#include "l2c_device.h"
#include "../../include/leg2cheb.h"

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
// The FP64 tile form: the same 16 x 16 x 4 shape on the FP64 matrix cores, whose
// accumulator register r of lane group q holds row 4r + q.  Every operand of the forms is
// built through row(q, r), so the step k of a product pairs the same rows on both sides.
template <>
struct Mx<double> {
    typedef double v4 __attribute__((ext_vector_type(4)));
    static __device__ __forceinline__ v4 mma(double a, double b, v4 c)
    {
        return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0);
    }
    static __host__ __device__ constexpr int row(int q, int r) { return 4 * r + q; }
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
    const float *ahat_inv;          // FP16X2: [blocks][3] factor that undoes a submatrix's scaling
    const T *Tm;                    // [2][s][M]
    const T *B0;                    // [M][M]
    const T *B1;                    // [M][M], nodal basis; null: B(1) = B(0) with odd diagonals negated
    const double *Pt;               // [2s]: P_d (the near field is FP64 in every form)
    const double *Qt;               // [n_pad + 2s]: Q_S
    T *w;                           // [tiles][NT][2][64][4]
    int64_t tile, bx;               // this workgroup's tile of 16 transforms and its block in the tile row
};

template <typename T>
using v4_t = typename Mx<T>::v4;

template <typename T>
__device__ __forceinline__ v4_t<T> v4_zero()
{
    return v4_t<T>{0, 0, 0, 0};
}

// Tile (node, parity) of this workgroup row: 64 lanes x 4 values, contiguous.
template <typename T>
__device__ __forceinline__ T *tile_ptr(const BatArgs<T> &a, int64_t node, int sig, int lane)
{
    return a.w + ((a.tile * a.NT + node) * 2 + sig) * 256 + lane * 4;
}

// The lane's transform: item 16 tile + lane mod 16 (length 0 past the batch).
struct LaneItem {
    const double *in;
    double *out;
    int64_t n;
};

template <typename T>
__device__ __forceinline__ LaneItem lane_item(const BatArgs<T> &a, int lane)
{
    LaneItem it{nullptr, nullptr, 0};
    const int64_t item = a.tile * 16 + (lane & 15);
    if (item < a.batch) {
        it.n = a.item_n ? a.item_n[item] : a.n;
        it.in = a.item_in ? a.item_in[item] : a.in + item * a.n;
        it.out = a.item_out ? a.item_out[item] : a.out + item * a.n;
    }
    return it;
}

// Value of lane r (r uniform) of a per-lane pointer or length.
template <typename P>
__device__ __forceinline__ P *lane_ptr(P *p, int r)
{
    const uint64_t v = (uint64_t)p;
    const uint32_t lo = (uint32_t)__builtin_amdgcn_readlane((int)(uint32_t)v, r);
    const uint32_t hi = (uint32_t)__builtin_amdgcn_readlane((int)(uint32_t)(v >> 32), r);
    return (P *)(((uint64_t)hi << 32) | lo);
}
__device__ __forceinline__ int64_t lane_i64(int64_t x, int r)
{
    const uint32_t lo = (uint32_t)__builtin_amdgcn_readlane((int)(uint32_t)(uint64_t)x, r);
    const uint32_t hi = (uint32_t)__builtin_amdgcn_readlane((int)(uint32_t)((uint64_t)x >> 32), r);
    return (int64_t)(((uint64_t)hi << 32) | lo);
}

// Transform r (uniform) of the tile: its input row, output row and length, read from
// lane r (lane r holds transform r).
__device__ __forceinline__ const double *row_in(const LaneItem &it, int r) { return lane_ptr(it.in, r); }
__device__ __forceinline__ double *row_out(const LaneItem &it, int r) { return lane_ptr(it.out, r); }
__device__ __forceinline__ int64_t row_n(const LaneItem &it, int r) { return lane_i64(it.n, r); }

// A transform's row as a raw buffer resource of n values: the hardware range check returns
// zero for loads past the end and drops stores past it (rows hold at most 2^28 values).
typedef unsigned int u32x2 __attribute__((ext_vector_type(2)));
constexpr unsigned kBufOut = 0xFFFFFFF0u;    // byte offset outside every row
__device__ __forceinline__ __amdgpu_buffer_rsrc_t row_rsrc(const double *p, int64_t n)
{
    return __builtin_amdgcn_make_buffer_rsrc((void *)p, (short)0, (int)(n * 8), 0x00020000);
}

// One node of input for the 16 transforms of the tile, row-coalesced: instruction r reads
// the node's 2s consecutive values of transform r (lane e: f[2 s t + e]), whole cache
// lines per instruction.  Zero past a transform's length and for lanes e >= 2s.
__device__ __forceinline__ void node_load(const LaneItem &it, int64_t t, int s, int lane, double (&x)[16])
{
    const unsigned off = lane < 2 * s ? (unsigned)(2 * s * t + lane) * 8u : kBufOut;
#pragma unroll
    for (int r = 0; r < 16; ++r) {
        const u32x2 v = __builtin_amdgcn_raw_buffer_load_b64(row_rsrc(row_in(it, r), row_n(it, r)), off, 0, 0);
        x[r] = __builtin_bit_cast(double, v);
    }
}

// Stage a loaded node into LDS for parity sg: row r (transform), column m = e / 2 for the
// lanes e of that parity; stage (0) applied (u = c .* f for cheb2leg, u_0 = 2 f_0), and
// g_j = j u_j for the near field (times_j).  Row stride kBatRow.
constexpr int kBatRow = 33;
template <typename T>
__device__ __forceinline__ void node_stage(T *slot, const double (&x)[16], int64_t t, int s, int lane, int sg, int dir,
                                           bool times_j)
{
    if ((lane & 1) == sg && lane < 2 * s) {
        const int64_t j = 2 * s * t + lane;
        double sc = 1.0;
        if (dir == 1) {
            if (j == 0) sc = 2.0;
            if (times_j) sc *= (double)(uint32_t)j;   // j < n <= 2^31 wherever x is nonzero
        }
#pragma unroll
        for (int r = 0; r < 16; ++r) slot[r * kBatRow + (lane >> 1)] = (T)(x[r] * sc);
    }
    __builtin_amdgcn_fence(__ATOMIC_ACQ_REL, "wavefront");
}

// ------------------------------------------------------------------------------------
// Forms.  FM = 0: FP32 products, four 16 x 16 x 4 instructions per tile product.
// FM = 1 (BF16 hi+lo): every FP32 operand x is split as hi = bf16(x), lo = bf16(x - hi),
// and a product of A and B is ah bh + ah bl + al bh (the al bl term, ~2^-16 relative, is
// dropped): three 16 x 16 x 16 BF16 instructions with FP32 accumulation.  The BF16
// instruction takes K = 4q + j (j = 0..3) from lane group q, the same rows the FP32 form
// takes in its steps kk = j, so both forms use the same per-lane values.
// FM = 2 (FP16 hi+lo): the same three products with FP16 operands, which keep 22 bits
// (about 2^-22 relative per product) but span only 2^-24 .. 2^16.  So every operand is
// scaled by a power of two before it is split: the A operands of the plan's Ahat per
// submatrix (the table spans about 16 decades; the factor that undoes the scaling is
// stored beside it), the other A operands (T, B(0), B(1), of magnitude <= 1) not at all,
// and every B operand per column, i.e. per transform, from the largest magnitude in that
// column (a reduction over the column's four lanes), so that transforms of any scale
// share a tile.  A product is then (A' B') / (s_A s_B), scaled back
// in FP32 before it joins the accumulator.
// FM = 3 (the FP64 tile form): FP64 products and accumulation, four 16 x 16 x 4 FP64
// instructions per tile product; tables and workspace in FP64.
typedef __bf16 bf16x4 __attribute__((ext_vector_type(4)));
typedef _Float16 f16x4 __attribute__((ext_vector_type(4)));
template <int FM>
using form_t = typename std::conditional<FM == 3, double, float>::type;
template <int FM>
struct Aop;
template <>
struct Aop<3> {
    double v[4];
};
template <>
struct Aop<0> {
    float v[4];
};
template <>
struct Aop<1> {
    bf16x4 hi, lo;
};
template <>
struct Aop<2> {
    f16x4 hi, lo;
    float inv;   // the operand is (hi + lo) inv
};

__device__ __forceinline__ void split_f16(const float (&x)[4], float sc, f16x4 &hi, f16x4 &lo)
{
#pragma unroll
    for (int j = 0; j < 4; ++j) {
        const float v = x[j] * sc;
        hi[j] = (_Float16)v;
        lo[j] = (_Float16)(v - (float)hi[j]);
    }
}

__device__ __forceinline__ void split_bf16(const float (&x)[4], bf16x4 &hi, bf16x4 &lo)
{
#pragma unroll
    for (int j = 0; j < 4; ++j) {
        hi[j] = (__bf16)x[j];
        lo[j] = (__bf16)(x[j] - (float)hi[j]);
    }
}

template <int FM>
__device__ __forceinline__ Aop<FM> aop(const form_t<FM> (&x)[4])
{
    Aop<FM> r;
    if constexpr (FM == 0 || FM == 3) {
#pragma unroll
        for (int j = 0; j < 4; ++j) r.v[j] = x[j];
    } else if constexpr (FM == 1) {
        split_bf16(x, r.hi, r.lo);
    } else {
        split_f16(x, 1.0f, r.hi, r.lo);
        r.inv = 1.0f;
    }
    return r;
}

// The 16 bytes of a packed table entry: four FP32 values, or four hi then four lo BF16 values.
// (FP16X2: four hi then four lo FP16 values of the scaled submatrix; inv undoes the scaling.)
template <int FM>
__device__ __forceinline__ Aop<FM> aop_raw(const v4_t<form_t<FM>> &raw, float inv = 1.0f)
{
    Aop<FM> r;
    if constexpr (FM == 0 || FM == 3) {
#pragma unroll
        for (int j = 0; j < 4; ++j) r.v[j] = raw[j];
    } else {
        typedef unsigned int u4 __attribute__((ext_vector_type(4)));
        typedef unsigned int u2 __attribute__((ext_vector_type(2)));
        const u4 b = __builtin_bit_cast(u4, raw);
        if constexpr (FM == 1) {
            r.hi = __builtin_bit_cast(bf16x4, u2{b[0], b[1]});
            r.lo = __builtin_bit_cast(bf16x4, u2{b[2], b[3]});
        } else {
            r.hi = __builtin_bit_cast(f16x4, u2{b[0], b[1]});
            r.lo = __builtin_bit_cast(f16x4, u2{b[2], b[3]});
            r.inv = inv;
        }
    }
    return r;
}

// a1 if c else a0, by value (a runtime index into an array of operands would go to the stack)
template <int FM>
__device__ __forceinline__ Aop<FM> pick(const Aop<FM> &a0, const Aop<FM> &a1, bool c)
{
    Aop<FM> r;
    if constexpr (FM == 0 || FM == 3) {
#pragma unroll
        for (int j = 0; j < 4; ++j) r.v[j] = c ? a1.v[j] : a0.v[j];
    } else {
        r.hi = c ? a1.hi : a0.hi;
        r.lo = c ? a1.lo : a0.lo;
        if constexpr (FM == 2) r.inv = c ? a1.inv : a0.inv;
    }
    return r;
}

// acc += A B for one tile, B given as the lane's four values (rows row(q, j) of its column).
template <int FM>
__device__ __forceinline__ v4_t<form_t<FM>> mac(v4_t<form_t<FM>> acc, const Aop<FM> &a, const form_t<FM> (&b)[4])
{
    if constexpr (FM == 0 || FM == 3) {
#pragma unroll
        for (int j = 0; j < 4; ++j) acc = Mx<form_t<FM>>::mma(a.v[j], b[j], acc);
    } else if constexpr (FM == 1) {
        bf16x4 bh, bl;
        split_bf16(b, bh, bl);
        acc = __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(a.hi, bh, acc, 0, 0, 0);
        acc = __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(a.hi, bl, acc, 0, 0, 0);
        acc = __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(a.lo, bh, acc, 0, 0, 0);
    } else {
        // the column (transform l mod 16) scaled so that its largest magnitude lies in
        // [2^13, 2^14): the four lanes l, l + 16, l + 32, l + 48 hold it
        float m = fmaxf(fmaxf(fabsf(b[0]), fabsf(b[1])), fmaxf(fabsf(b[2]), fabsf(b[3])));
        m = fmaxf(m, __shfl_xor(m, 16));
        m = fmaxf(m, __shfl_xor(m, 32));
        int e = 0;
        (void)frexpf(m, &e);                          // m = f 2^e, f in [1/2, 1)
        const int sh = m > 0.0f ? min(14 - e, 100) : 0;
        f16x4 bh, bl;
        split_f16(b, ldexpf(1.0f, sh), bh, bl);
        v4_t<float> p = {0.0f, 0.0f, 0.0f, 0.0f};
        p = __builtin_amdgcn_mfma_f32_16x16x16f16(a.hi, bh, p, 0, 0, 0);
        p = __builtin_amdgcn_mfma_f32_16x16x16f16(a.hi, bl, p, 0, 0, 0);
        p = __builtin_amdgcn_mfma_f32_16x16x16f16(a.lo, bh, p, 0, 0, 0);
        const float inv = ldexpf(a.inv, -sh);
#pragma unroll
        for (int j = 0; j < 4; ++j) acc[j] = fmaf(p[j], inv, acc[j]);
    }
    return acc;
}
template <int FM>
__device__ __forceinline__ v4_t<form_t<FM>> mac_tile(v4_t<form_t<FM>> acc, const Aop<FM> &a,
                                                     const v4_t<form_t<FM>> &x)
{
    const form_t<FM> b[4] = {x[0], x[1], x[2], x[3]};
    return mac<FM>(acc, a, b);
}

// ------------------------------------------------------------------------------------
// Upward pass of one parity over 2^K leaves starting at t0 (level gleaf): leaf tiles from
// step (1) (LEAF_STEP1) or from the workspace; the loads of leaf i + 1 are issued before
// the products of leaf i.
template <typename T, int K, bool LEAF_STEP1, int FM>
__device__ __forceinline__ void up_walk(const BatArgs<T> &a, int64_t t0, int gleaf, int sg, int lane, T *slot)
{
    const int li = lane & 15, q = lane >> 4;
    const int M = a.M, s = a.s;
    // A operands of the parent transfer: B(0) and B(1) (modal: B(0) with odd diagonals
    // negated; nodal: its own table)
    Aop<FM> b0a, b1a;
    {
        T v0[4], v1[4];
#pragma unroll
        for (int kk = 0; kk < 4; ++kk) {
            const int k = Mx<T>::row(q, kk);
            const bool ok = li < M && k < M;
            const T v = ok ? a.B0[li * M + k] : T(0);
            v0[kk] = v;
            v1[kk] = a.B1 ? (ok ? a.B1[li * M + k] : T(0)) : (((li - k) & 1) ? -v : v);
        }
        b0a = aop<FM>(v0);
        b1a = aop<FM>(v1);
    }
    // A operands of step (1): T(sigma)^T, column m = 16 c + 4 q + kk
    Aop<FM> ta[2];
#pragma unroll
    for (int c = 0; c < 2; ++c) {
        T v[4];
#pragma unroll
        for (int kk = 0; kk < 4; ++kk) {
            const int m = 16 * c + 4 * q + kk;
            v[kk] = (LEAF_STEP1 && li < M && m < s) ? a.Tm[(sg * s + m) * M + li] : T(0);
        }
        ta[c] = aop<FM>(v);
    }
    LaneItem it{nullptr, nullptr, 0};
    if (LEAF_STEP1) it = lane_item(a, lane);
    const int nch = s > 16 ? 2 : 1;

    // leaf inputs: step (1) reads u[2 s t + 2 m + sigma], m = 16 c + 4 q + kk, from the
    // wave's LDS slot [transform][m]; the next leaf's loads are in flight meanwhile
    double xn[16];
    v4_t<T> wn = v4_zero<T>();
    auto issue = [&](int64_t t) {
        if (LEAF_STEP1) node_load(it, t, s, lane, xn);
        else wn = *reinterpret_cast<const v4_t<T> *>(tile_ptr(a, node_offset(gleaf) + t, sg, lane));
    };
    issue(t0);
    if (LEAF_STEP1) node_stage<T>(slot, xn, t0, s, lane, sg, a.dir, false);
    v4_t<T> stk[K > 0 ? K : 1];
    for (int i = 0; i < (1 << K); ++i) {
        const int64_t t = t0 + i;
        v4_t<T> cur;
        if (LEAF_STEP1) {
            T y[2][4];
#pragma unroll
            for (int c = 0; c < 2; ++c)
#pragma unroll
                for (int kk = 0; kk < 4; ++kk) y[c][kk] = slot[li * kBatRow + (16 * c + 4 * q + kk)];
            if (i + 1 < (1 << K)) issue(t + 1);
            // step (1): w_k(t, sigma) = sum_m T_k(X_m^sigma) u[2 s t + 2 m + sigma]
            cur = v4_zero<T>();
#pragma unroll
            for (int c = 0; c < 2; ++c) {
                if (c < nch) {
                    T b[4];
#pragma unroll
                    for (int kk = 0; kk < 4; ++kk) b[kk] = 16 * c + 4 * q + kk < s ? y[c][kk] : T(0);
                    cur = mac<FM>(cur, ta[c], b);
                }
            }
            *reinterpret_cast<v4_t<T> *>(tile_ptr(a, node_offset(gleaf) + t, sg, lane)) = cur;
            if (i + 1 < (1 << K)) node_stage<T>(slot, xn, t + 1, s, lane, sg, a.dir, false);
        } else {
            cur = wn;
            if (i + 1 < (1 << K)) issue(t + 1);
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
                    cur = mac_tile<FM>(mac_tile<FM>(v4_zero<T>(), b0a, stk[d - 1]), b1a, cur);
                    *reinterpret_cast<v4_t<T> *>(tile_ptr(a, node_offset(gleaf - d) + (t >> d), sg, lane)) = cur;
                }
            }
        }
    }
}

// Waves of a workgroup: wave w takes subtree 2 bx + w / 2 and parity w mod 2.
template <typename T, int KU, int FM>
__device__ __forceinline__ void up_body(const BatArgs<T> &a)
{
    __shared__ T slots[4][16 * kBatRow];
    const int lane = threadIdx.x & 63, wv = wave_id();
    const int64_t sub = a.bx * 2 + (wv >> 1);
    const int64_t P = int64_t(1) << (a.L + 1);   // finest nodes
    if ((sub << KU) >= P) return;
    up_walk<T, KU, true, FM>(a, sub << KU, a.L - 1, wv & 1, lane, slots[wv]);
}

template <typename T, int KT, int FM>
__device__ __forceinline__ void top_body(const BatArgs<T> &a)
{
    const int lane = threadIdx.x & 63, wv = wave_id();
    const int64_t sub = a.bx * 2 + (wv >> 1);
    if ((sub << KT) >= (int64_t(1) << (a.gin + 2))) return;
    up_walk<T, KT, false, FM>(a, sub << KT, a.gin, wv & 1, lane, nullptr);
}

// ------------------------------------------------------------------------------------
// Far field of one row node v of level g and one parity (step (3), Eq. (cfrompq)):
// block b = v >> 1, c(2b) = Ahat(0) w(2b+2) + Ahat(1) w(2b+3), c(2b+1) = Ahat(2) w(2b+3);
// zero when the block lies past the last one of the level (b >= b_g = 2^(g+1) - 1).
// far_issue loads the operands and far_do multiplies, so loads can run ahead.
template <typename T>
struct FarIn {
    v4_t<T> A0, A1, W2, W3;
    float i0, i1;                   // FP16X2: the factors that undo the scaling of A0, A1
    int kind;                       // 0: no block, 1: even row node, 2: odd row node
};

template <typename T>
__device__ __forceinline__ FarIn<T> far_issue(const BatArgs<T> &a, int g, int64_t v, int sg, int lane)
{
    FarIn<T> f;
    f.kind = 0;
    f.A0 = f.A1 = f.W2 = f.W3 = v4_zero<T>();
    f.i0 = f.i1 = 1.0f;
    const int64_t b = v >> 1;
    if (b >= (int64_t(1) << (g + 1)) - 1) return f;
    const T *ab = a.ahat + ((level_block_offset(g) + b) * 3 * 64 + lane) * 4;
    const int64_t cn = node_offset(g) + v + 2;
    if (a.ahat_inv) {
        const float *iv = a.ahat_inv + (level_block_offset(g) + b) * 3;
        f.i0 = (v & 1) == 0 ? iv[0] : iv[2];
        f.i1 = iv[1];
    }
    if ((v & 1) == 0) {
        f.kind = 1;
        f.A0 = *reinterpret_cast<const v4_t<T> *>(ab);
        f.A1 = *reinterpret_cast<const v4_t<T> *>(ab + 64 * 4);
        f.W2 = *reinterpret_cast<const v4_t<T> *>(tile_ptr(a, cn, sg, lane));
        f.W3 = *reinterpret_cast<const v4_t<T> *>(tile_ptr(a, cn + 1, sg, lane));
    } else {
        f.kind = 2;
        f.A0 = *reinterpret_cast<const v4_t<T> *>(ab + 2 * 64 * 4);
        f.W2 = *reinterpret_cast<const v4_t<T> *>(tile_ptr(a, cn, sg, lane));
    }
    return f;
}

template <int FM, typename T>
__device__ __forceinline__ v4_t<T> far_do(const FarIn<T> &f)
{
    v4_t<T> r = v4_zero<T>();
    if (f.kind == 0) return r;
    r = mac_tile<FM>(r, aop_raw<FM>(f.A0, f.i0), f.W2);
    if (f.kind == 1) r = mac_tile<FM>(r, aop_raw<FM>(f.A1, f.i1), f.W3);
    return r;
}

// The same for the two parity waves of a subtree sharing one staged node: wave h loads rows
// 8h .. 8h + 7 and stages both parities, slot[sigma][row][m] (parity stride SL).
__device__ __forceinline__ void node_load8(const LaneItem &it, int64_t t, int s, int lane, int h, double (&x)[8])
{
    const unsigned off = lane < 2 * s ? (unsigned)(2 * s * t + lane) * 8u : kBufOut;
#pragma unroll
    for (int r = 0; r < 8; ++r) {
        const u32x2 v =
            __builtin_amdgcn_raw_buffer_load_b64(row_rsrc(row_in(it, 8 * h + r), row_n(it, 8 * h + r)), off, 0, 0);
        x[r] = __builtin_bit_cast(double, v);
    }
}
template <typename T>
__device__ __forceinline__ void node_stage8(T *slot, int SL, const double (&x)[8], int64_t t, int s, int lane, int h,
                                            int dir, bool times_j)
{
    if (lane < 2 * s) {
        const int64_t j = 2 * s * t + lane;
        double sc = 1.0;
        if (dir == 1) {
            if (j == 0) sc = 2.0;
            if (times_j) sc *= (double)(uint32_t)j;   // j < n <= 2^28 wherever x is nonzero
        }
        T *dst = slot + (lane & 1) * SL + 8 * h * kBatRow + (lane >> 1);
#pragma unroll
        for (int r = 0; r < 8; ++r) dst[r * kBatRow] = (T)(x[r] * sc);
    }
}

// Steps (3)-(7) for one level-groot subtree of 2^KD finest row nodes and one parity.
// NC = ceil(2s / 16) column chunks of the near-field band; rows need two 16-row tiles
// when s > 16 (NC > 2).  LDS per wave: the far-field tiles of the own nodes above the
// finest depth (node idx of depth d at slot 2^d - 2 + idx) and the Q window of the finest
// nodes; per subtree (shared by its two parity waves, two workgroup barriers per leaf):
// two input nodes [parity][transform][m] (row-coalesced loads, the next node in flight)
// and the output rows of the current node [transform][2s].  The grid holds an even number
// of subtrees, so every wave of a workgroup has a subtree and reaches every barrier.
template <typename T, int KD, int NC, int FM>
__device__ __forceinline__ void main_body(const BatArgs<T> &a)
{
    constexpr int nc = NC, nrt = NC > 2 ? 2 : 1;
    constexpr int INNER = (1 << KD) - 2;             // own nodes of depths 1..KD-1
    constexpr int QW = 64 * (1 << KD) + 32;          // Q window: 2s 2^KD + s, s <= 32
    constexpr int SL = 16 * kBatRow;                 // one staged node
    __shared__ v4_t<T> Fl[4][INNER > 0 ? INNER : 1][64];
    __shared__ double Ql[4][QW];
    constexpr int OBS = 65;                          // output row stride (2s <= 64)
    __shared__ double Sl[2][4 * SL + 16 * OBS];      // per subtree: input nodes u, u + 1; output rows
    L2C_TS(1, 0);
    const int lane = threadIdx.x & 63, wv = wave_id();
    const int li = lane & 15, q = lane >> 4, sg = wv & 1;
    const int s = a.s, M = a.M, dir = a.dir;
    const int groot = a.L - 1 - KD;
    const int64_t Rn = a.bx * 2 + (wv >> 1);   // < 2^(groot+2): the grid is exact
    const int64_t u0 = Rn << KD;                      // first finest row node
    const LaneItem it = lane_item(a, lane);
    // a workgroup whose rows all lie past every transform of its tile writes nothing and
    // ends before any barrier (ragged batches order each group longest first, so tiles of
    // short transforms skip the end of the group's padded length)
    {
        double nm = (double)it.n;
#pragma unroll
        for (int m = 8; m >= 1; m >>= 1) nm = fmax(nm, __shfl_xor(nm, m, 16));
        if ((double)(2 * (int64_t)s * ((a.bx * 2) << KD)) >= nm) return;
    }
    double *Qw = Ql[wv];
    double *in_sl = Sl[wv >> 1], *ob = Sl[wv >> 1] + 4 * SL;

    // Every load of the prologue is issued before the first one is waited for.
    // The first two input nodes (this wave: rows 8 sg .. 8 sg + 7).
    double xn[8], xn1[8];
    node_load8(it, u0, s, lane, sg, xn);
    node_load8(it, u0 + 1, s, lane, sg, xn1);
    // Q_S for S = 2 s u0 + [0, 2 s 2^KD + s); the rest of the window is zero, so every
    // read of the leaf loop below is of initialized memory
    constexpr int QR = QW / 64 + 1;
    double qreg[QR];
    {
        const int qn = 2 * s * (1 << KD) + s;
#pragma unroll
        for (int k = 0; k < QR; ++k) {
            const int e = lane + 64 * k;
            qreg[k] = e < qn ? a.Qt[2 * s * u0 + (e < qn ? e : 0)] : 0.0;
        }
    }
    // A operands: B(p)^T (step (4)) and T(sigma) (Eq. (step5))
    T btv[2][4], tev[2][4];
#pragma unroll
    for (int kk = 0; kk < 4; ++kk) {
        const int k = Mx<T>::row(q, kk);
        const bool ok = li < M && k < M;
        const T v = a.B0[ok ? k * M + li : 0];
        btv[0][kk] = ok ? v : T(0);
        btv[1][kk] = a.B1 ? (ok ? a.B1[k * M + li] : T(0)) : (((k - li) & 1) ? -btv[0][kk] : btv[0][kk]);
    }
#pragma unroll
    for (int rt = 0; rt < 2; ++rt)
#pragma unroll
        for (int kk = 0; kk < 4; ++kk) {
            const int m = 16 * rt + li, k = Mx<T>::row(q, kk);
            const bool ok = m < s && k < M;
            const T v = a.Tm[ok ? (sg * s + m) * M + k : 0];
            tev[rt][kk] = ok ? v : T(0);
        }
    // near-field factor P_{m'-m} of row m = 16 rt + l mod 16 and column m' = 16 c + 4 q + kk,
    // zero outside the band m <= m' < 2s: read per leaf from an LDS copy of P with 32
    // leading zeros (d < 0) instead of 32 FP64 values per lane; entries with m' >= 2s or
    // m >= s meet zero operands or unused rows there.
    __shared__ double Pband[96];
    for (int e = threadIdx.x; e < 96; e += blockDim.x) {
        const int d = e - 32;
        Pband[e] = (d >= 0 && d < 2 * s) ? a.Pt[d >= 0 && d < 2 * s ? d : 0] : 0.0;
    }
    auto pband = [&](int rt, int c, int kk) -> double { return Pband[16 * c + 4 * q + kk - 16 * rt - li + 32]; };
    const Aop<FM> bt0 = aop<FM>(btv[0]), bt1 = aop<FM>(btv[1]);
    const Aop<FM> te[2] = {aop<FM>(tev[0]), aop<FM>(tev[1])};
    // the first two ancestor levels' far-field operands
    FarIn<T> n1 = far_issue(a, 0, Rn >> groot, sg, lane);
    FarIn<T> n2 = groot >= 1 ? far_issue(a, 1, Rn >> (groot - 1), sg, lane) : n1;
    // now the LDS stores of the Q window and the first input node
#pragma unroll
    for (int k = 0; k < QR; ++k) {
        const int e = lane + 64 * k;
        if (e < QW) Qw[e] = qreg[k];
    }
    node_stage8<double>(in_sl, SL, xn, u0, s, lane, sg, dir, true);

    // ancestors a_g = Rn >> (groot - g): c(a_0) = far; c(a_g) = far + B(p)^T c(a_{g-1});
    // the operands of levels g + 1 and g + 2 are in flight while level g is multiplied
    v4_t<T> cp = v4_zero<T>();
    for (int g = 0; g <= groot; ++g) {
        const FarIn<T> cu = n1;
        n1 = n2;
        if (g + 2 <= groot) n2 = far_issue(a, g + 2, Rn >> (groot - g - 2), sg, lane);
        v4_t<T> cv = far_do<FM>(cu);
        if (g > 0) cv = mac_tile<FM>(cv, pick<FM>(bt0, bt1, (Rn >> (groot - g)) & 1), cp);
        cp = cv;
    }
    node_stage8<double>(in_sl + 2 * SL, SL, xn1, u0 + 1, s, lane, sg, dir, true);
    L2C_TS(1, 1);
    // far field of the own nodes above the finest depth (depth-major), pipelined, into LDS
    if (INNER > 0) {
        auto own_node = [&](int j, int &d, int64_t &v) {
            d = 31 - __builtin_clz(j + 2);
            v = (Rn << d) + (j + 2 - (1 << d));
        };
        int d0;
        int64_t v0;
        own_node(0, d0, v0);
        FarIn<T> nx = far_issue(a, groot + d0, v0, sg, lane);
        for (int j = 0; j < INNER; ++j) {
            const FarIn<T> cu = nx;
            if (j + 1 < INNER) {
                int d1;
                int64_t v1;
                own_node(j + 1, d1, v1);
                nx = far_issue(a, groot + d1, v1, sg, lane);
            }
            Fl[wv][j][lane] = far_do<FM>(cu);
        }
    }
    // LDS writes (far tiles, Q window, staged input of both parity waves) complete
    __syncthreads();
    L2C_TS(1, 2);

    // depth-first walk: stk[d] = c of the current node at depth d; then steps (5)-(7).
    // The finest node's far-field operands and the input node u + 2 are loaded one leaf ahead.
    v4_t<T> stk[KD + 1];
    stk[0] = cp;
    FarIn<T> fnx = far_issue(a, groot + KD, u0, sg, lane);
    for (int i = 0; i < (1 << KD); ++i) {
        const int64_t u = u0 + i;
        const int64_t base = 2 * s * u;
        const FarIn<T> fcu = fnx;
        // B operands: g at m' = 16 c + 4 q + kk (node u for m' < s, node u + 1 after)
        double y[4][4];
        {
            const double *n0 = in_sl + (i & 1) * 2 * SL + sg * SL + li * kBatRow;
            const double *n1 = in_sl + ((i + 1) & 1) * 2 * SL + sg * SL + li * kBatRow;
#pragma unroll
            for (int c = 0; c < 4; ++c)
#pragma unroll
                for (int kk = 0; kk < 4; ++kk) {
                    const int mp = 16 * c + 4 * q + kk;
                    const double *src = mp < s ? n0 + mp : n1 + (mp < 2 * s ? mp - s : 0);
                    const double v = *src;
                    y[c][kk] = (c < nc && mp < 2 * s) ? v : 0.0;
                }
        }
        if (i + 1 < (1 << KD)) {
            fnx = far_issue(a, groot + KD, u + 1, sg, lane);
            node_load8(it, u + 2, s, lane, sg, xn);
        }
#pragma unroll
        for (int d = 1; d < KD; ++d) {
            const int dmin = i == 0 ? 1 : KD - __builtin_ctz(i);
            if (d >= dmin) {
                const int idx = i >> (KD - d);
                stk[d] = mac_tile<FM>(Fl[wv][(1 << d) - 2 + idx][lane], pick<FM>(bt0, bt1, idx & 1), stk[d - 1]);
            }
        }
        v4_t<T> cu = far_do<FM>(fcu);
        if (KD > 0) cu = mac_tile<FM>(cu, pick<FM>(bt0, bt1, i & 1), stk[KD > 0 ? KD - 1 : 0]);
        else cu = stk[0];
        v4_t<T> acc[2] = {v4_zero<T>(), v4_zero<T>()};
        // far part (Eq. (step5)): rows m = 16 rt + l mod 16 of T(sigma).  The last two row
        // nodes (u >= P - 2) have no far-field block on any level, so their c is zero.
#pragma unroll
        for (int rt = 0; rt < 2; ++rt)
            if (rt < nrt) acc[rt] = mac_tile<FM>(acc[rt], te[rt], cu);
        // near field (step (6)), in FP64 in every form (products and sums on the FP64 matrix
        // cores): row m, column m' = 16 c + 4 q + kk:
        //   rs_i P_{m'-m} Q_{2 s u + sigma + m + m'} (m <= m' < 2s) times g_{2 s u + 2 m' + sigma}
        // Q enters through m + m' = 16 (c + rt) + 4 q + kk + l mod 16: 20 values per leaf
        const double *Qu = Qw + 2 * s * i + sg + 4 * q + li;
        double qv[5][4];
#pragma unroll
        for (int cr = 0; cr < 5; ++cr)
#pragma unroll
            for (int kk = 0; kk < 4; ++kk) qv[cr][kk] = Qu[16 * cr + kk];
        // the FP64 form adds the band to the far part's accumulator; the others keep it apart
        // (FP64 accumulator, rows row(q, r) of the FP64 layout) and add the two in FP64 below
        v4_t<double> an[2];
#pragma unroll
        for (int rt = 0; rt < 2; ++rt) {
            if constexpr (FM == 3) an[rt] = acc[rt];
            else an[rt] = v4_zero<double>();
        }
#pragma unroll
        for (int rt = 0; rt < 2; ++rt) {
            if (rt < nrt) {
                // rs_i = 2i + 1 (cheb2leg)
                const int64_t ir = base + 2 * (16 * rt + li) + sg;
                const double rs = dir == 1 ? (double)(2 * ir + 1) : 1.0;
#pragma unroll
                for (int c = 0; c < 4; ++c) {
                    if (c < nc && c >= rt) {
#pragma unroll
                        for (int kk = 0; kk < 4; ++kk)
                            an[rt] = Mx<double>::mma(pband(rt, c, kk) * (qv[c + rt][kk] * rs), y[c][kk], an[rt]);
                    }
                }
            }
        }
        // output rows of this parity through LDS: lane holds rows m = 16 rt + row(q, r) of
        // transform l mod 16; stored two transforms per instruction, lane -> row
        if constexpr (FM != 3) {
#pragma unroll
            for (int rt = 0; rt < 2; ++rt)
                if (rt < nrt) {
#pragma unroll
                    for (int r = 0; r < 4; ++r)
                        ob[li * OBS + 2 * (16 * rt + Mx<float>::row(q, r)) + sg] = (double)acc[rt][r];
                }
            __builtin_amdgcn_fence(__ATOMIC_ACQ_REL, "wavefront");   // other lanes add to these rows
        }
#pragma unroll
        for (int rt = 0; rt < 2; ++rt)
            if (rt < nrt) {
#pragma unroll
                for (int r = 0; r < 4; ++r) {
                    double *o = ob + li * OBS + 2 * (16 * rt + Mx<double>::row(q, r)) + sg;
                    if constexpr (FM == 3) *o = an[rt][r];
                    else *o += an[rt][r];
                }
            }
        __syncthreads();
        {
            // wave sg stores rows 8 sg .. 8 sg + 7 of the node, lane e -> output 2 s u + e
            const int64_t iz = base + lane;
            const unsigned off = lane < 2 * s ? (unsigned)iz * 8u : kBufOut;
            const double sc = dir == 0 ? (iz == 0 ? 1.0 / kPi : 2.0 / kPi) : 1.0;
#pragma unroll
            for (int r = 0; r < 8; ++r) {
                const int tr = 8 * sg + r;
                const int64_t nr = row_n(it, tr);
                double v = ob[tr * OBS + (lane < 2 * s ? lane : 0)] * sc;
                if (dir == 1 && base == 0 && nr > 0) {
                    const double f0 = row_in(it, tr)[0];
                    if (iz == 0) v += f0;   // K_00 u_0 = u_0 / 2 = f_0
                }
                __builtin_amdgcn_raw_buffer_store_b64(__builtin_bit_cast(u32x2, v), row_rsrc(row_out(it, tr), nr), off, 0, 0);
            }
        }
        // the next leaf's second node replaces node u (read above by both parity waves)
        if (i + 1 < (1 << KD)) {
            node_stage8<double>(in_sl + (i & 1) * 2 * SL, SL, xn, u + 2, s, lane, sg, dir, true);
            __syncthreads();
        }
        if (i == 0) L2C_TS(1, 3);
    }
    L2C_TS(1, 4);
}

// ------------------------------------------------------------------------------------
// Launches.  Plain: one group, blockIdx.y = tile, blockIdx.x = block in the tile row.
// Grouped: one launch for many groups of a ragged batch that share the kernel's template
// shape; blocks [blk0[g], blk0[g+1]) belong to entry g, gx blocks per tile.
template <typename T>
struct BatEntry {
    BatArgs<T> a;
    int64_t gx;
};

template <typename T>
__device__ __forceinline__ BatArgs<T> plain_args(BatArgs<T> a)
{
    a.tile = blockIdx.y;
    a.bx = blockIdx.x;
    return a;
}

template <typename T>
__device__ __forceinline__ BatArgs<T> entry_args(const BatEntry<T> *E, const int64_t *blk0, int n)
{
    const int64_t b = blockIdx.x;
    int lo = 0, hi = n - 1;                      // last entry g with blk0[g] <= b
    while (lo < hi) {
        const int mid = (lo + hi + 1) >> 1;
        if (blk0[mid] <= b) lo = mid;
        else hi = mid - 1;
    }
    BatArgs<T> a = E[lo].a;
    const int64_t loc = b - blk0[lo];
    a.tile = loc / E[lo].gx;
    a.bx = loc - a.tile * E[lo].gx;
    return a;
}

template <typename T, int KU, int FM>
__global__ __launch_bounds__(256) void kb_up(BatArgs<T> a) { up_body<T, KU, FM>(plain_args(a)); }
template <typename T, int KT, int FM>
__global__ __launch_bounds__(256) void kb_top(BatArgs<T> a) { top_body<T, KT, FM>(plain_args(a)); }
template <typename T, int KD, int NC, int FM>
__global__ __launch_bounds__(256) void kb_main(BatArgs<T> a) { main_body<T, KD, NC, FM>(plain_args(a)); }

template <typename T, int KU, int FM>
__global__ __launch_bounds__(256) void kbg_up(const BatEntry<T> *E, const int64_t *blk0, int n)
{
    up_body<T, KU, FM>(entry_args(E, blk0, n));
}
template <typename T, int KT, int FM>
__global__ __launch_bounds__(256) void kbg_top(const BatEntry<T> *E, const int64_t *blk0, int n)
{
    top_body<T, KT, FM>(entry_args(E, blk0, n));
}
template <typename T, int KD, int NC, int FM>
__global__ __launch_bounds__(256) void kbg_main(const BatEntry<T> *E, const int64_t *blk0, int n)
{
    main_body<T, KD, NC, FM>(entry_args(E, blk0, n));
}

// ------------------------------------------------------------------------------------
// Plan-time helpers: Ahat (FP64 plan tables) -> A-operand order of the form's type;
// Q_S for S < len.
// Ahat entry (k, l) of submatrix r of level-major block b (zero outside M x M).
template <int M>
__device__ __forceinline__ double ahat_entry(const double *top, const double *bot, const Geometry &G, int64_t b, int r,
                                             int k, int l)
{
    if (k >= M || l >= M) return 0.0;
    int g = 0;
    while (b >= (int64_t(1) << (g + 1)) - 1) {
        b -= (int64_t(1) << (g + 1)) - 1;
        ++g;
    }
    if (g <= G.groot) return top[((level_block_offset(g) + b) * 3 + r) * M * M + k * M + l];
    constexpr int NCH = 3 * M / 2;
    const int d = g - G.groot;
    const int64_t Rn = b >> (d - 1);
    const int64_t j = ((int64_t(1) << G.kd) - (int64_t(1) << d)) + (b - (Rn << (d - 1)));
    const int64_t slot = j * M + k;
    const int64_t grp = Rn * G.sub_groups + slot / 64;
    const int ln = (int)(slot % 64);
    const int el = r * M + l;
    return bot[((grp * NCH + el / 2) * 64 + ln) * 2 + (el & 1)];
}

// FP16X2: per submatrix (block-major, r fastest) the power of two 2^-e that undoes its
// scaling: the scaled entries have magnitude < 2^13.
template <int M>
__global__ void kb_ahat_scale(const double *top, const double *bot, Geometry G, float *inv, int64_t nsub)
{
    const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (e >= nsub) return;
    double m = 0.0;
    for (int k = 0; k < M && k < 16; ++k)
        for (int l = 0; l < M && l < 16; ++l) m = fmax(m, fabs(ahat_entry<M>(top, bot, G, e / 3, (int)(e % 3), k, l)));
    int ex = 0;
    (void)frexp(m, &ex);                       // m = f 2^ex, f in [1/2, 1)
    inv[e] = m > 0.0 ? ldexpf(1.0f, ex - 13) : 1.0f;
}

template <int M, int FM>
__global__ void kb_pack_ahat(const double *top, const double *bot, Geometry G, void *dst, int64_t blocks,
                             const float *inv)
{
    const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;   // (blk, r, lane, kk)
    if (e >= blocks * 3 * 256) return;
    const int kk = (int)(e & 3), lane = (int)((e >> 2) & 63);
    const int64_t br = e >> 8;
    const int r = (int)(br % 3);
    const int k = lane & 15, l = FM == 3 ? Mx<double>::row(lane >> 4, kk) : Mx<float>::row(lane >> 4, kk);
    const double v = ahat_entry<M>(top, bot, G, br / 3, r, k, l);
    if (FM == 3) {
        ((double *)dst)[e] = v;
    } else if (FM == 0) {
        ((float *)dst)[e] = (float)v;
    } else if (FM == 1) {
        // 16 bytes per lane entry: four hi then four lo BF16 values
        const __bf16 hi = (__bf16)(float)v;
        const __bf16 lo = (__bf16)(float)(v - (double)(float)hi);
        unsigned short *d16 = (unsigned short *)dst + (e >> 2) * 8 + kk;
        d16[0] = __builtin_bit_cast(unsigned short, hi);
        d16[4] = __builtin_bit_cast(unsigned short, lo);
    } else {
        // four hi then four lo FP16 values of the entry scaled by 1 / inv (a power of two)
        const double vs = v / (double)inv[br];
        const _Float16 hi = (_Float16)vs;
        const _Float16 lo = (_Float16)(vs - (double)hi);
        unsigned short *d16 = (unsigned short *)dst + (e >> 2) * 8 + kk;
        d16[0] = __builtin_bit_cast(unsigned short, hi);
        d16[4] = __builtin_bit_cast(unsigned short, lo);
    }
}

__global__ void kb_q_table(double *Qt, int64_t len, int dir)
{
    const int64_t S = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (S < len) Qt[S] = near_Q(dir, S);
}

template <int M>
static hipError_t pack(const l2c_plan_s &p, void *dst, hipStream_t st)
{
    const int64_t blocks = level_block_offset(p.L);
    const int64_t total = blocks * 3 * 256;
    const dim3 grid((unsigned)((total + 255) / 256));
    if (p.precision == L2C_FP64) {
        hipLaunchKernelGGL((kb_pack_ahat<M, 3>), grid, dim3(256), 0, st, p.d_top, p.d_bot, p.geo, dst, blocks,
                           (const float *)nullptr);
    } else if (p.precision == L2C_FP16X2) {
        if (!p.d_bS) return hipErrorInvalidValue;
        hipLaunchKernelGGL((kb_ahat_scale<M>), dim3((unsigned)((blocks * 3 + 255) / 256)), dim3(256), 0, st, p.d_top,
                           p.d_bot, p.geo, p.d_bS, blocks * 3);
        hipLaunchKernelGGL((kb_pack_ahat<M, 2>), grid, dim3(256), 0, st, p.d_top, p.d_bot, p.geo, dst, blocks,
                           (const float *)p.d_bS);
    } else if (p.precision == L2C_BF16X2) {
        hipLaunchKernelGGL((kb_pack_ahat<M, 1>), grid, dim3(256), 0, st, p.d_top, p.d_bot, p.geo, dst, blocks,
                           (const float *)nullptr);
    } else {
        hipLaunchKernelGGL((kb_pack_ahat<M, 0>), grid, dim3(256), 0, st, p.d_top, p.d_bot, p.geo, dst, blocks,
                           (const float *)nullptr);
    }
    return hipGetLastError();
}

hipError_t batched_build_tables(const l2c_plan_s &p, void *ahat_dst, void *q_dst, int64_t q_len, hipStream_t st)
{
    hipError_t e;
    switch (p.M) {
    case 12: e = pack<12>(p, ahat_dst, st); break;
    case 16: e = pack<16>(p, ahat_dst, st); break;
    default: return hipErrorInvalidValue;
    }
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(kb_q_table, dim3((unsigned)((q_len + 255) / 256)), dim3(256), 0, st, (double *)q_dst, q_len,
                       p.direction);
    return hipGetLastError();
}

// ------------------------------------------------------------------------------------
template <typename T, int FM>
static hipError_t run_batched(const l2c_plan_s &p, const double *in, double *out, int64_t batch, hipStream_t st,
                              const ItemArrays *ia)
{
    const int L = p.L;
    const int ku = L - 1 < kBatUpDepth ? L - 1 : kBatUpDepth;
    const int kdmax = bat_main_depth(FM);
    const int kd = L - 1 < kdmax ? L - 1 : kdmax;
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
        a.ahat_inv = p.d_bS;
        a.Tm = (const T *)p.d_bT;
        a.B0 = (const T *)p.d_bB;
        a.B1 = p.basis == L2C_NODAL ? (const T *)p.d_bB + p.M * p.M : nullptr;
        a.Pt = (const double *)p.d_bP;
        a.Qt = (const double *)p.d_bQ;
        a.w = (T *)p.d_bw;
        {
            const unsigned gx = (unsigned)(((Pn >> ku) + 1) / 2);
            switch (ku) {
#define L2C_UP(KK) \
    case KK: hipLaunchKernelGGL((kb_up<T, KK, FM>), dim3(gx, tiles), dim3(256), 0, st, a); break;
                L2C_UP(0) L2C_UP(1) L2C_UP(2) L2C_UP(3)
#undef L2C_UP
            default: return hipErrorInvalidValue;
            }
        }
        for (int gin = L - 1 - ku; gin > 0;) {
            const int kt = gin < kBatTopDepth ? gin : kBatTopDepth;
            const int gout = gin - kt;
            a.gin = gin;
            const unsigned gx = (unsigned)((((int64_t)1 << (gout + 2)) + 1) / 2);
            switch (kt) {
#define L2C_TOP(KK) \
    case KK: hipLaunchKernelGGL((kb_top<T, KK, FM>), dim3(gx, tiles), dim3(256), 0, st, a); break;
                L2C_TOP(1) L2C_TOP(2) L2C_TOP(3)
#undef L2C_TOP
            default: return hipErrorInvalidValue;
            }
            gin = gout;
        }
        {
            const int groot = L - 1 - kd;
            const unsigned gx = (unsigned)((((int64_t)1 << (groot + 2)) + 1) / 2);
            const int nc = (2 * p.s + 15) / 16;
            const bool timed = p.ev_before && p.ev_after && b0 == 0;   // around the dominant kernel
            if (timed) (void)hipEventRecord(p.ev_before, st);
            switch (kd * 8 + nc) {
#define L2C_MAIN(KK, NN) \
    case KK * 8 + NN: hipLaunchKernelGGL((kb_main<T, KK, NN, FM>), dim3(gx, tiles), dim3(256), 0, st, a); break;
#define L2C_MAIN4(KK) L2C_MAIN(KK, 1) L2C_MAIN(KK, 2) L2C_MAIN(KK, 3) L2C_MAIN(KK, 4)
                L2C_MAIN4(0) L2C_MAIN4(1) L2C_MAIN4(2)
#undef L2C_MAIN4
#undef L2C_MAIN
            default: return hipErrorInvalidValue;
            }
            if (timed) (void)hipEventRecord(p.ev_after, st);
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
    if (p.precision == L2C_FP64) return run_batched<double, 3>(p, in, out, batch, st, ia);
    if (p.precision == L2C_FP16X2) return run_batched<float, 2>(p, in, out, batch, st, ia);
    if (p.precision == L2C_BF16X2) return run_batched<float, 1>(p, in, out, batch, st, ia);
    return run_batched<float, 0>(p, in, out, batch, st, ia);
}

}  // namespace l2c

// ------------------------------------------------------------------------------------
// Grouped launches (ragged batches).
#include "l2c_alloc.h"
#include "l2c_batched.h"
#include <map>
#include <tuple>
#include <vector>

namespace l2c {

struct BatGrouped {
    struct Launch {
        int kind;       // 0 up, 1 top, 2 main
        int k1, k2;     // KU | KT | (KD, NC)
        void *E;        // BatEntry<float>[n] (device)
        int64_t *blk0;  // [n + 1] (device)
        int n;
        int64_t blocks;
    };
    int fm = 0;
    std::vector<Launch> launches;
};

void batched_grouped_free(BatGrouped *g)
{
    if (!g) return;
    for (auto &l : g->launches) {
        dev_free(l.E);
        dev_free(l.blk0);
    }
    delete g;
}

hipError_t batched_grouped_make(const l2c_plan_s *const *plans, const ItemArrays *ia, const int64_t *items, int ngroups,
                                BatGrouped **out)
{
    typedef float T;
    *out = nullptr;
    // class key (kind, k1, k2, pass) -> entries
    std::map<std::tuple<int, int, int, int>, std::vector<BatEntry<T>>> cls;
    int fm = 0;
    for (int g = 0; g < ngroups; ++g) {
        const l2c_plan_s &p = *plans[g];
        if (p.L < 1) continue;
        if (p.s > 32 || p.M > 16) return hipErrorInvalidValue;
        fm = p.precision == L2C_FP16X2 ? 2 : p.precision == L2C_BF16X2 ? 1 : 0;
        const int64_t tiles = (items[g] + 15) / 16;
        if (tiles > p.bw_tiles) return hipErrorInvalidValue;
        const int L = p.L;
        const int ku = L - 1 < kBatUpDepth ? L - 1 : kBatUpDepth;
        const int kd = L - 1 < kBatMainDepth ? L - 1 : kBatMainDepth;
        const int64_t Pn = int64_t(1) << (L + 1);
        BatArgs<T> a{};
        a.in = nullptr;
        a.out = nullptr;
        a.n = p.n;
        a.item_n = ia[g].n;
        a.item_in = ia[g].in;
        a.item_out = ia[g].out;
        a.batch = items[g];
        a.dir = p.direction;
        a.L = L;
        a.s = p.s;
        a.M = p.M;
        a.gin = 0;
        a.NT = p.geo.NT;
        a.ahat = (const T *)p.d_bA;
        a.ahat_inv = p.d_bS;
        a.Tm = (const T *)p.d_bT;
        a.B0 = (const T *)p.d_bB;
        a.B1 = p.basis == L2C_NODAL ? (const T *)p.d_bB + p.M * p.M : nullptr;
        a.Pt = (const double *)p.d_bP;
        a.Qt = (const double *)p.d_bQ;
        a.w = (T *)p.d_bw;
        a.tile = a.bx = 0;
        cls[std::make_tuple(0, ku, 0, 0)].push_back({a, ((Pn >> ku) + 1) / 2});
        int pass = 0;
        for (int gin = L - 1 - ku; gin > 0; ++pass) {
            const int kt = gin < kBatTopDepth ? gin : kBatTopDepth;
            const int gout = gin - kt;
            BatArgs<T> at = a;
            at.gin = gin;
            cls[std::make_tuple(1, kt, 0, pass)].push_back({at, ((int64_t(1) << (gout + 2)) + 1) / 2});
            gin = gout;
        }
        const int groot = L - 1 - kd;
        cls[std::make_tuple(2, kd, (2 * p.s + 15) / 16, 0)].push_back({a, (int64_t(1) << (groot + 2)) / 2});
    }
    BatGrouped *G = new (std::nothrow) BatGrouped;
    if (!G) return hipErrorOutOfMemory;
    G->fm = fm;
    // launch order: every kb_up, then the kb_top passes in pass order, then every kb_main
    std::vector<std::tuple<int, int, int, int>> keys;
    for (auto &kv : cls) keys.push_back(kv.first);
    std::stable_sort(keys.begin(), keys.end(), [](const auto &x, const auto &y) {
        const int ox = std::get<0>(x) == 1 ? 1 + std::get<3>(x) : (std::get<0>(x) == 0 ? 0 : 1000);
        const int oy = std::get<0>(y) == 1 ? 1 + std::get<3>(y) : (std::get<0>(y) == 0 ? 0 : 1000);
        return ox < oy;
    });
    for (const auto &k : keys) {
        const auto &ents = cls[k];
        std::vector<int64_t> blk0(ents.size() + 1, 0);
        for (size_t e = 0; e < ents.size(); ++e) {
            const int64_t tiles = (ents[e].a.batch + 15) / 16;
            blk0[e + 1] = blk0[e] + ents[e].gx * tiles;
        }
        BatGrouped::Launch l{std::get<0>(k), std::get<1>(k), std::get<2>(k), nullptr, nullptr, (int)ents.size(),
                             blk0.back()};
        if (l.blocks > 0x7fffffff || dev_alloc(&l.E, ents.size() * sizeof(BatEntry<T>)) != hipSuccess ||
            dev_alloc(&l.blk0, blk0.size() * sizeof(int64_t)) != hipSuccess ||
            hipMemcpy(l.E, ents.data(), ents.size() * sizeof(BatEntry<T>), hipMemcpyHostToDevice) != hipSuccess ||
            hipMemcpy(l.blk0, blk0.data(), blk0.size() * sizeof(int64_t), hipMemcpyHostToDevice) != hipSuccess) {
            (void)hipGetLastError();
            G->launches.push_back(l);
            batched_grouped_free(G);
            return hipErrorOutOfMemory;
        }
        G->launches.push_back(l);
    }
    *out = G;
    return hipSuccess;
}

template <int FM>
static hipError_t grouped_launch_fm(const BatGrouped *G, hipStream_t st)
{
    typedef float T;
    for (const auto &l : G->launches) {
        if (l.blocks == 0) continue;
        const BatEntry<T> *E = (const BatEntry<T> *)l.E;
        const dim3 grid((unsigned)l.blocks), blk(256);
        switch (l.kind * 64 + l.k1 * 8 + l.k2) {
#define L2C_GUP(KK) \
    case 0 * 64 + KK * 8: hipLaunchKernelGGL((kbg_up<T, KK, FM>), grid, blk, 0, st, E, l.blk0, l.n); break;
            L2C_GUP(0) L2C_GUP(1) L2C_GUP(2) L2C_GUP(3)
#undef L2C_GUP
#define L2C_GTOP(KK) \
    case 1 * 64 + KK * 8: hipLaunchKernelGGL((kbg_top<T, KK, FM>), grid, blk, 0, st, E, l.blk0, l.n); break;
            L2C_GTOP(1) L2C_GTOP(2) L2C_GTOP(3)
#undef L2C_GTOP
#define L2C_GMAIN(KK, NN) \
    case 2 * 64 + KK * 8 + NN: hipLaunchKernelGGL((kbg_main<T, KK, NN, FM>), grid, blk, 0, st, E, l.blk0, l.n); break;
#define L2C_GMAIN4(KK) L2C_GMAIN(KK, 1) L2C_GMAIN(KK, 2) L2C_GMAIN(KK, 3) L2C_GMAIN(KK, 4)
            L2C_GMAIN4(0) L2C_GMAIN4(1) L2C_GMAIN4(2)
#undef L2C_GMAIN4
#undef L2C_GMAIN
        default: return hipErrorInvalidValue;
        }
        const hipError_t e = hipGetLastError();
        if (e != hipSuccess) return e;
    }
    return hipSuccess;
}

hipError_t batched_grouped_launch(const BatGrouped *G, hipStream_t st)
{
    return G->fm == 2 ? grouped_launch_fm<2>(G, st) : G->fm == 1 ? grouped_launch_fm<1>(G, st) : grouped_launch_fm<0>(G, st);
}

}  // namespace l2c
