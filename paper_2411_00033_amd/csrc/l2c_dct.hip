// l2c_dct.hip -- discrete cosine transforms of types 2 and 3 on a hand-written complex FFT,
// and the pipeline that evaluates a Legendre series on the Chebyshev-Gauss grid and back.
//
// Sec. 1 motivates the transform between Legendre and Chebyshev coefficients by the fast
// cosine transforms that the Chebyshev side allows: a Legendre series sum_k f_k P_k(x) is
// evaluated on the n Chebyshev-Gauss points x_j = cos((j + 1/2) pi / n) as leg2cheb
// (c = C^-1 A f, Eq. (directmv)) followed by u_j = sum_k c_k T_k(x_j) = sum_k c_k cos(pi k
// (j + 1/2) / n), a DCT of type 3; the inverse takes the DCT of type 2 of the values,
// c_k = (2 - delta_k0) / n sum_j u_j cos(pi k (j + 1/2) / n) (Chebyshev-Gauss quadrature,
// exact for the degree < n interpolant), then cheb2leg.  Sec. 5.2 times the FMM against a
// DCT of type 2.
//
// DCT through an n-point complex DFT (Makhoul's reordering): with v_m = x_{p(m)},
// p(m) = 2m for m < ceil(n/2) and 2(n-1-m)+1 otherwise,
//   DCT-2:  y_k = Re(e^{-i pi k / (2n)} V_k),  V = DFT(v);
//   DCT-3:  V_k = e^{i pi k / (2n)} (X_k - i X_{n-k}), X_0 = c_0, X_k = c_k / 2 (k >= 1),
//           X_n = 0;  v = unnormalized inverse DFT of V;  y_{p(m)} = Re v_m.
// The reordering and the quarter-wave factors are applied while the FFT loads its input
// and stores its output, so a DCT is one pass over the data (n <= 4096) or two (larger n).
//
// A DCT-3 of even length n >= 16 runs on a complex DFT of half the length, P = n / 2.
// Since V is Hermitian, v is real, and z_m = v_2m + i v_2m+1 (m < P) is the unnormalized
// inverse P-point DFT of
//   Z_k = q (A + B) + i q^5 (A - B),  q = e^{i pi k / (2n)},  A = X_k - i X_{n-k},
//   B = e^{i pi / 4} (X_{k+P} - i X_{P-k})        (V_k = q A, V_{k+P} = q B),
// so each Z_k reads the input at k, n - k, k + P and P - k, and the last pass writes
// Re z_m and Im z_m to rows p(2m) and p(2m+1): half the points, half the bytes per pass.
//
// The FFT: Stockham autosort passes of radix 8, 4, 2, 3, 5 and 7 on lines held in LDS
// (a workgroup takes C lines of length n, C n <= 4096 complex values, 64 KiB); every
// pass reads all its butterflies' inputs into registers, then writes the outputs in
// place, so one LDS buffer serves.  For n > 4096 the four-step split n = na nb, applied
// once (two passes: na, nb <= 512) or twice (three passes, n = na nb nc, each <= 4096 and
// as equal as the factors allow): with n = na (nb nc) and index t = ta (nb nc) + t',
// pass 1 takes the DFTs of length na along stride nb nc (one per t'; adjacent lines are
// adjacent in memory) and multiplies output ka by the twist exp(-+2 pi i ka t' / n); the
// rest is, for each ka, a DFT of length nb nc of contiguous data, split the same way, and
// output K of that DFT is output ka + na K of the whole.  The last pass stores adjacent
// lines (adjacent ka) at adjacent addresses.  Small factors keep many lines per workgroup
// (4096 / length), so every strided access moves hundreds of contiguous bytes.  The roots of unity come
// from tables built on the device with sincospi: per length, exp(-2 pi i t / len); for the
// twist and quarter-wave factors of length n, the product of two tables of about sqrt(n)
// entries (exact index split t = th b + tl), which keeps them in cache.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdlib>
#include <mutex>
#include <new>
#include <vector>

#include "l2c_alloc.h"
#include "../../include/leg2cheb.h"

namespace l2c {

constexpr int kFftLds = 4096;                    // complex values per workgroup, at most
constexpr int kFftSmall = 2048;                  // ... for lengths up to this
constexpr int kFftPre = 512;                     // lines up to this long load the store factors first
static_assert(kFftPre <= kFftSmall, "the up-front store factors live in the small kernel shape");
constexpr int kFftMaxPass = 16;
constexpr int64_t kFftMaxN = int64_t(1) << 27;

// kLoadDct3H / kStoreDct3H: the DCT-3 of an even length NR on a complex FFT of length
// N = NR / 2 (the split of the input before the first pass, of the output after the last)
enum { kLoadComplex = 0, kLoadDct2 = 1, kLoadDct3 = 2, kLoadDct3H = 3 };
enum { kStoreComplex = 0, kStoreDct2 = 1, kStoreDct3 = 2, kStoreDct3H = 3 };

struct FftArgs {
    int n;                     // DFT length of this launch
    int npass;
    int radix[kFftMaxPass];
    int C;                     // lines per workgroup
    int64_t lpt;               // lines per transform
    int64_t lines;             // lines of the launch (transforms x lpt)
    int64_t L1;                // line li of a transform = l1 + L1 l2
    int64_t es_in, ls1_in, ls2_in, es_out, ls1_out, ls2_out;   // index in a transform: e es + l1 ls1 + l2 ls2
    int64_t N;                 // transform length (of the complex DFT)
    int64_t NR;                // length of a real input or output row (N, or 2 N for the half-length DCT-3)
    int sign;                  // -1: forward DFT; +1: unnormalized inverse
    const double2 *tw;         // [n]: exp(-2 pi i t / n)
    int twist;                 // store: times exp(sign 2 pi i ((tw_full ? li : l1) e tmul mod N) / N)
    int tw_full;
    int64_t tmul;
    const double2 *wh, *wl;    // exp(-2 pi i m / N) = wh[m / wb] wl[m % wb]
    int64_t wb;
    const double2 *qh, *ql;    // exp(i pi k / (2N)) = qh[k / qb] ql[k % qb]
    int64_t qb;
    int load, store;
    int pre;                   // store factors loaded up front (n <= kFftPre, CAP = kFftSmall)
    double scale0, scale;      // DCT-2 store: y_0 scale0, y_k scale (k >= 1)
    const double *rin;         // real input [transform][N]
    double *rout;              // real output [transform][N]
    const double2 *cin;        // complex input [transform][N]
    double2 *cout;             // complex output [transform][N]
};

__device__ __forceinline__ double2 cmul(double2 a, double2 b)
{
    return make_double2(a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x);
}
__device__ __forceinline__ double2 cadd(double2 a, double2 b) { return make_double2(a.x + b.x, a.y + b.y); }
__device__ __forceinline__ double2 csub(double2 a, double2 b) { return make_double2(a.x - b.x, a.y - b.y); }
// sign * i * a
__device__ __forceinline__ double2 cmuli(double2 a, int sign)
{
    return sign < 0 ? make_double2(a.y, -a.x) : make_double2(-a.y, a.x);
}
__device__ __forceinline__ double2 conj_if(double2 a, bool c) { return c ? make_double2(a.x, -a.y) : a; }

// floor(x / d) for 0 <= x < 2^31 and 1 <= d < 2^18 in three FP64 operations: (x + 1/2) / d
// lies at least 1/(2d) from every integer, far above the product's rounding error.
struct FastDiv {
    int d;
    double inv;
    __device__ explicit FastDiv(int d_) : d(d_), inv(1.0 / (double)d_) {}
    __device__ __forceinline__ int quot(int x) const { return (int)(((double)x + 0.5) * inv); }
};


// cos and sin of 2 pi m / R, m = 1 .. (R-1)/2, for the odd radices
template <int R>
struct OddRoots;
template <>
struct OddRoots<3> {
    static constexpr double c[1] = {-0.5};
    static constexpr double s[1] = {0.8660254037844386467637};
};
template <>
struct OddRoots<5> {
    static constexpr double c[2] = {0.3090169943749474241023, -0.8090169943749474241023};
    static constexpr double s[2] = {0.9510565162951535721164, 0.5877852522924731291687};
};
template <>
struct OddRoots<7> {
    static constexpr double c[3] = {0.6234898018587335305251, -0.2225209339563144042889, -0.9009688679024191262361};
    static constexpr double s[3] = {0.7818314824680298087084, 0.9749279121818236070181, 0.4338837391175581204758};
};

// y_q = sum_r v_r w^(r q), w = exp(sign 2 pi i / R).  Odd R: with s_r = v_r + v_{R-r},
// d_r = v_r - v_{R-r} (r = 1 .. H, H = (R-1)/2), y_q = A_q + sign i B_q and
// y_{R-q} = A_q - sign i B_q, A_q = v_0 + sum_r s_r cos(2 pi r q / R),
// B_q = sum_r d_r sin(2 pi r q / R).
template <int R>
__device__ __forceinline__ void small_dft(double2 (&v)[R], int sign)
{
    if constexpr (R == 2) {
        const double2 a = v[0], b = v[1];
        v[0] = cadd(a, b);
        v[1] = csub(a, b);
    } else if constexpr (R == 4) {
        const double2 s02 = cadd(v[0], v[2]), d02 = csub(v[0], v[2]);
        const double2 s13 = cadd(v[1], v[3]), d13 = cmuli(csub(v[1], v[3]), sign);
        v[0] = cadd(s02, s13);
        v[2] = csub(s02, s13);
        v[1] = cadd(d02, d13);
        v[3] = csub(d02, d13);
    } else if constexpr (R == 8) {
        double2 e[4] = {v[0], v[2], v[4], v[6]}, o[4] = {v[1], v[3], v[5], v[7]};
        small_dft<4>(e, sign);
        small_dft<4>(o, sign);
        constexpr double h = 0.70710678118654752440;   // 1 / sqrt(2)
        const double sg = (double)sign;
        const double2 w1 = make_double2(h, sg * h), w3 = make_double2(-h, sg * h);
        const double2 t[4] = {o[0], cmul(o[1], w1), cmuli(o[2], sign), cmul(o[3], w3)};
#pragma unroll
        for (int q = 0; q < 4; ++q) {
            v[q] = cadd(e[q], t[q]);
            v[q + 4] = csub(e[q], t[q]);
        }
    } else {
        constexpr int H = (R - 1) / 2;
        double2 sm[H], df[H];
        double2 y0 = v[0];
#pragma unroll
        for (int r = 1; r <= H; ++r) {
            sm[r - 1] = cadd(v[r], v[R - r]);
            df[r - 1] = csub(v[r], v[R - r]);
            y0 = cadd(y0, sm[r - 1]);
        }
#pragma unroll
        for (int q = 1; q <= H; ++q) {
            double2 A = v[0], B = make_double2(0.0, 0.0);
#pragma unroll
            for (int r = 1; r <= H; ++r) {
                const int m = (r * q) % R, mm = m <= H ? m : R - m;   // cos is even, sin odd in m
                const double cs = OddRoots<R>::c[mm - 1], sn = m <= H ? OddRoots<R>::s[mm - 1] : -OddRoots<R>::s[mm - 1];
                A = make_double2(fma(sm[r - 1].x, cs, A.x), fma(sm[r - 1].y, cs, A.y));
                B = make_double2(fma(df[r - 1].x, sn, B.x), fma(df[r - 1].y, sn, B.y));
            }
            const double2 iB = cmuli(B, sign);
            v[q] = cadd(A, iB);
            v[R - q] = csub(A, iB);
        }
        v[0] = y0;
    }
}

// One Stockham pass of radix R over C lines of length n in LDS (Ns = product of the
// radices of the earlier passes): butterfly j of a line reads elements j + r n/R, applies
// exp(sign 2 pi i r k / (Ns R)), k = j mod Ns, and writes (j / Ns) Ns R + k + q Ns.
// CAP values of the workgroup's NT threads; tw = exp(-2 pi i t / n) in LDS.
template <int R, int CAP, int NT>
__device__ void fft_pass(double2 *buf, int n, int C, int Ns, int sign, const double2 *tw)
{
    constexpr int MB = (CAP / R + NT - 1) / NT;
    const int nb = n / R, tot = C * nb;
    const FastDiv dnb(nb), dns(Ns);
    double2 v[MB][R];
#pragma unroll
    for (int i = 0; i < MB; ++i) {
        const int b = (int)threadIdx.x + i * NT;
        if (b < tot) {
            const int c = dnb.quot(b), j = b - c * nb;
#pragma unroll
            for (int r = 0; r < R; ++r) v[i][r] = buf[c * n + j + r * nb];
        }
    }
    __syncthreads();
    const int step = n / (Ns * R);
#pragma unroll
    for (int i = 0; i < MB; ++i) {
        const int b = (int)threadIdx.x + i * NT;
        if (b < tot) {
            const int c = dnb.quot(b), j = b - c * nb, jq = dns.quot(j), k = j - jq * Ns;
#pragma unroll
            for (int r = 1; r < R; ++r) v[i][r] = cmul(v[i][r], conj_if(tw[r * k * step], sign > 0));
            small_dft<R>(v[i], sign);
            const int o = c * n + jq * Ns * R + k;
#pragma unroll
            for (int q = 0; q < R; ++q) buf[o + q * Ns] = v[i][q];
        }
    }
    __syncthreads();
}

// m = x mod N for 0 <= x < 2^52, in FP64 (exact: every value is an integer below 2^53)
__device__ __forceinline__ int mod_n(double x, double N, double invN)
{
    double r = x - trunc(x * invN) * N;
    if (r < 0.0) r += N;
    if (r >= N) r -= N;
    return (int)r;
}

// Per line of the workgroup, set up once: the transform's offset, the line's part of the
// in-transform index on both sides, and the twist multiplier (line index times tmul, mod N).
struct FftLine {
    int64_t base;        // transform * N; -1: past the last line
    int64_t rbase;       // transform * NR (the real rows)
    int gin, gout;
    int twa;
};

// One launch of the FFT: C lines per workgroup, loaded (with the DCT reordering or the
// quarter-wave factors of the first pass), transformed in LDS, stored (with the twist of
// the four-step split or the DCT's last factors).  LOAD and STORE are the kLoad / kStore
// modes.  Every global load of a workgroup is issued before the first of them is used:
// the input, the pass's root table, and (CAP / NT <= 4 values per thread) the twist or
// quarter-wave factors of the store, so a launch waits for memory once before its radix
// passes instead of three times.
template <int CAP, int NT, int LOAD, int STORE>
__global__ __launch_bounds__(NT, CAP <= 2048 ? 4 : 2) void k_fft(FftArgs a)
{
    extern __shared__ double2 smem[];
    const int n = a.n, C = a.C, N = (int)a.N;
    // store factors loaded up front (lines of at most kFftPre points): one per value, in a
    // slot of LDS private to the thread, so that no register holds them across the passes
    constexpr bool kPreOk = CAP == kFftSmall && (STORE == kStoreComplex || STORE == kStoreDct2) &&
                            (LOAD == kLoadComplex || LOAD == kLoadDct2);   // fft_pre_ok
    const bool pre = kPreOk && a.pre;
    double2 *buf = smem, *tw = smem + C * n, *fqs = tw + n;
    FftLine *ln = reinterpret_cast<FftLine *>(fqs + (pre ? CAP : 0));
    const int64_t line0 = (int64_t)blockIdx.x * C;
    for (int c = threadIdx.x; c < C; c += NT) {
        const int64_t line = line0 + c;
        FftLine L{-1, 0, 0, 0};
        if (line < a.lines) {
            const int64_t tr = line / a.lpt, li = line - tr * a.lpt;
            const int64_t l2 = li / a.L1, l1 = li - l2 * a.L1;
            L.base = tr * a.N;
            L.rbase = tr * a.NR;
            L.gin = (int)(l1 * a.ls1_in + l2 * a.ls2_in);
            L.gout = (int)(l1 * a.ls1_out + l2 * a.ls2_out);
            L.twa = a.twist ? (int)(((a.tw_full ? li : l1) * a.tmul) % a.N) : 0;
        }
        ln[c] = L;
    }
    __syncthreads();
    const int cnt = C * n;
    const int es_in = (int)a.es_in, es_out = (int)a.es_out;
    constexpr int EPT = CAP / NT;                 // elements per thread, at most
    constexpr int TPT = (CAP + NT - 1) / NT;      // root-table entries per thread, at most
    const double Nd = (double)N, invN = 1.0 / Nd;
    // input: adjacent threads take adjacent elements of a line, or (strided lines) the same
    // element of adjacent lines, whichever is adjacent in memory
    double2 raw[EPT], raw2[EPT], rh[EPT], rl[EPT];
    int pos[EPT], gg[EPT];
    const int NR = (int)a.NR;
    {
        const bool lcol = es_in != 1;
        const FastDiv dv(lcol ? C : n), dqb((int)a.qb);
#pragma unroll
        for (int u = 0; u < EPT; ++u) {
            const int idx = (int)threadIdx.x + u * NT;
            pos[u] = -1;
            gg[u] = -1;
            raw[u] = make_double2(0.0, 0.0);
            if (idx < cnt) {
                const int q = dv.quot(idx), rm = idx - q * dv.d;
                const int c = lcol ? rm : q, e = lcol ? q : rm;
                const FftLine L = ln[c];
                pos[u] = c * n + e;
                if (L.base >= 0) {
                    const int g = L.gin + e * es_in;
                    gg[u] = g;
                    if constexpr (LOAD == kLoadComplex) {
                        raw[u] = a.cin[L.base + g];
                    } else if constexpr (LOAD == kLoadDct2) {
                        raw[u].x = a.rin[L.rbase + (g < (N + 1) / 2 ? 2 * g : 2 * (N - 1 - g) + 1)];
                    } else if constexpr (LOAD == kLoadDct3) {
                        const double *x = a.rin + L.rbase;
                        raw[u] = make_double2(x[g], x[g == 0 ? 0 : N - g]);
                        const int th = dqb.quot(g);
                        rh[u] = a.qh[th];
                        rl[u] = a.ql[g - th * dqb.d];
                    } else {
                        // c at g, NR - g (none for g = 0), g + N and N - g (all inside the row)
                        const double *x = a.rin + L.rbase;
                        raw[u] = make_double2(x[g], g == 0 ? 0.0 : x[NR - g]);
                        raw2[u] = make_double2(x[g + N], x[N - g]);
                        const int th = dqb.quot(g);
                        rh[u] = a.qh[th];
                        rl[u] = a.ql[g - th * dqb.d];
                    }
                }
            }
        }
    }
    // the pass's roots
    double twx[TPT], twy[TPT];                  // (components: a conditional struct copy stays in memory)
#pragma unroll
    for (int u = 0; u < TPT; ++u) {
        const int t = (int)threadIdx.x + u * NT;
        twx[u] = twy[u] = 0.0;
        if (t < n) {
            const double2 w = a.tw[t];
            twx[u] = w.x;
            twy[u] = w.y;
        }
    }
    // store side: where each value goes and the factor it takes
    const bool scol = es_out != 1;
    const FastDiv dvs(scol ? C : n), dtb((int)(STORE == kStoreDct2 ? a.qb : a.wb));
    double2 sh[EPT], sl[EPT];
    int64_t dst[EPT], dst2[EPT];
    int sp[EPT], sg[EPT], st[EPT];
#pragma unroll
    for (int u = 0; u < EPT; ++u) {
        const int idx = (int)threadIdx.x + u * NT;
        dst[u] = -1;
        sg[u] = 0;
        sp[u] = 0;
        st[u] = -1;
        if (idx < cnt) {
            const int q = dvs.quot(idx), rm = idx - q * dvs.d;
            const int c = scol ? rm : q, e = scol ? q : rm;
            const FftLine L = ln[c];
            if (L.base >= 0) {
                const int g = L.gout + e * es_out;
                sg[u] = g;
                sp[u] = c * n + e;
                if constexpr (STORE == kStoreComplex) {
                    dst[u] = L.base + g;
                    if (a.twist) st[u] = mod_n((double)L.twa * (double)e, Nd, invN);
                } else if constexpr (STORE == kStoreDct2) {
                    dst[u] = L.rbase + g;
                    st[u] = g;
                } else if constexpr (STORE == kStoreDct3) {
                    dst[u] = L.rbase + (g < (N + 1) / 2 ? 2 * g : 2 * (N - 1 - g) + 1);
                } else {
                    // z_g = v_2g + i v_2g+1 goes to rows p(2g) and p(2g+1) of Makhoul's order
                    const int j0 = 2 * g, j1 = 2 * g + 1;
                    dst[u] = L.rbase + (j0 < NR / 2 ? 2 * j0 : 2 * (NR - 1 - j0) + 1);
                    dst2[u] = L.rbase + (j1 < NR / 2 ? 2 * j1 : 2 * (NR - 1 - j1) + 1);
                }
                if constexpr (kPreOk) {
                    if (pre && st[u] >= 0) {
                        const double2 *hi = STORE == kStoreDct2 ? a.qh : a.wh, *lo = STORE == kStoreDct2 ? a.ql : a.wl;
                        const int th = dtb.quot(st[u]);
                        sh[u] = hi[th];
                        sl[u] = lo[st[u] - th * dtb.d];
                    }
                }
            }
        }
    }
#pragma unroll
    for (int u = 0; u < TPT; ++u) {
        const int t = (int)threadIdx.x + u * NT;
        if (t < n) tw[t] = make_double2(twx[u], twy[u]);
    }
#pragma unroll
    for (int u = 0; u < EPT; ++u) {
        if (pos[u] < 0) continue;
        double2 v = raw[u];
        if constexpr (LOAD == kLoadDct3) {
            if (gg[u] >= 0) {
                const bool z = gg[u] == 0;
                v = cmul(cmul(rh[u], rl[u]), make_double2(z ? v.x : 0.5 * v.x, z ? 0.0 : -0.5 * v.y));
            }
        } else if constexpr (LOAD == kLoadDct3H) {
            if (gg[u] >= 0) {
                // Z_g = q (A + B) + i q^5 (A - B), q = exp(i pi g / (2 NR)), A = X_g - i X_(NR-g),
                // B = exp(i pi / 4) (X_(g+N) - i X_(N-g)); X_0 = c_0, X_k = c_k / 2, X_NR = 0
                const bool z = gg[u] == 0;
                const double2 A = make_double2(z ? v.x : 0.5 * v.x, -0.5 * v.y);
                const double2 b0 = make_double2(0.5 * raw2[u].x, -0.5 * raw2[u].y);
                constexpr double h = 0.70710678118654752440;   // 1 / sqrt(2)
                const double2 B = make_double2(h * (b0.x - b0.y), h * (b0.x + b0.y));
                // q^4 = e^{2 pi i g / NR} = e^{i pi g / N} from sincospi (powers of q would
                // compound the rounding of the tabulated q)
                double s4, c4;
                sincospi((double)gg[u] / (double)N, &s4, &c4);
                const double2 q = cmul(rh[u], rl[u]), q5 = cmul(q, make_double2(c4, s4));
                v = cadd(cmul(q, cadd(A, B)), cmuli(cmul(q5, csub(A, B)), 1));
            }
        }
        buf[pos[u]] = v;
    }
    // the store factor of each value as one complex number (twist: conjugated for the
    // inverse; DCT-2: times the output scale)
    if constexpr (kPreOk) {
        if (pre) {
#pragma unroll
            for (int u = 0; u < EPT; ++u) {
                double2 f = make_double2(1.0, 0.0);
                if (dst[u] >= 0 && st[u] >= 0) {
                    const double2 q = cmul(sh[u], sl[u]);
                    if constexpr (STORE == kStoreComplex) {
                        f = conj_if(q, a.sign > 0);
                    } else {
                        const double sc = sg[u] == 0 ? a.scale0 : a.scale;
                        f = make_double2(q.x * sc, q.y * sc);
                    }
                }
                fqs[u * NT + threadIdx.x] = f;
            }
        }
    }
    __syncthreads();
    int Ns = 1;
    for (int p = 0; p < a.npass; ++p) {
        const int R = a.radix[p];
        switch (R) {
        case 8: fft_pass<8, CAP, NT>(buf, n, C, Ns, a.sign, tw); break;
        case 4: fft_pass<4, CAP, NT>(buf, n, C, Ns, a.sign, tw); break;
        case 2: fft_pass<2, CAP, NT>(buf, n, C, Ns, a.sign, tw); break;
        case 3: fft_pass<3, CAP, NT>(buf, n, C, Ns, a.sign, tw); break;
        case 5: fft_pass<5, CAP, NT>(buf, n, C, Ns, a.sign, tw); break;
        default: fft_pass<7, CAP, NT>(buf, n, C, Ns, a.sign, tw); break;
        }
        Ns *= R;
    }
    double2 fq[EPT];
    if constexpr (STORE == kStoreComplex || STORE == kStoreDct2) {
#pragma unroll
        for (int u = 0; u < EPT; ++u) {
            fq[u] = make_double2(1.0, 0.0);
            if (kPreOk && pre) {
                fq[u] = fqs[u * NT + threadIdx.x];
            } else if (dst[u] >= 0 && st[u] >= 0) {
                const double2 *hi = STORE == kStoreDct2 ? a.qh : a.wh, *lo = STORE == kStoreDct2 ? a.ql : a.wl;
                const int th = dtb.quot(st[u]);
                const double2 q = cmul(hi[th], lo[st[u] - th * dtb.d]);
                if constexpr (STORE == kStoreComplex) {
                    fq[u] = conj_if(q, a.sign > 0);
                } else {
                    const double sc = sg[u] == 0 ? a.scale0 : a.scale;
                    fq[u] = make_double2(q.x * sc, q.y * sc);
                }
            }
        }
    }
#pragma unroll
    for (int u = 0; u < EPT; ++u) {
        if (dst[u] < 0) continue;
        const double2 val = buf[sp[u]];
        if constexpr (STORE == kStoreComplex) {
            a.cout[dst[u]] = cmul(val, fq[u]);
        } else if constexpr (STORE == kStoreDct2) {
            a.rout[dst[u]] = fq[u].x * val.x + fq[u].y * val.y;   // Re(conj(q) V), scaled
        } else if constexpr (STORE == kStoreDct3) {
            a.rout[dst[u]] = val.x;
        } else {
            a.rout[dst[u]] = val.x;
            a.rout[dst2[u]] = val.y;
        }
    }
}

// dst[t] = exp(i pi num(t) / den), num(t) = sgn * 2^e2 * t * mult, t < count
__global__ void k_roots(double2 *dst, int64_t count, int64_t mult, double den, double fac)
{
    const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= count) return;
    double s, c;
    sincospi(fac * (double)(t * mult) / den, &s, &c);
    dst[t] = make_double2(c, s);
}

}  // namespace l2c

// ------------------------------------------------------------------------------------
// Plans and the C ABI.

struct l2c_dct_s {
    int64_t n = 0;
    int kind = 2;
    int device = 0;
    int64_t nf = 0;                          // length of the complex DFT: n, or n / 2 for the half-length DCT-3
    std::vector<int64_t> dim;                // pass lengths (1 to 3), product nf
    std::vector<std::vector<int>> rad;       // radices per pass
    std::vector<double2 *> tw;               // per pass: exp(-2 pi i t / dim)
    double2 *wh = nullptr, *wl = nullptr;    // twist: exp(-2 pi i m / nf) = wh[m / wb] wl[m % wb]
    double2 *qh = nullptr, *ql = nullptr;    // quarter wave: exp(i pi k / (2 n)) = qh[k / qb] ql[k % qb]
    int64_t wb = 1, qb = 1;
    double2 *work = nullptr;                 // four-step intermediate [items][n]
    int64_t work_items = 0;
    double scale0 = 1.0, scale = 1.0;
};

struct l2c_grid_s {
    int64_t n = 0;
    int direction = 0;
    l2c_plan_t fmm = nullptr;
    l2c_dct_t dct = nullptr;
    double *tmp = nullptr;                   // [items][n]
    int64_t tmp_items = 0;
    int device = 0;
};

namespace {

constexpr int64_t kDct3HalfMin = 16;     // shortest DCT-3 taken on a half-length DFT

bool radices(int64_t n, std::vector<int> &out)
{
    out.clear();
    while (n % 8 == 0) { out.push_back(8); n /= 8; }
    while (n % 4 == 0) { out.push_back(4); n /= 4; }
    while (n % 2 == 0) { out.push_back(2); n /= 2; }
    for (int r : {3, 5, 7})
        while (n % r == 0) { out.push_back(r); n /= r; }
    return n == 1 && (int)out.size() <= l2c::kFftMaxPass;
}

int64_t isqrt_up(int64_t n)
{
    int64_t b = (int64_t)std::sqrt((double)n);
    while (b * b < n) ++b;
    return std::max<int64_t>(b, 1);
}

hipError_t roots(double2 **dst, int64_t count, int64_t mult, double den, double fac, hipStream_t st)
{
    hipError_t e = l2c::dev_alloc(dst, (size_t)count * sizeof(double2));
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(l2c::k_roots, dim3((unsigned)((count + 255) / 256)), dim3(256), 0, st, *dst, count, mult, den, fac);
    return hipGetLastError();
}

void free_dct(l2c_dct_t d)
{
    if (!d) return;
    for (const void *p : {(const void *)d->wh, (const void *)d->wl, (const void *)d->qh, (const void *)d->ql,
                          (const void *)d->work})
        l2c::dev_free(p);
    for (double2 *t : d->tw) l2c::dev_free(t);
    delete d;
}

int ensure_work(l2c_dct_t d, int64_t items)
{
    if (d->dim.size() == 1 || items <= d->work_items) return L2C_OK;
    if (hipDeviceSynchronize() != hipSuccess) return L2C_EHIP;
    l2c::dev_free(d->work);
    d->work = nullptr;
    d->work_items = 0;
    if (l2c::dev_alloc(&d->work, (size_t)items * d->n * sizeof(double2)) != hipSuccess) {
        (void)hipGetLastError();
        return L2C_ENOMEM;
    }
    d->work_items = items;
    return L2C_OK;
}

l2c::FftArgs base_args(const l2c_dct_t d)
{
    l2c::FftArgs a{};
    a.N = d->nf;
    a.NR = d->n;
    a.sign = d->kind == 2 ? -1 : 1;
    a.wh = d->wh;
    a.wl = d->wl;
    a.wb = d->wb;
    a.qh = d->qh;
    a.ql = d->ql;
    a.qb = d->qb;
    a.scale0 = d->scale0;
    a.scale = d->scale;
    return a;
}

void set_pass(l2c::FftArgs &a, int n, const std::vector<int> &r, const double2 *tw)
{
    a.n = n;
    a.npass = (int)r.size();
    for (int i = 0; i < a.npass; ++i) a.radix[i] = r[i];
    a.tw = tw;
    a.C = std::max(1, (n <= l2c::kFftSmall ? l2c::kFftSmall : l2c::kFftLds) / n);
}

// The launches whose kernel loads the store factors up front (the kernel's kPreOk, plus the
// line length): the LDS size depends on it.
bool fft_pre_ok(const l2c::FftArgs &a)
{
    return a.n <= l2c::kFftPre && (a.store == l2c::kStoreComplex || a.store == l2c::kStoreDct2) &&
           (a.load == l2c::kLoadComplex || a.load == l2c::kLoadDct2);
}

// The (load, store) pairs a DCT uses: one pass (DCT load and store), the first of several
// (DCT load, complex store), a middle one (complex, complex) and the last (complex load,
// DCT store).
template <int CAP>
const void *fft_kernel(int load, int store)
{
    using namespace l2c;
    if (load == kLoadDct2 && store == kStoreDct2) return (const void *)k_fft<CAP, 512, kLoadDct2, kStoreDct2>;
    if (load == kLoadDct3 && store == kStoreDct3) return (const void *)k_fft<CAP, 512, kLoadDct3, kStoreDct3>;
    if (load == kLoadDct2 && store == kStoreComplex) return (const void *)k_fft<CAP, 512, kLoadDct2, kStoreComplex>;
    if (load == kLoadDct3 && store == kStoreComplex) return (const void *)k_fft<CAP, 512, kLoadDct3, kStoreComplex>;
    if (load == kLoadComplex && store == kStoreComplex) return (const void *)k_fft<CAP, 512, kLoadComplex, kStoreComplex>;
    if (load == kLoadComplex && store == kStoreDct2) return (const void *)k_fft<CAP, 512, kLoadComplex, kStoreDct2>;
    if (load == kLoadComplex && store == kStoreDct3) return (const void *)k_fft<CAP, 512, kLoadComplex, kStoreDct3>;
    if (load == kLoadDct3H && store == kStoreDct3H) return (const void *)k_fft<CAP, 512, kLoadDct3H, kStoreDct3H>;
    if (load == kLoadDct3H && store == kStoreComplex) return (const void *)k_fft<CAP, 512, kLoadDct3H, kStoreComplex>;
    if (load == kLoadComplex && store == kStoreDct3H) return (const void *)k_fft<CAP, 512, kLoadComplex, kStoreDct3H>;
    return nullptr;
}

// Every kernel shape may take more than 64 KiB of dynamic LDS (up to 128 KiB + the line
// table at n = 4096): raise their limit once per process.
hipError_t fft_attrs()
{
    static std::once_flag once;
    static hipError_t err = hipSuccess;
    std::call_once(once, [] {
        const int lds = 160 * 1024;
        const int pairs[10][2] = {{l2c::kLoadDct2, l2c::kStoreDct2},       {l2c::kLoadDct3, l2c::kStoreDct3},
                                  {l2c::kLoadDct2, l2c::kStoreComplex},    {l2c::kLoadDct3, l2c::kStoreComplex},
                                  {l2c::kLoadComplex, l2c::kStoreComplex}, {l2c::kLoadComplex, l2c::kStoreDct2},
                                  {l2c::kLoadComplex, l2c::kStoreDct3},    {l2c::kLoadDct3H, l2c::kStoreDct3H},
                                  {l2c::kLoadDct3H, l2c::kStoreComplex},   {l2c::kLoadComplex, l2c::kStoreDct3H}};
        for (const auto &pr : pairs) {
            for (const void *k : {fft_kernel<l2c::kFftSmall>(pr[0], pr[1]), fft_kernel<l2c::kFftLds>(pr[0], pr[1])}) {
                if (err == hipSuccess) err = hipFuncSetAttribute(k, hipFuncAttributeMaxDynamicSharedMemorySize, lds);
            }
        }
    });
    return err;
}

hipError_t launch(const l2c::FftArgs &a, hipStream_t st)
{
    const int64_t blocks = (a.lines + a.C - 1) / a.C;
    if (blocks <= 0) return hipSuccess;
    const hipError_t e = fft_attrs();
    if (e != hipSuccess) return e;
    l2c::FftArgs b = a;
    b.pre = fft_pre_ok(a) ? 1 : 0;
    const size_t lds = ((size_t)a.C * a.n + a.n + (b.pre ? l2c::kFftSmall : 0)) * sizeof(double2) +
                       (size_t)a.C * sizeof(l2c::FftLine);
    const void *k = a.n <= l2c::kFftSmall ? fft_kernel<l2c::kFftSmall>(a.load, a.store)
                                          : fft_kernel<l2c::kFftLds>(a.load, a.store);
    if (!k) return hipErrorInvalidValue;
    void *args[] = {(void *)&b};
    return hipLaunchKernel(k, dim3((unsigned)blocks), dim3(512), args, lds, st);
}

int dct_run(l2c_dct_t d, const double *in, double *out, int64_t batch, hipStream_t st)
{
    const bool half = d->nf != d->n;         // the DCT-3 on a DFT of half the length
    const int load = d->kind == 2 ? l2c::kLoadDct2 : half ? l2c::kLoadDct3H : l2c::kLoadDct3;
    const int store = d->kind == 2 ? l2c::kStoreDct2 : half ? l2c::kStoreDct3H : l2c::kStoreDct3;
    const int P = (int)d->dim.size();
    const int64_t n = d->n, nf = d->nf;     // real rows of n; complex DFTs of nf
    // at most 2^30 lines per launch (grid.x), in whole transforms
    const int64_t per = std::max<int64_t>(1, (int64_t(1) << 30) / (P == 1 ? 1 : nf));
    for (int64_t b0 = 0; b0 < batch; b0 += per) {
        const int64_t nb = std::min(per, batch - b0);
        for (int p = 0; p < P; ++p) {
            l2c::FftArgs a = base_args(d);
            set_pass(a, (int)d->dim[p], d->rad[p], d->tw[p]);
            a.load = p == 0 ? load : l2c::kLoadComplex;
            a.store = p == P - 1 ? store : l2c::kStoreComplex;
            a.rin = in + b0 * n;
            a.rout = out + b0 * n;
            a.cin = d->work;
            a.cout = d->work;
            const int64_t lpt = nf / d->dim[p];
            a.lpt = lpt;
            a.lines = nb * lpt;
            a.L1 = lpt;
            a.tmul = 1;
            if (P == 1) {                       // one line per transform
                a.es_in = a.es_out = 1;
            } else if (p == 0) {                // along stride n / na, twist by the whole line index
                a.es_in = a.es_out = lpt;
                a.ls1_in = a.ls1_out = 1;
                a.twist = 1;
                a.tw_full = 1;
            } else if (p == P - 1) {            // contiguous rows; out at l1 + L1 (l2 + ...) order
                const int64_t nl = d->dim[P - 1];
                if (P == 2) {                   // lines ka
                    a.ls1_in = nl;
                    a.es_in = 1;
                    a.ls1_out = 1;
                    a.es_out = d->dim[0];
                } else {                        // lines (ka, kb), ka fastest
                    a.L1 = d->dim[0];
                    a.ls1_in = nf / d->dim[0];
                    a.ls2_in = nl;
                    a.es_in = 1;
                    a.ls1_out = 1;
                    a.ls2_out = d->dim[0];
                    a.es_out = d->dim[0] * d->dim[1];
                }
            } else {                            // P = 3, pass 2: lines (nc, ka) along stride nc
                const int64_t nc = d->dim[2], inner = d->dim[1] * nc;
                a.L1 = nc;
                a.es_in = a.es_out = nc;
                a.ls1_in = a.ls1_out = 1;
                a.ls2_in = a.ls2_out = inner;
                a.twist = 1;
                a.tw_full = 0;
                a.tmul = d->dim[0];             // exp(-2 pi i kb nc / (nb nc)) = exp(-2 pi i kb nc na / nf)
            }
            if (launch(a, st) != hipSuccess) return L2C_EHIP;
        }
    }
    return L2C_OK;
}

// Pass lengths: n itself (n <= 4096); two balanced factors when both are <= 512; else
// three factors <= 4096, the largest as small as possible.  Empty: not supported.
std::vector<int64_t> pass_lengths(int64_t n)
{
    if (n <= l2c::kFftLds) return {n};
    int64_t best = 0;
    for (int64_t f = 2; f * f <= n; ++f)
        if (n % f == 0) best = f;                       // the largest divisor <= sqrt(n)
    if (best && n / best <= 512) return {n / best, best};
    std::vector<int64_t> b3;
    for (int64_t a = 2; a <= l2c::kFftLds; ++a) {
        if (n % a) continue;
        const int64_t m = n / a;
        for (int64_t f = 1; f * f <= m; ++f) {
            if (m % f || m / f > l2c::kFftLds) continue;
            const int64_t c = m / f, mx = std::max(a, std::max(f, c));
            if (b3.empty() || mx < std::max(b3[0], std::max(b3[1], b3[2]))) b3 = {a, c, f};
        }
    }
    return b3;
}

int dct_length_ok(int64_t n)
{
    if (n > l2c::kFftMaxN) return L2C_EUNSUPPORTED;
    int64_t m = n;
    for (int64_t r : {2, 3, 5, 7})
        while (m % r == 0) m /= r;
    if (m != 1) return L2C_EUNSUPPORTED;            // prime factors 2, 3, 5, 7 only
    return pass_lengths(n).empty() ? L2C_EUNSUPPORTED : L2C_OK;
}

int dct_plan_impl(l2c_dct_t *dct, int64_t n, int kind, int64_t max_batch, void *stream)
{
    if (!dct) return L2C_EINVAL;
    *dct = nullptr;
    if (n < 1 || (kind != 2 && kind != 3) || max_batch < 1) return L2C_EINVAL;
    const int lrc = dct_length_ok(n);
    if (lrc != L2C_OK) return lrc;
    l2c_dct_t d = new (std::nothrow) l2c_dct_s();
    if (!d) return L2C_ENOMEM;
    d->n = n;
    d->kind = kind;
    if (hipGetDevice(&d->device) != hipSuccess) {
        delete d;
        return L2C_EHIP;
    }
    // the DCT-3 of an even length takes a complex DFT of half the length (the input split
    // into z_m = v_2m + i v_2m+1 of Makhoul's sequence v), when that length is supported
    d->nf = (kind == 3 && n % 2 == 0 && n >= kDct3HalfMin && !pass_lengths(n / 2).empty()) ? n / 2 : n;
    const int64_t nf = d->nf;
    d->dim = pass_lengths(nf);
    d->rad.resize(d->dim.size());
    d->tw.assign(d->dim.size(), nullptr);
    for (size_t i = 0; i < d->dim.size(); ++i) radices(d->dim[i], d->rad[i]);
    hipStream_t st = (hipStream_t)stream;
    d->wb = isqrt_up(nf);
    d->qb = isqrt_up(n);
    const int64_t wh_n = (nf + d->wb - 1) / d->wb + 1, qh_n = (n + d->qb - 1) / d->qb + 1;
    bool ok = true;
    for (size_t i = 0; i < d->dim.size() && ok; ++i)
        ok = roots(&d->tw[i], d->dim[i], 1, (double)d->dim[i], -2.0, st) == hipSuccess;
    ok = ok && roots(&d->wl, d->wb, 1, (double)nf, -2.0, st) == hipSuccess &&
              roots(&d->wh, wh_n, d->wb, (double)nf, -2.0, st) == hipSuccess &&
              roots(&d->ql, d->qb, 1, 2.0 * (double)n, 1.0, st) == hipSuccess &&
              roots(&d->qh, qh_n, d->qb, 2.0 * (double)n, 1.0, st) == hipSuccess;
    if (!ok) {
        (void)hipGetLastError();
        free_dct(d);
        return L2C_ENOMEM;
    }
    const int rc = ensure_work(d, max_batch);
    if (rc != L2C_OK || hipStreamSynchronize(st) != hipSuccess) {
        (void)hipGetLastError();
        free_dct(d);
        return rc != L2C_OK ? rc : L2C_EHIP;
    }
    *dct = d;
    return L2C_OK;
}

int check_io(int64_t n, const double *in, double *out, int64_t batch, int device)
{
    if (!in || !out || batch < 0) return L2C_EINVAL;
    if (batch > (int64_t(1) << 40) / n) return L2C_EINVAL;
    const int64_t len = batch * n;
    const char *ib = (const char *)in, *ie = (const char *)(in + len);
    const char *ob = (const char *)out, *oe = (const char *)(out + len);
    if (ib < oe && ob < ie) return L2C_EINVAL;
    int dev = -1;
    if (hipGetDevice(&dev) != hipSuccess) return L2C_EHIP;
    if (dev != device) return L2C_EINVAL;
    return L2C_OK;
}

}  // namespace

extern "C" {

int leg2cheb_dct_plan(l2c_dct_t *dct, int64_t n, int kind, int64_t max_batch, void *stream)
{
    return dct_plan_impl(dct, n, kind, max_batch, stream);
}

int leg2cheb_dct_execute(l2c_dct_t dct, const double *in, double *out, int64_t batch, void *stream)
{
    if (!dct || batch < 0) return L2C_EINVAL;
    if (batch == 0) return L2C_OK;
    int rc = check_io(dct->n, in, out, batch, dct->device);
    if (rc != L2C_OK) return rc;
    rc = ensure_work(dct, batch);
    if (rc != L2C_OK) return rc;
    return dct_run(dct, in, out, batch, (hipStream_t)stream);
}

int leg2cheb_dct_destroy(l2c_dct_t dct)
{
    if (!dct) return L2C_OK;
    const bool ok = hipDeviceSynchronize() == hipSuccess;
    free_dct(dct);
    return ok ? L2C_OK : L2C_EHIP;
}

int leg2cheb_grid_plan(l2c_grid_t *grid, int64_t n, int direction, int leaf_size, int rank, int64_t max_batch,
                       void *stream)
{
    if (!grid) return L2C_EINVAL;
    *grid = nullptr;
    if (n < 1 || (direction != L2C_LEG2GRID && direction != L2C_GRID2LEG) || max_batch < 1) return L2C_EINVAL;
    if (leaf_size < 4 || leaf_size > 128 || (leaf_size & 1) || rank < 1 || rank > 32) return L2C_EINVAL;
    const int lrc = dct_length_ok(n);
    if (lrc != L2C_OK) return lrc;
    l2c_grid_t g = new (std::nothrow) l2c_grid_s();
    if (!g) return L2C_ENOMEM;
    g->n = n;
    g->direction = direction;
    if (hipGetDevice(&g->device) != hipSuccess) {
        delete g;
        return L2C_EHIP;
    }
    int rc = leg2cheb_dct_plan(&g->dct, n, direction == L2C_LEG2GRID ? 3 : 2, max_batch, stream);
    if (rc == L2C_OK) {
        if (direction == L2C_GRID2LEG) {   // Chebyshev coefficients of the interpolant
            g->dct->scale0 = 1.0 / (double)n;
            g->dct->scale = 2.0 / (double)n;
        }
        rc = leg2cheb_plan_ex(&g->fmm, n, direction == L2C_LEG2GRID ? L2C_LEG2CHEB : L2C_CHEB2LEG, leaf_size, rank,
                              L2C_FP64, max_batch, stream);
    }
    if (rc == L2C_OK && l2c::dev_alloc(&g->tmp, (size_t)max_batch * n * sizeof(double)) != hipSuccess) {
        (void)hipGetLastError();
        rc = L2C_ENOMEM;
    }
    if (rc != L2C_OK) {
        leg2cheb_grid_destroy(g);
        return rc;
    }
    g->tmp_items = max_batch;
    *grid = g;
    return L2C_OK;
}

int leg2cheb_grid_execute(l2c_grid_t grid, const double *in, double *out, int64_t batch, void *stream)
{
    if (!grid || batch < 0) return L2C_EINVAL;
    if (batch == 0) return L2C_OK;
    int rc = check_io(grid->n, in, out, batch, grid->device);
    if (rc != L2C_OK) return rc;
    if (batch > grid->tmp_items) {
        if (hipDeviceSynchronize() != hipSuccess) return L2C_EHIP;
        l2c::dev_free(grid->tmp);
        grid->tmp = nullptr;
        grid->tmp_items = 0;
        if (l2c::dev_alloc(&grid->tmp, (size_t)batch * grid->n * sizeof(double)) != hipSuccess) {
            (void)hipGetLastError();
            return L2C_ENOMEM;
        }
        grid->tmp_items = batch;
    }
    if (grid->direction == L2C_LEG2GRID) {
        rc = leg2cheb_execute(grid->fmm, in, grid->tmp, batch, stream);
        return rc != L2C_OK ? rc : leg2cheb_dct_execute(grid->dct, grid->tmp, out, batch, stream);
    }
    rc = leg2cheb_dct_execute(grid->dct, in, grid->tmp, batch, stream);
    return rc != L2C_OK ? rc : leg2cheb_execute(grid->fmm, grid->tmp, out, batch, stream);
}

l2c_plan_t leg2cheb_grid_fmm(l2c_grid_t grid) { return grid ? grid->fmm : nullptr; }

l2c_dct_t leg2cheb_grid_dct(l2c_grid_t grid) { return grid ? grid->dct : nullptr; }

int leg2cheb_grid_destroy(l2c_grid_t grid)
{
    if (!grid) return L2C_OK;
    const bool ok = hipDeviceSynchronize() == hipSuccess;
    int rc = leg2cheb_destroy(grid->fmm);
    const int rc2 = leg2cheb_dct_destroy(grid->dct);
    l2c::dev_free(grid->tmp);
    delete grid;
    if (rc == L2C_OK) rc = rc2;
    return !ok ? L2C_EHIP : rc;
}

}  // extern "C"
