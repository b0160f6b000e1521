/*
 * cpu_fmm.cpp -- single-threaded CPU implementation of the modal multipole
 * Legendre <-> Chebyshev transform (Mortensen, arXiv 2411.00033, Alg. 4), the
 * CPU baseline that the GPU path is timed against.
 *
 * TEST AND BENCHMARK INFRASTRUCTURE ONLY.  The product library never links, loads
 * or calls it; only the test suite and the CPU-baseline leg of the benchmark do.
 * It shares no code with the direct oracle (oracle.c) or with the GPU library:
 * every table and step below is written here from the paper.
 *
 * Plan (Secs. 3.1-3.3, 4.2-4.3), all FP64:
 *   sizes      Eq. (numlevels): s_hat = leaf/2, L = ceil(log2(n/s_hat)) - 2,
 *              s = ceil(n/2^(L+2)), N = s 2^(L+2); L <= 0: the direct product (Alg. 1).
 *   lambda_k   Eq. (Lambdaint) upward from sqrt(pi) for k < 20; from k = 20 on, every
 *              8th value from the asymptotic series of Eq. (tau) and the recursion in
 *              between (the resynchronisation of Sec. 4.3).
 *   Lambda(z)  for real z (kernel samples): Eq. (tau) at z >= 20, shifted up with
 *              Lambda(z) = Lambda(z+1) (z+1)/(z+1/2) below.
 *   B(0),B(1)  Eq. (Tky): coefficients of T_n((Y + 2l - 1)/2) in T_k(Y), by the
 *              three-term recurrence (exact dyadic rationals).
 *   T(sigma)   Eq. (Xs): T_k(-1 + (2m + sigma)/s).
 *   Ahat       Eq. (aklmore): the kernel (Sec. 3.2 for leg2cheb, Eq. (Lxymod) for
 *              cheb2leg) sampled at the M x M Chebyshev-Gauss points of each
 *              submatrix, then the 2-D DCT-II.  The factor Lambda((y-x)/2) depends only
 *              on the level, the submatrix kind r and the sample pair, so it is
 *              evaluated once per level (Sec. 4.3); Lambda((x+y)/2) once per submatrix.
 * Execute (Alg. 4), per parity sigma, with the input and output split by parity
 * (u_sigma[k] = u[2k + sigma], so every step reads and writes contiguously) and
 * level-major node arrays (level g has 2^(g+2) nodes; w and c hold [node][sigma][k],
 * so each table row is read once for both parities):
 *   (0) u = f zero-padded to N; cheb2leg applies c first (u_0 = 2 f_0).
 *   (1) w(L-1, t) = T(sigma)^T u[2 s t + 2m + sigma], Eq. (wMM), column nodes t >= 2.
 *   (2) w(g-1, v) = B(0) w(g, 2v) + B(1) w(g, 2v+1), Eq. (wtk), with B(1) = B(0) with
 *       its odd diagonals negated (App. A2): one lower-triangular product of
 *       z_{(n-k) mod 2} with z0 = x + y, z1 = x - y.
 *   (3) c(g, 2b + p) += Ahat(g, b, r(p,q)) w(g, 2b + q + 2), Eqs. (globalij), (cfrompq).
 *   (4) c(g+1, v) += B(v mod 2)^T c(g, v/2), the downward pass.
 *   (5) z[2 s u + 2m + sigma] = T(sigma) c(L-1, u), Eq. (step5), rows below N - 4s.
 *   (6) the near-diagonal entries: finest row node u against columns [2su, 2s(u+2)).
 *       leg2cheb a_ij = lambda_{(j-i)/2} lambda_{(i+j)/2} (Eq. (hik)); cheb2leg the
 *       entries of Eq. (Lxymod) regrouped exactly as (2i+1) P_d Q_S j with d = (j-i)/2,
 *       S = (i+j)/2, P_d = lambda_d/(1-2d), Q_S = 1/(2S(2S+1) lambda_S), and the
 *       (0,0) entry 1/2 (its limit).
 *   (7) leg2cheb: z_i /= c_i pi/2.
 * Single thread, no BLAS: plain loops in the order that keeps each table read once.
 */
#include <cmath>
#include <cstdint>
#include <cstdlib>
#include <cstring>
#include <new>
#include <vector>

namespace {

constexpr double kSqrtPi = 1.77245385090551602729816748334114518;
constexpr double kPi = 3.14159265358979323846264338327950288;

double tau(double x)   // Eq. (tau): Lambda(z) = tau(z + 1/4) / sqrt(z + 1/4)
{
    const double t = 1.0 / (x * x);
    return 1.0 + t * (-1.0 / 64.0 + t * (21.0 / 8192.0 + t * (-671.0 / 524288.0 + t * (180323.0 / 134217728.0))));
}

double Lambda_real(double z)
{
    double scale = 1.0;
    while (z < 20.0) {
        scale *= (z + 1.0) / (z + 0.5);
        z += 1.0;
    }
    const double x = z + 0.25;
    return scale * tau(x) / std::sqrt(x);
}

struct Fmm {
    int64_t n = 0, N = 0;
    int L = 0, s = 0, M = 0, dir = 0;
    std::vector<double> lam;     // lambda_k, k < N + 2s (near-field arguments)
    std::vector<double> Pd, Qs;  // cheb2leg near-field factors
    std::vector<double> T;       // [2][s][M]
    std::vector<double> B0;      // [M][M], lower triangular
    std::vector<std::vector<double>> A;   // per level: [b][3][M][M]
    // execution scratch
    std::vector<double> u, z;
    std::vector<std::vector<double>> w, c;   // per level: [2^(g+2)][sigma][M]
};

void lambda_table(Fmm &F, int64_t len)
{
    F.lam.assign(len, 0.0);
    double v = kSqrtPi;
    for (int64_t k = 0; k < len; ++k) {
        if (k > 0) v *= ((double)k - 0.5) / (double)k;
        if (k >= 20 && k % 8 == 0) {
            const double x = (double)k + 0.25;
            v = tau(x) / std::sqrt(x);
        }
        F.lam[k] = v;
    }
}

void b_matrix(Fmm &F)
{
    const int M = F.M;
    // rows n: T_n((Y - 1)/2) in T_k(Y) (l = 0); u = (Y - 1)/2, T_{n+1} = 2u T_n - T_{n-1},
    // Y T_k = (T_{k+1} + T_{|k-1|}) / 2
    std::vector<double> prev(M + 1, 0.0), cur(M + 1, 0.0), nxt(M + 1, 0.0);
    F.B0.assign((size_t)M * M, 0.0);
    prev[0] = 1.0;                        // T_0
    cur[0] = -0.5;
    cur[1] = 0.5;                         // T_1(u) = (Y - 1)/2
    for (int k = 0; k < M; ++k) F.B0[k] = k == 0 ? 1.0 : 0.0;
    if (M > 1)
        for (int k = 0; k < M; ++k) F.B0[M + k] = cur[k];
    for (int r = 2; r < M; ++r) {
        std::fill(nxt.begin(), nxt.end(), 0.0);
        for (int k = 0; k < r; ++k) {
            const double a = cur[k];
            if (a == 0.0) continue;
            // (Y - 1) T_k = T_{k+1}/2 + T_{|k-1|}/2 - T_k
            nxt[k + 1] += 0.5 * a;
            nxt[k == 0 ? 1 : k - 1] += 0.5 * a;
            nxt[k] -= a;
        }
        for (int k = 0; k <= r; ++k) nxt[k] -= prev[k];
        prev = cur;
        cur = nxt;
        for (int k = 0; k < M; ++k) F.B0[(size_t)r * M + k] = cur[k];
    }
}

void build_ahat(Fmm &F)
{
    const int L = F.L, M = F.M, s = F.s;
    std::vector<double> X(M), D((size_t)M * M), Lm((size_t)3 * M * M), S((size_t)M * M), U((size_t)M * M);
    for (int m = 0; m < M; ++m) X[m] = std::cos((m + 0.5) * kPi / M);
    for (int k = 0; k < M; ++k)
        for (int m = 0; m < M; ++m) D[(size_t)k * M + m] = std::cos(k * (m + 0.5) * kPi / M);
    F.A.assign(L, std::vector<double>());
    for (int g = 0; g < L; ++g) {
        const int64_t bg = (int64_t(1) << (g + 1)) - 1;
        const double h = (double)((int64_t)s << (L - g - 1));
        F.A[g].assign((size_t)bg * 3 * M * M, 0.0);
        // Lambda((y - x)/2): y - x = 2h (q - p + 2) + h (X_n - X_m), fixed per level and r
        for (int r = 0; r < 3; ++r) {
            const int p = r == 2 ? 1 : 0, q = r == 0 ? 0 : 1;
            for (int m = 0; m < M; ++m)
                for (int nn = 0; nn < M; ++nn)
                    Lm[((size_t)r * M + m) * M + nn] = Lambda_real(0.5 * (2.0 * h * (q - p + 2) + h * (X[nn] - X[m])));
        }
        for (int64_t b = 0; b < bg; ++b)
            for (int r = 0; r < 3; ++r) {
                const int p = r == 2 ? 1 : 0, q = r == 0 ? 0 : 1;
                const double i0 = 2.0 * h * (double)(2 * b + p), j0 = 2.0 * h * (double)(2 * b + q + 2);
                for (int m = 0; m < M; ++m)
                    for (int nn = 0; nn < M; ++nn) {
                        const double x = i0 + h * (X[m] + 1.0), y = j0 + h * (X[nn] + 1.0);
                        const double lm = Lm[((size_t)r * M + m) * M + nn];
                        double v;
                        if (F.dir == 0) {
                            v = lm * Lambda_real(0.5 * (x + y));
                        } else {
                            const double gg = 2.0 * (x + 0.5) * y / ((x + y) * (x + y + 1.0) * (x - y + 1.0));
                            v = gg * lm / Lambda_real(0.5 * (x + y));
                        }
                        S[(size_t)m * M + nn] = v;
                    }
                // 2-D DCT-II: Ahat_kl = 4/(c_k c_l M^2) sum_m D_km sum_n S_mn D_ln
                for (int m = 0; m < M; ++m)
                    for (int l = 0; l < M; ++l) {
                        double acc = 0.0;
                        for (int nn = 0; nn < M; ++nn) acc += S[(size_t)m * M + nn] * D[(size_t)l * M + nn];
                        U[(size_t)m * M + l] = acc;
                    }
                double *Ab = &F.A[g][((size_t)b * 3 + r) * M * M];
                for (int k = 0; k < M; ++k)
                    for (int l = 0; l < M; ++l) {
                        double acc = 0.0;
                        for (int m = 0; m < M; ++m) acc += D[(size_t)k * M + m] * U[(size_t)m * M + l];
                        Ab[(size_t)k * M + l] = acc * 4.0 / ((k == 0 ? 2.0 : 1.0) * (l == 0 ? 2.0 : 1.0) * M * M);
                    }
            }
    }
}

// (2): w(g-1, v) = B(0) w(g, 2v) + B(1) w(g, 2v+1) for the column nodes v >= 2 of level g-1,
// both parities (nodes hold [sigma][k])
void upward_level(const Fmm &F, const double *child, double *par, int64_t vlo, int64_t vhi)
{
    const int M = F.M, M2 = 2 * M;
    double z0[128], z1[128];
    for (int64_t v = vlo; v < vhi; ++v) {
        const double *x = child + 2 * v * M2, *y = x + M2;
#pragma omp simd
        for (int k = 0; k < M2; ++k) {
            z0[k] = x[k] + y[k];
            z1[k] = x[k] - y[k];
        }
        double *o = par + v * M2;
        for (int nn = 0; nn < M; ++nn) {
            const double *b = &F.B0[(size_t)nn * M];
            double a0 = 0.0, a1 = 0.0;
            for (int k = 0; k <= nn; ++k) {
                const double *zz = ((nn - k) & 1) ? z1 : z0;
                a0 += b[k] * zz[k];
                a1 += b[k] * zz[M + k];
            }
            o[nn] = a0;
            o[M + nn] = a1;
        }
    }
}

// (4): c(g+1, v) += B(v mod 2)^T c(g, v/2); (B(p)^T c)_n = s_p(n) sum_{k >= n} b_kn s_p(k) c_k,
// both parities
void downward_level(const Fmm &F, const double *par, double *child, int64_t vhi)
{
    const int M = F.M, M2 = 2 * M;
    double cs[128];
    for (int64_t v = 0; v < vhi; ++v) {
        const int p = (int)(v & 1);
        const double *cp = par + (v >> 1) * M2;
        for (int k = 0; k < M; ++k) {
            const double sg = (p && (k & 1)) ? -1.0 : 1.0;
            cs[k] = sg * cp[k];
            cs[M + k] = sg * cp[M + k];
        }
        double *o = child + v * M2;
        for (int nn = 0; nn < M; ++nn) {
            double a0 = 0.0, a1 = 0.0;
            for (int k = nn; k < M; ++k) {
                const double b = F.B0[(size_t)k * M + nn];
                a0 += b * cs[k];
                a1 += b * cs[M + k];
            }
            const double sg = (p && (nn & 1)) ? -1.0 : 1.0;
            o[nn] += sg * a0;
            o[M + nn] += sg * a1;
        }
    }
}

void execute(Fmm &F, const double *f, double *out)
{
    const int64_t n = F.n, N = F.N, H = (N + 1) / 2;
    // (0) the input split by parity: up[sigma][k] = u[2k + sigma] (zero past n)
    double *up[2] = {F.u.data(), F.u.data() + H + 64};
    double *zp[2] = {F.z.data(), F.z.data() + H + 64};
    std::fill(F.u.begin(), F.u.end(), 0.0);
    std::fill(F.z.begin(), F.z.end(), 0.0);
    for (int64_t j = 0; j < n; ++j) up[j & 1][j >> 1] = f[j];
    if (F.dir == 1) up[0][0] *= 2.0;
    if (F.L > 0) {
        const int L = F.L, M = F.M, s = F.s, M2 = 2 * M;
        const int64_t P = N / (2 * s);   // finest nodes
        // (1): node t of parity sigma covers up[sigma][s t .. s t + s); w holds [node][sigma][k]
        double *wf = F.w[L - 1].data();
        for (int64_t t = 2; t < P; ++t)
            for (int sig = 0; sig < 2; ++sig) {
                double *o = wf + t * M2 + sig * M;
                const double *Ts = &F.T[(size_t)sig * s * M];
                for (int k = 0; k < M; ++k) o[k] = 0.0;
                const double *ut = up[sig] + s * t;
                for (int m = 0; m < s; ++m) {
                    const double um = ut[m];
                    const double *tr = Ts + (size_t)m * M;
#pragma omp simd
                    for (int k = 0; k < M; ++k) o[k] += tr[k] * um;
                }
            }
        // (2)
        for (int g = L - 1; g > 0; --g)
            upward_level(F, F.w[g].data(), F.w[g - 1].data(), 2, (int64_t(1) << (g + 1)));
        // (3): each row of Ahat is read once and applied to both parities
        for (int g = 0; g < L; ++g) {
            const int64_t bg = (int64_t(1) << (g + 1)) - 1;
            double *cg = F.c[g].data();
            std::fill(F.c[g].begin(), F.c[g].end(), 0.0);
            const double *wg = F.w[g].data();
            for (int64_t b = 0; b < bg; ++b) {
                const double *Ab = &F.A[g][(size_t)b * 3 * M * M];
                const double *w2 = wg + (2 * b + 2) * M2, *w3 = w2 + M2;
                double *c0 = cg + 2 * b * M2, *c1 = c0 + M2;
                for (int k = 0; k < M; ++k) {
                    const double *a0 = Ab + (size_t)k * M, *a1 = a0 + M * M, *a2 = a1 + M * M;
                    double e00 = 0.0, e01 = 0.0, e10 = 0.0, e11 = 0.0;
#pragma omp simd reduction(+ : e00, e01, e10, e11)
                    for (int l = 0; l < M; ++l) {
                        e00 += a0[l] * w2[l] + a1[l] * w3[l];
                        e01 += a0[l] * w2[M + l] + a1[l] * w3[M + l];
                        e10 += a2[l] * w3[l];
                        e11 += a2[l] * w3[M + l];
                    }
                    c0[k] += e00;
                    c0[M + k] += e01;
                    c1[k] += e10;
                    c1[M + k] += e11;
                }
            }
        }
        // (4)
        for (int g = 0; g + 1 < L; ++g)
            downward_level(F, F.c[g].data(), F.c[g + 1].data(), (int64_t(1) << (g + 3)) - 4);
        // (5): row node uu of parity sigma covers zp[sigma][s uu .. s uu + s)
        const double *cf = F.c[L - 1].data();
        for (int sig = 0; sig < 2; ++sig) {
            const double *Ts = &F.T[(size_t)sig * s * M];
            double *zs = zp[sig];
            for (int64_t uu = 0; uu + 2 < P; ++uu) {
                const double *cu = cf + uu * M2 + sig * M;
                double *zu = zs + s * uu;
                for (int m = 0; m < s; ++m) {
                    const double *tr = Ts + (size_t)m * M;
                    double acc = 0.0;
#pragma omp simd reduction(+ : acc)
                    for (int k = 0; k < M; ++k) acc += tr[k] * cu[k];
                    zu[m] = acc;
                }
            }
        }
    }
    // (6): row i = 2m + sigma of node block [i0, i0 + span) against j = i + 2d < jhi;
    // cheb2leg reads g_j = j u_j
    if (F.dir == 1)
        for (int sig = 0; sig < 2; ++sig)
            for (int64_t k = 0; k < H; ++k) up[sig][k] *= (double)(2 * k + sig);
    const int64_t span = F.L > 0 ? 2 * (int64_t)F.s : N;
    const double *fac = F.dir == 0 ? F.lam.data() : F.Pd.data();
    const double *row = F.dir == 0 ? F.lam.data() : F.Qs.data();
    for (int64_t i0 = 0; i0 < N; i0 += span) {
        const int64_t jhi = std::min(N, i0 + 2 * span);
        for (int64_t i = i0; i < std::min(N, i0 + span); ++i) {
            const int sig = (int)(i & 1);
            const int64_t m = i >> 1, dn = (jhi - i + 1) / 2;   // terms d < dn
            const double *us = up[sig] + m, *r1 = row + i;
            double acc = 0.0;
#pragma omp simd reduction(+ : acc)
            for (int64_t d = 0; d < dn; ++d) acc += fac[d] * r1[d] * us[d];
            if (F.dir == 1) {
                acc *= 2.0 * (double)i + 1.0;
                if (i == 0) acc += 0.5 * (2.0 * f[0]);   // K_00 u_0, u_0 = 2 f_0
            }
            zp[sig][m] += acc;
        }
    }
    // (7) and the output (interleave the parities)
    for (int64_t i = 0; i < n; ++i) {
        double v = zp[i & 1][i >> 1];
        if (F.dir == 0) v *= i == 0 ? 1.0 / kPi : 2.0 / kPi;
        out[i] = v;
    }
}

}  // namespace

extern "C" {

/* Plan a transform of length n (direction 0 leg2cheb, 1 cheb2leg); NULL on bad arguments. */
void *cpu_fmm_plan(int64_t n, int direction, int leaf, int rank)
{
    if (n < 1 || (direction != 0 && direction != 1) || leaf < 4 || (leaf & 1) || rank < 1 || rank > 64) return nullptr;
    Fmm *F = new (std::nothrow) Fmm;
    if (!F) return nullptr;
    F->n = n;
    F->dir = direction;
    F->M = rank;
    const int64_t shat = leaf / 2;
    int p = 0;
    while ((shat << p) < n) ++p;
    F->L = p - 2;
    if (F->L <= 0) {
        F->L = 0;
        F->s = 0;
        F->N = n;
    } else {
        F->s = (int)((n + (int64_t(1) << (F->L + 2)) - 1) >> (F->L + 2));
        F->N = (int64_t)F->s << (F->L + 2);
    }
    const int64_t N = F->N, nn2 = N + 2 * (int64_t)F->s + 2;
    lambda_table(*F, nn2);
    if (direction == 1) {
        F->Pd.assign(nn2, 0.0);
        F->Qs.assign(nn2, 0.0);
        for (int64_t d = 0; d < nn2; ++d) F->Pd[d] = F->lam[d] / (1.0 - 2.0 * (double)d);
        for (int64_t S = 1; S < nn2; ++S) F->Qs[S] = 1.0 / (2.0 * S * (2.0 * S + 1.0) * F->lam[S]);
    }
    F->u.assign((size_t)2 * ((N + 1) / 2 + 64), 0.0);   // two parity halves
    F->z.assign((size_t)2 * ((N + 1) / 2 + 64), 0.0);
    if (F->L > 0) {
        const int s = F->s, M = F->M;
        F->T.assign((size_t)2 * s * M, 0.0);
        for (int sig = 0; sig < 2; ++sig)
            for (int m = 0; m < s; ++m) {
                const double X = -1.0 + (double)(2 * m + sig) / (double)s;
                double t0 = 1.0, t1 = X;
                for (int k = 0; k < M; ++k) {
                    F->T[((size_t)sig * s + m) * M + k] = t0;
                    const double t2 = 2.0 * X * t1 - t0;
                    t0 = t1;
                    t1 = t2;
                }
            }
        b_matrix(*F);
        build_ahat(*F);
        F->w.assign(F->L, std::vector<double>());
        F->c.assign(F->L, std::vector<double>());
        for (int g = 0; g < F->L; ++g) {
            F->w[g].assign((size_t)(int64_t(1) << (g + 2)) * 2 * M, 0.0);
            F->c[g].assign((size_t)(int64_t(1) << (g + 2)) * 2 * M, 0.0);
        }
    }
    return F;
}

/* out[0:n] = the transform of in[0:n] (host arrays). */
int cpu_fmm_execute(void *plan, const double *in, double *out)
{
    if (!plan || !in || !out) return -1;
    execute(*static_cast<Fmm *>(plan), in, out);
    return 0;
}

/* info[0..2] = L, s, N. */
int cpu_fmm_info(void *plan, int64_t *info)
{
    if (!plan || !info) return -1;
    const Fmm *F = static_cast<const Fmm *>(plan);
    info[0] = F->L;
    info[1] = F->s;
    info[2] = F->N;
    return 0;
}

void cpu_fmm_destroy(void *plan) { delete static_cast<Fmm *>(plan); }

}  // extern "C"
