/*
 * oracle.c -- direct O(N^2) CPU reference for the Legendre <-> Chebyshev
 * coefficient transforms of Mortensen, "A faster multipole Legendre-Chebyshev
 * transform" (arXiv 2411.00033).
 *
 * TEST INFRASTRUCTURE ONLY.  Nothing in the product path links, loads or calls
 * this file.  Only the test suite, the smoke check and the CPU-baseline leg of
 * the benchmark use it.  It shares no code, table or constant generator with
 * the GPU library.
 *
 * What it computes (plain definitions, no blocking or approximation):
 *
 *   Sec. 1, Eqs. (AfCf), (directmv):   A f_leg = C f_cheb,  C = diag(c_i pi/2),
 *                                       c_0 = 2, c_i = 1 for i > 0.
 *   Eqs. (aij), (hik):                  a_{i,i+2k} = lambda_k lambda_{i+k};
 *                                       every other entry of A is zero.
 *   Eq. (Lambda):                       lambda_k = Gamma(k+1/2) / Gamma(k+1).
 *
 *   leg2cheb :  z = C^{-1} A f          (the sum of Alg. 1, DIRECTL2C)
 *   cheb2leg :  z = A^{-1} C f, written with the reverse kernel of
 *               Eq. (Lxymod) (Sec. 4.3):  z = K (c .* f), where for j > i,
 *               j - i even,
 *                   K_ij = 2(i+1/2) j / ((i+j)(i+j+1)(i-j+1))
 *                          * lambda_{(j-i)/2} / lambda_{(i+j)/2},
 *               and on the diagonal K_ii = (pi/2) / a_ii = sqrt(pi)/(2 lambda_i)
 *               (the kernel is 0/0 at i = j = 0; its limit there is 1/2).
 *               Because K already holds the pi/2 of C, only the c_i factor of
 *               C is applied to the input ("apply C first", Sec. 4.1).
 *   cheb2leg_backsub : an independent second route for cheb2leg, solving the
 *               upper-triangular system A z = C f by back substitution.
 *
 * Precision.  The paper's own reference is a ~32-digit direct solver (Sec. 5.1).
 * Here lambda is carried in x87 long double (64-bit mantissa) through the
 * recursion of Eq. (Lambdaint), lambda_k = lambda_{k-1} (k - 1/2)/k, from
 * lambda_0 = sqrt(pi); the products are formed in long double and every output
 * is a Neumaier-compensated long-double sum, rounded once to double.  The
 * result is within about one ulp of the exact product of the FP64 input.
 *
 * Threads: OpenMP over output rows, dynamic schedule (row i costs ~ (n-i)/2).
 */
#include <math.h>
#include <quadmath.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

#define SQRT_PI_L 1.772453850905516027298167483341145183L

/* lambda_k for k < n, by the recursion of Eq. (Lambdaint), in long double. */
static long double *lambda_table_ld(int64_t n)
{
    if (n < 1) n = 1;
    long double *lam = (long double *)malloc((size_t)n * sizeof(long double));
    if (!lam) return NULL;
    lam[0] = SQRT_PI_L;
    for (int64_t k = 1; k < n; ++k)
        lam[k] = lam[k - 1] * ((long double)k - 0.5L) / (long double)k;
    return lam;
}

/* Neumaier (improved Kahan-Babuska) compensated accumulation. */
typedef struct { long double s, c; } nsum_t;

static inline void nsum_add(nsum_t *a, long double x)
{
    long double t = a->s + x;
    if (fabsl(a->s) >= fabsl(x))
        a->c += (a->s - t) + x;
    else
        a->c += (x - t) + a->s;
    a->s = t;
}

static inline long double nsum_get(const nsum_t *a) { return a->s + a->c; }

int oracle_num_threads(void)
{
#ifdef _OPENMP
    return omp_get_max_threads();
#else
    return 1;
#endif
}

/* lambda_k, k < n, rounded to double. */
int oracle_lambda(int64_t n, double *out)
{
    if (n < 0 || (n > 0 && !out)) return -1;
    if (n == 0) return 0;
    long double *lam = lambda_table_ld(n);
    if (!lam) return -2;
    for (int64_t k = 0; k < n; ++k) out[k] = (double)lam[k];
    free(lam);
    return 0;
}

/* One output row of z = C^{-1} A f. */
static double l2c_row(int64_t n, const double *f, const long double *lam, int64_t i)
{
    nsum_t acc = {0.0L, 0.0L};
    for (int64_t k = 0; i + 2 * k < n; ++k) {
        long double a_ij = lam[k] * lam[i + k];          /* a_{i,i+2k}, Eq. (hik) */
        nsum_add(&acc, a_ij * (long double)f[i + 2 * k]);
    }
    long double ci = (i == 0) ? 2.0L : 1.0L;
    /* pi/2 * c_i, with pi = lambda_0^2 */
    return (double)(nsum_get(&acc) / (ci * SQRT_PI_L * SQRT_PI_L * 0.5L));
}

/*
 * z[r] = (C^{-1} A f)_{rows[r]} for r < nrows; rows == NULL means all n rows
 * (then nrows is ignored and z has n entries).
 */
int oracle_leg2cheb(int64_t n, const double *f, int64_t nrows, const int64_t *rows, double *z)
{
    if (n < 1 || !f || !z) return -1;
    int64_t m = rows ? nrows : n;
    if (m < 0) return -1;
    for (int64_t r = 0; rows && r < m; ++r)
        if (rows[r] < 0 || rows[r] >= n) return -1;
    long double *lam = lambda_table_ld(n);
    if (!lam) return -2;
#pragma omp parallel for schedule(dynamic, 16)
    for (int64_t r = 0; r < m; ++r) {
        int64_t i = rows ? rows[r] : r;
        z[r] = l2c_row(n, f, lam, i);
    }
    free(lam);
    return 0;
}

/* K_ij of cheb2leg, j >= i, j - i even (see header). */
static inline long double c2l_entry(const long double *lam, int64_t i, int64_t j)
{
    if (j == i) return SQRT_PI_L / (2.0L * lam[i]);
    long double x = (long double)i, y = (long double)j;
    long double g = 2.0L * (x + 0.5L) * y / ((x + y) * (x + y + 1.0L) * (x - y + 1.0L));
    return g * lam[(j - i) / 2] / lam[(i + j) / 2];
}

static double c2l_row(int64_t n, const double *f, const long double *lam, int64_t i)
{
    nsum_t acc = {0.0L, 0.0L};
    for (int64_t j = i; j < n; j += 2) {
        long double u = (long double)f[j] * (j == 0 ? 2.0L : 1.0L);   /* u = c .* f */
        nsum_add(&acc, c2l_entry(lam, i, j) * u);
    }
    return (double)nsum_get(&acc);
}

/* z[r] = (A^{-1} C f)_{rows[r]} via the reverse kernel; rows == NULL: all rows. */
int oracle_cheb2leg(int64_t n, const double *f, int64_t nrows, const int64_t *rows, double *z)
{
    if (n < 1 || !f || !z) return -1;
    int64_t m = rows ? nrows : n;
    if (m < 0) return -1;
    for (int64_t r = 0; rows && r < m; ++r)
        if (rows[r] < 0 || rows[r] >= n) return -1;
    long double *lam = lambda_table_ld(n);
    if (!lam) return -2;
#pragma omp parallel for schedule(dynamic, 16)
    for (int64_t r = 0; r < m; ++r) {
        int64_t i = rows ? rows[r] : r;
        z[r] = c2l_row(n, f, lam, i);
    }
    free(lam);
    return 0;
}

/*
 * Second, independent cheb2leg route: solve A z = C f (Eq. (AfCf)) by back
 * substitution on the upper-triangular A of Eq. (hik).  Sequential, O(n^2/4).
 */
int oracle_cheb2leg_backsub(int64_t n, const double *f, double *z)
{
    if (n < 1 || !f || !z) return -1;
    long double *lam = lambda_table_ld(n);
    long double *zl = (long double *)malloc((size_t)n * sizeof(long double));
    if (!lam || !zl) { free(lam); free(zl); return -2; }
    const long double half_pi = SQRT_PI_L * SQRT_PI_L * 0.5L;
    for (int64_t i = n - 1; i >= 0; --i) {
        nsum_t acc = {0.0L, 0.0L};
        nsum_add(&acc, (i == 0 ? 2.0L : 1.0L) * half_pi * (long double)f[i]);
        for (int64_t k = 1; i + 2 * k < n; ++k)
            nsum_add(&acc, -(lam[k] * lam[i + k]) * zl[i + 2 * k]);
        zl[i] = nsum_get(&acc) / (lam[0] * lam[i]);
    }
    for (int64_t i = 0; i < n; ++i) z[i] = (double)zl[i];
    free(lam);
    free(zl);
    return 0;
}

/*
 * ---- The grid pipeline of Sec. 1 (Chebyshev-Gauss points x_j = cos(pi (2j+1) / (2n))).
 *
 *   oracle_dct, kind 2:  y_k = sum_{j<n} x_j cos(pi k (2j+1) / (2n))
 *               kind 3:  y_j = sum_{k<n} x_k cos(pi k (2j+1) / (2n))
 *   oracle_legval_cg:    u_j = sum_{k<n} f_k P_k(x_j), the Legendre polynomials from the
 *                        three-term recurrence (k+1) P_{k+1}(x) = (2k+1) x P_k(x) - k P_{k-1}(x),
 *                        P_0 = 1, P_1 = x, in binary128 (see there).
 * The DCTs' cosine argument pi k (2j+1) / (2n) = 2 pi m / (4n) is reduced exactly in
 * integers, m = k (2j+1) mod 4n, before cosl, with Neumaier-compensated long-double sums,
 * rounded once to double.  Rows as in oracle_leg2cheb (rows == NULL: all n).
 */
#define PI_L 3.141592653589793238462643383279502884L

static inline long double cos_frac(int64_t m, int64_t den)   /* cos(2 pi m / den) */
{
    return cosl(2.0L * PI_L * (long double)m / (long double)den);
}

int oracle_dct(int64_t n, const double *x, int kind, int64_t nrows, const int64_t *rows, double *y)
{
    if (n < 1 || !x || !y || (kind != 2 && kind != 3)) return -1;
    int64_t m = rows ? nrows : n;
    if (m < 0) return -1;
    for (int64_t r = 0; rows && r < m; ++r)
        if (rows[r] < 0 || rows[r] >= n) return -1;
#pragma omp parallel for schedule(static)
    for (int64_t r = 0; r < m; ++r) {
        const int64_t out = rows ? rows[r] : r;
        nsum_t acc = {0.0L, 0.0L};
        for (int64_t t = 0; t < n; ++t) {
            /* kind 2: out = k, t = j;  kind 3: out = j, t = k */
            const int64_t k = kind == 2 ? out : t, j = kind == 2 ? t : out;
            const int64_t q = (k * (2 * j + 1)) % (4 * n);
            nsum_add(&acc, (long double)x[t] * cos_frac(q, 4 * n));
        }
        y[r] = (double)nsum_get(&acc);
    }
    return 0;
}

int oracle_legval_cg(int64_t n, const double *f, int64_t nrows, const int64_t *rows, double *u)
{
    if (n < 1 || !f || !u) return -1;
    int64_t m = rows ? nrows : n;
    if (m < 0) return -1;
    for (int64_t r = 0; rows && r < m; ++r)
        if (rows[r] < 0 || rows[r] >= n) return -1;
    /* binary128: for large n the outer points lie within ~1/n^2 of +-1, where P_k moves
     * like k^2 / 2 per unit of x, so the point itself must carry ~30 digits (in long
     * double its rounding alone would shift P_k by up to ~k^2 5e-20, 3e-8 at k = 10^6). */
#pragma omp parallel for schedule(dynamic, 1)
    for (int64_t r = 0; r < m; ++r) {
        const int64_t j = rows ? rows[r] : r;
        const __float128 x = cosq(M_PIq * (__float128)(2 * j + 1) / (__float128)(2 * n));
        __float128 pm = 1, p = x, acc = (__float128)f[0];
        for (int64_t k = 1; k < n; ++k) {
            acc += (__float128)f[k] * p;
            const __float128 pn = ((__float128)(2 * k + 1) * x * p - (__float128)k * pm) / (__float128)(k + 1);
            pm = p;
            p = pn;
        }
        u[r] = (double)acc;
    }
    return 0;
}
