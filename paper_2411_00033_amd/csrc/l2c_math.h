// l2c_math.h -- device evaluation of Lambda(z) = Gamma(z+1/2)/Gamma(z+1) (Eq. (Lambda)).
//
// For z >= 20 the expansion of Eq. (tau) (Sec. 4.3) is used per element:
//     Lambda(z) = tau(x)/sqrt(x),  x = z + 1/4,
//     tau(x) ~ 1 - 1/(2^6 x^2) + 21/(2^13 x^4) - 671/(2^19 x^6) + 180323/(2^27 x^8),
// which is accurate to about one FP64 ulp once z > 19.88.  Evaluating it
// independently for every index replaces the paper's sequential recursion
// (Eq. (Lambdaint)) and its periodic resynchronisation, so every thread can
// produce its own lambda values.
// For integer z < 20, Lambda(k) = sqrt(pi) binom(2k,k) / 4^k, whose rational
// factor is exact in FP64 for k <= 28.
// For real z < 20 the argument is shifted up with Lambda(z) = Lambda(z+1)(z+1)/(z+1/2).
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace l2c {

constexpr double kSqrtPi = 1.7724538509055160272981674833411452;
constexpr double kPi = 3.1415926535897932384626433832795029;

__host__ __device__ inline double tau_series(double x)
{
    const double t = 1.0 / (x * x);
    double p = 180323.0 / 134217728.0;
    p = p * t - 671.0 / 524288.0;
    p = p * t + 21.0 / 8192.0;
    p = p * t - 1.0 / 64.0;
    return p * t + 1.0;
}

// Lambda(k) for integer k >= 0.
__host__ __device__ inline double lambda_int(int64_t k)
{
    if (k < 20) {
        double c = 1.0;  // binom(2k, k), exact: every partial product is an integer < 2^53
        for (int i = 1; i <= (int)k; ++i) c = c * (double)(k + i) / (double)i;
        return kSqrtPi * (c * ldexp(1.0, -2 * (int)k));
    }
    const double x = (double)k + 0.25;
    return tau_series(x) / sqrt(x);
}

// 1 / Lambda(k), k >= 0.
__host__ __device__ inline double inv_lambda_int(int64_t k)
{
    if (k < 20) return 1.0 / lambda_int(k);
    const double x = (double)k + 0.25;
    return sqrt(x) / tau_series(x);
}

// Lambda(z) for real z > 0.
__host__ __device__ inline double lambda_real(double z)
{
    double num = 1.0, den = 1.0;
    while (z < 20.0) {
        num *= z + 1.0;
        den *= z + 0.5;
        z += 1.0;
    }
    const double x = z + 0.25;
    return tau_series(x) / sqrt(x) * (num / den);
}

}  // namespace l2c
