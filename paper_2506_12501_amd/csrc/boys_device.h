// boys_device.h -- Boys function F_m(x) = int_0^1 y^{2m} exp(-x y^2) dy on gfx950.
//
// Sec. 3.2.1 of the paper evaluates F_m by upward recursion, an asymptotic
// form and Chebyshev interpolation on CPUs, and notes that downward recursion
// may suit GPUs better.  Here:
//   x <  45: F_M(x) from a 10-term Taylor series about the nearest node of a
//            1/8-spaced table (dF_m/dx = -F_{m+1}; truncation below
//            (1/16)^10/10! relative), then the downward recursion
//            F_m = (2x F_{m+1} + e^{-x}) / (2m+1): one exp, no cancellation.
//   x >= 45: F_0 = sqrt(pi/(4x)) (erf(sqrt x) = 1 to double precision) and the
//            upward recursion F_{m+1} = ((2m+1) F_m - e^{-x}) / (2x), which
//            keeps e^{-x}; (2m+1)/(2x) < 1 for every m <= 32, so it is stable.
#pragma once

#include "mdx_internal.h"

namespace mdx {

template <int M>
__device__ __forceinline__ void boys_eval(double x, double *__restrict__ F, const double *__restrict__ tab)
{
    static_assert(M >= 0 && M <= BOYS_MMAX, "Boys order out of range");
    if (x < (double)BOYS_XMAX) {
        const int k = __double2int_rn(x * (double)BOYS_STEP_INV);
        const double d = (double)k * (1.0 / BOYS_STEP_INV) - x;   // node minus x
        const double *row = tab + k * BOYS_NCOL + M;
        double f = row[BOYS_NTERM - 1];
#pragma unroll
        for (int i = BOYS_NTERM - 2; i >= 0; --i) f = fma(f, d * (1.0 / (i + 1)), row[i]);
        F[M] = f;
        const double e = exp(-x);
        const double x2 = x + x;
#pragma unroll
        for (int m = M - 1; m >= 0; --m) F[m] = fma(x2, F[m + 1], e) * (1.0 / (2 * m + 1));
    } else {
        const double rx = 1.0 / x;
        F[0] = sqrt(0.78539816339744830962 * rx);   // pi/4
        if (M > 0) {
            const double e = exp(-x);
            const double hrx = 0.5 * rx;
#pragma unroll
            for (int m = 0; m < M; ++m) F[m + 1] = fma((double)(2 * m + 1), F[m], -e) * hrx;
        }
    }
}

}  // namespace mdx
