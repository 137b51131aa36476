// boys_device.h -- Boys function F_m(x) = int_0^1 y^{2m} exp(-x y^2) dy on gfx950.
//
// Sec. 3.2.1 of the paper evaluates F_m by upward recursion, an asymptotic
// form and Chebyshev interpolation on CPUs, and notes that downward recursion
// may suit GPUs better.  Here:
//   x <  45: F_M(x) from a 10-term Taylor series about the nearest node of a
//            1/8-spaced table (dF_m/dx = -F_{m+1}; truncation below
//            (1/16)^10/10! relative), then the downward recursion
//            F_m = (2x F_{m+1} + e^{-x}) / (2m+1): no cancellation.
//   x >= 45: F_0 = sqrt(pi/(4x)) (erf(sqrt x) = 1 to double precision) and the
//            upward recursion F_{m+1} = ((2m+1) F_m - e^{-x}) / (2x), which
//            keeps e^{-x}; (2m+1)/(2x) < 1 for every m <= 32, so it is stable.
// e^{-x} of the downward branch comes from the node value and a short series
// (boys_exp); reciprocal square roots from the hardware estimate and Newton
// steps (rsqrt_d).
#pragma once

#include "kernels.h"
#include "mdx_internal.h"

namespace mdx {

// e^{-x} for 0 <= x < BOYS_XMAX from the node value e^{-x_k} and e^{d},
// d = x_k - x in [-1/16, 1/16], by its Taylor series to d^9 (remainder below
// 3e-19): a table read and nine fused multiply-adds instead of a full exp
__device__ __forceinline__ double boys_exp(int k, double d, const double *__restrict__ tab)
{
    double e = 2.7557319223985893e-06;   // 1/9!
    e = fma(e, d, 2.4801587301587302e-05);
    e = fma(e, d, 1.9841269841269841e-04);
    e = fma(e, d, 1.3888888888888889e-03);
    e = fma(e, d, 8.3333333333333333e-03);
    e = fma(e, d, 4.1666666666666667e-02);
    e = fma(e, d, 1.6666666666666667e-01);
    e = fma(e, d, 0.5);
    e = fma(e, d, 1.0);
    e = fma(e, d, 1.0);
    return tab[BOYS_EXP_OFF + k] * e;
}

// TEXP: e^{-x} of the downward branch from the table (boys_exp) rather than
// exp(); the table read adds a dependent load, which lanes that evaluate one
// quartet between other work (the matrix-core kernels) feel more than lanes
// that stream quartets (the register kernels)
template <int M, bool TEXP = true>
__device__ __forceinline__ void boys_eval(double x, double *__restrict__ F, const double *__restrict__ tab)
{
    static_assert(M >= 0 && M <= BOYS_MMAX, "Boys order out of range");
    if (x < (double)BOYS_XMAX) {
        const int k = __double2int_rn(x * (double)BOYS_STEP_INV);
        const double d = (double)k * (1.0 / BOYS_STEP_INV) - x;   // node minus x
        const double *row = tab + k * BOYS_NCOL + M;
        double f = row[BOYS_NTERM - 1];
#pragma unroll
        for (int i = BOYS_NTERM - 2; i >= 0; --i) f = fma(f * (1.0 / (i + 1)), d, row[i]);   // no d/(i+1) registers
        F[M] = f;
        if constexpr (M > 0) {
            const double e = TEXP ? boys_exp(k, d, tab) : exp(-x);
            const double x2 = x + x;
#pragma unroll
            for (int m = M - 1; m >= 0; --m) F[m] = fma(x2, F[m + 1], e) * (1.0 / (2 * m + 1));
        }
    } else {
        const double y = rsqrt_d(x);
        F[0] = 0.88622692545275801365 * y;   // sqrt(pi/4) / sqrt(x)
        if constexpr (M > 0) {
            const double e = exp(-x);
            const double hrx = 0.5 * rcp_d(x);   // (y*y would carry ~3 ulp into every upward step)
#pragma unroll
            for (int m = 0; m < M; ++m) F[m + 1] = fma((double)(2 * m + 1), F[m], -e) * hrx;
        }
    }
}

}  // namespace mdx
