// boys.hip -- mdx_boys: F_m(x), m = 0..mmax, for an array of arguments.
// One lane per argument; the order mmax is a run-time value here, so the
// lane walks the downward (or upward) recursion and stores as it goes.
#include "boys_device.h"
#include "kernels.h"

namespace mdx {

__global__ void __launch_bounds__(256) boys_kernel(const double *__restrict__ x, int n, int mmax,
                                                   double *__restrict__ F, const double *__restrict__ tab)
{
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    const double xi = x[i];
    if (xi < (double)BOYS_XMAX) {
        const int k = __double2int_rn(xi * (double)BOYS_STEP_INV);
        const double d = (double)k * (1.0 / BOYS_STEP_INV) - xi;
        const double *row = tab + k * BOYS_NCOL + mmax;
        double f = row[BOYS_NTERM - 1];
#pragma unroll
        for (int j = BOYS_NTERM - 2; j >= 0; --j) f = fma(f, d * (1.0 / (j + 1)), row[j]);
        F[(int64_t)mmax * n + i] = f;
        const double e = exp(-xi);
        const double x2 = xi + xi;
        for (int m = mmax - 1; m >= 0; --m) {
            f = fma(x2, f, e) / (double)(2 * m + 1);
            F[(int64_t)m * n + i] = f;
        }
    } else {
        const double rx = 1.0 / xi;
        double f = sqrt(0.78539816339744830962 * rx);
        F[i] = f;
        const double e = exp(-xi);
        const double hrx = 0.5 * rx;
        for (int m = 0; m < mmax; ++m) {
            f = fma((double)(2 * m + 1), f, -e) * hrx;
            F[(int64_t)(m + 1) * n + i] = f;
        }
    }
}

void launch_boys(const double *x, int n, int mmax, double *F, const double *tab, hipStream_t s)
{
    if (n <= 0) return;
    hipLaunchKernelGGL(boys_kernel, dim3((n + 255) / 256), dim3(256), 0, s, x, n, mmax, F, tab);
}

}  // namespace mdx
