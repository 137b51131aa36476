// boys.hip -- mdx_boys: F_m(x), m = 0..mmax, for an array of arguments.
// One lane per argument, through boys_eval (the evaluation every integral
// kernel uses), instantiated per order.
#include <utility>

#include "boys_device.h"
#include "kernels.h"

namespace mdx {

template <int M>
__global__ void __launch_bounds__(256) boys_kernel(const double *__restrict__ x, int n, double *__restrict__ F,
                                                   const double *__restrict__ tab)
{
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    double f[M + 1];
    boys_eval<M>(x[i], f, tab);
#pragma unroll
    for (int m = 0; m <= M; ++m) F[(int64_t)m * n + i] = f[m];
}

template <int M>
static void launch_boys_order(int mmax, const double *x, int n, double *F, const double *tab, hipStream_t s)
{
    if (mmax == M) hipLaunchKernelGGL(boys_kernel<M>, dim3((n + 255) / 256), dim3(256), 0, s, x, n, F, tab);
}

template <int... Ms>
static void launch_boys_m(int mmax, const double *x, int n, double *F, const double *tab, hipStream_t s,
                          std::integer_sequence<int, Ms...>)
{
    (launch_boys_order<Ms>(mmax, x, n, F, tab, s), ...);
}

void launch_boys(const double *x, int n, int mmax, double *F, const double *tab, hipStream_t s)
{
    if (n <= 0) return;
    launch_boys_m(mmax, x, n, F, tab, s, std::make_integer_sequence<int, BOYS_MMAX + 1>{});
}

}  // namespace mdx
