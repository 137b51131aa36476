// util.hip -- small helper kernels: Schwarz factors from diagonal shellsets,
// and an int fill (used instead of a memset so that it can sit in a graph).
#include "kernels.h"

namespace mdx {

// Q[i] = sqrt(max_ab |(ab|ab)|) from the diagonal blocks diag[i][cd][ab]
// (nab x nab, column-major) of pair i
__global__ void __launch_bounds__(256) schwarz_kernel(const double *diag, int npair, int nab, double *Q)
{
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= npair) return;
    const double *d = diag + (int64_t)i * nab * nab;
    double m = 0.0;
    for (int ab = 0; ab < nab; ++ab) m = fmax(m, fabs(d[ab + nab * ab]));
    Q[i] = sqrt(m);
}

__global__ void __launch_bounds__(256) fill_i32_kernel(int32_t *p, int n, int32_t v)
{
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) p[i] = v;
}

void launch_schwarz(const double *diag, int npair, int nab, double *Q, hipStream_t s)
{
    if (npair > 0) hipLaunchKernelGGL(schwarz_kernel, dim3((npair + 255) / 256), dim3(256), 0, s, diag, npair, nab, Q);
}

void launch_fill_i32(int32_t *p, int n, int32_t v, hipStream_t s)
{
    if (n > 0) hipLaunchKernelGGL(fill_i32_kernel, dim3((n + 255) / 256), dim3(256), 0, s, p, n, v);
}

}  // namespace mdx
