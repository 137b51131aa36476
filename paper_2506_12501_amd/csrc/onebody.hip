// onebody.hip -- overlap and kinetic-energy integrals of batches of shell
// pairs (the 1-particle set; Sec. 2.1 with Eq. (8)).
//
// One shell pair per lane, as the paper assigns one contracted pair to one
// SIMD lane.  Per primitive pair and Cartesian axis the lane builds the 1-D
// Hermite coefficients E^{ij}_t by the recursion of Eqs. (10)-(11) (with the
// Gaussian factor of Eq. (14) taken once for all three axes), keeps the
// t = 0 column, and forms
//   overlap  s_ij = E^{ij}_0 (times (pi/p)^{1/2}, Eq. (8)),
//   kinetic  t_ij = -1/2 [ j(j-1) s_{i,j-2} - 2 zeta_b (2j+1) s_ij + 4 zeta_b^2 s_{i,j+2} ]
// (the Laplacian acting on the ket Gaussian), then
//   S_ab = sum_prims c_a c_b s_x s_y s_z,  T_ab = sum_prims c_a c_b (t_x s_y s_z + s_x t_y s_z + s_x s_y t_z),
// and transforms both to real solid harmonics (Eq. (18)) unless Cartesian
// components were asked for.
#include "runtime.h"

namespace mdx {

static inline size_t al256(size_t x) { return (x + 255) & ~size_t(255); }

struct OneBodyArgs {
    const PairRec *pairs;
    int npair;
    const double *center, *expo, *coef;
    const double *Ca, *Cb;   // solid coefficients [nsph][ncart] (spherical only)
    double *S, *T;           // [ij + npair*ab] or null
};

// (x, y, z) exponents of Cartesian component idx of angular momentum l, in
// the order (l,0,0), (l-1,1,0), (l-1,0,1), (l-2,2,0), ...
__host__ __device__ constexpr int cart_exp(int l, int idx, int axis)
{
    int s = 0;
    while ((s + 1) * (s + 2) / 2 <= idx) ++s;
    const int z = idx - s * (s + 1) / 2, y = s - z, x = l - s;
    return axis == 0 ? x : (axis == 1 ? y : z);
}

// E^{ij}_0 for i <= LA, j <= LBP along one axis, Eqs. (10)-(11), with
// E^{00}_0 = 1 (the Gaussian factor is applied by the caller)
template <int LA, int LBP>
__device__ __forceinline__ void e0_axis(double p, double XPA, double XPB, double (&E0)[LA + 1][LBP + 1])
{
    constexpr int TM = LA + LBP + 1;
    const double i2p = 0.5 / p;
    double E[LA + 1][LBP + 1][TM];
    auto get = [&](int i, int j, int t) -> double { return (t < 0 || t > i + j) ? 0.0 : E[i][j][t]; };
#pragma unroll
    for (int i = 0; i <= LA; ++i) {
        if (i == 0) {
            E[0][0][0] = 1.0;
        } else {
#pragma unroll
            for (int t = 0; t <= i; ++t)
                E[i][0][t] = i2p * get(i - 1, 0, t - 1) + XPA * get(i - 1, 0, t) + (t + 1) * get(i - 1, 0, t + 1);
        }
#pragma unroll
        for (int j = 1; j <= LBP; ++j)
#pragma unroll
            for (int t = 0; t <= i + j; ++t)
                E[i][j][t] = i2p * get(i, j - 1, t - 1) + XPB * get(i, j - 1, t) + (t + 1) * get(i, j - 1, t + 1);
#pragma unroll
        for (int j = 0; j <= LBP; ++j) E0[i][j] = E[i][j][0];
    }
}

template <int LA, int LB, bool CART>
__global__ void __launch_bounds__(64) onebody_kernel(OneBodyArgs a)
{
    const int ij = blockIdx.x * 64 + (int)threadIdx.x;
    if (ij >= a.npair) return;
    constexpr int NA = ncart(LA), NB = ncart(LB);
    const PairRec pr = a.pairs[ij];
    const double A[3] = {a.center[3 * pr.sa], a.center[3 * pr.sa + 1], a.center[3 * pr.sa + 2]};
    const double B[3] = {a.center[3 * pr.sb], a.center[3 * pr.sb + 1], a.center[3 * pr.sb + 2]};
    const double AB2 = (A[0] - B[0]) * (A[0] - B[0]) + (A[1] - B[1]) * (A[1] - B[1]) + (A[2] - B[2]) * (A[2] - B[2]);
    double S[NA][NB], T[NA][NB];
#pragma unroll
    for (int i = 0; i < NA; ++i)
#pragma unroll
        for (int j = 0; j < NB; ++j) S[i][j] = T[i][j] = 0.0;

    for (int ka = 0; ka < pr.ka; ++ka) {
        const double za = a.expo[pr.offa + ka], ca = a.coef[pr.offa + ka];
        for (int kb = 0; kb < pr.kb; ++kb) {
            const double zb = a.expo[pr.offb + kb], cb = a.coef[pr.offb + kb];
            const double p = za + zb;
            double E0[3][LA + 1][LB + 3];
#pragma unroll
            for (int ax = 0; ax < 3; ++ax) {
                const double P = (za * A[ax] + zb * B[ax]) / p;
                e0_axis<LA, LB + 2>(p, P - A[ax], P - B[ax], E0[ax]);
            }
            // c_a c_b (pi/p)^{3/2} exp(-za zb/p |A-B|^2), Eqs. (8), (14)
            const double f = ca * cb * (M_PI / p) * sqrt(M_PI / p) * exp(-za * zb / p * AB2);
#pragma unroll
            for (int i = 0; i < NA; ++i)
#pragma unroll
                for (int j = 0; j < NB; ++j) {
                    double s[3], t[3];
#pragma unroll
                    for (int ax = 0; ax < 3; ++ax) {
                        const int ia = cart_exp(LA, i, ax), jb = cart_exp(LB, j, ax);
                        s[ax] = E0[ax][ia][jb];
                        double d2 = 4.0 * zb * zb * E0[ax][ia][jb + 2] - 2.0 * zb * (2 * jb + 1) * s[ax];
                        if (jb >= 2) d2 += (double)(jb * (jb - 1)) * E0[ax][ia][jb - 2];
                        t[ax] = -0.5 * d2;
                    }
                    S[i][j] = fma(f, s[0] * s[1] * s[2], S[i][j]);
                    T[i][j] = fma(f, t[0] * s[1] * s[2] + s[0] * t[1] * s[2] + s[0] * s[1] * t[2], T[i][j]);
                }
        }
    }
    if constexpr (CART) {
#pragma unroll
        for (int i = 0; i < NA; ++i)
#pragma unroll
            for (int j = 0; j < NB; ++j) {
                const int64_t o = ij + (int64_t)a.npair * (i * NB + j);
                if (a.S) a.S[o] = S[i][j];
                if (a.T) a.T[o] = T[i][j];
            }
    } else {
        constexpr int MA = 2 * LA + 1, MB = 2 * LB + 1;
#pragma unroll
        for (int m = 0; m < MA; ++m)
#pragma unroll
            for (int n = 0; n < MB; ++n) {
                double vs = 0.0, vt = 0.0;
#pragma unroll
                for (int i = 0; i < NA; ++i) {
                    double us = 0.0, ut = 0.0;
#pragma unroll
                    for (int j = 0; j < NB; ++j) {
                        const double cbj = a.Cb[n * NB + j];
                        us = fma(cbj, S[i][j], us);
                        ut = fma(cbj, T[i][j], ut);
                    }
                    const double cai = a.Ca[m * NA + i];
                    vs = fma(cai, us, vs);
                    vt = fma(cai, ut, vt);
                }
                const int64_t o = ij + (int64_t)a.npair * (m * MB + n);
                if (a.S) a.S[o] = vs;
                if (a.T) a.T[o] = vt;
            }
    }
}

template <int LA, int LB>
static void launch_onebody(const OneBodyArgs &a, bool cart, hipStream_t s)
{
    const int nblk = (a.npair + 63) / 64;
    if (cart) hipLaunchKernelGGL((onebody_kernel<LA, LB, true>), dim3(nblk), dim3(64), 0, s, a);
    else hipLaunchKernelGGL((onebody_kernel<LA, LB, false>), dim3(nblk), dim3(64), 0, s, a);
}

// validation shared by the size query and the call; l = (l_a, l_b)
static mdx_status check_pairs(mdx_ctx *c, const mdx_shells *sh, int32_t npair, const int32_t *pairs, int flags,
                              int l[2])
{
    l[0] = l[1] = -1;
    if (!c) return fail(MDX_EINVAL, "null context");
    if (!sh) return fail(MDX_EINVAL, "null shell table");
    if (npair < 0) return fail(MDX_EINVAL, "negative pair count");
    if (npair > 0 && !pairs) return fail(MDX_EINVAL, "null pair list");
    if (flags & ~MDX_CARTESIAN) return fail(MDX_EINVAL, "unknown flags 0x%x", flags);
    if (sh->nshell < 0 || (sh->nshell > 0 && (!sh->l || !sh->nprim || !sh->prim_offset || !sh->center ||
                                               !sh->exponent || !sh->coef)))
        return fail(MDX_EINVAL, "incomplete shell table");
    for (int32_t i = 0; i < npair; ++i)
        for (int k = 0; k < 2; ++k) {
            const int32_t s = pairs[2 * i + k];
            if (s < 0 || s >= sh->nshell || sh->nprim[s] < 1)
                return fail(MDX_EINVAL, "pair %d: bad shell index %d or nprim < 1", i, s);
            if (i == 0) l[k] = sh->l[s];
            else if (sh->l[s] != l[k]) return fail(MDX_EINVAL, "pair %d: class differs from pair 0", i);
        }
    if (npair > 0 && (l[0] < 0 || l[1] < 0 || l[0] > 2 || l[1] > 2))
        return fail(MDX_EUNSUPPORTED, "one-body integrals for l_a = %d, l_b = %d (compiled for l <= 2)", l[0], l[1]);
    return MDX_OK;
}

}  // namespace mdx

using namespace mdx;

extern "C" size_t mdx_one_body_workspace_size(mdx_ctx *c, const mdx_shells *sh, int32_t npair, const int32_t *pairs,
                                              int flags)
{
    int l[2];
    if (check_pairs(c, sh, npair, pairs, flags, l) != MDX_OK) return 0;
    return al256((size_t)npair * sizeof(PairRec)) + 256;
}

extern "C" mdx_status mdx_one_body_batch(mdx_ctx *c, const mdx_shells *sh, int32_t npair, const int32_t *pairs,
                                         int flags, double *S, double *T, void *ws, size_t ws_bytes,
                                         mdx_stream_t stream)
{
    int l[2];
    mdx_status st = check_pairs(c, sh, npair, pairs, flags, l);
    if (st != MDX_OK) return st;
    if (npair == 0 || (!S && !T)) return MDX_OK;
    if (!ws) return fail(MDX_EINVAL, "mdx_one_body_batch: null workspace");
    if ((uintptr_t)ws & 255) return fail(MDX_EINVAL, "mdx_one_body_batch: workspace not 256-byte aligned");
    const size_t need = al256((size_t)npair * sizeof(PairRec));
    if (ws_bytes < need) return fail(MDX_EWORKSPACE, "workspace %zu bytes < %zu required", ws_bytes, need);
    std::vector<PairRec> pr((size_t)npair);
    for (int32_t i = 0; i < npair; ++i) {
        const int32_t sa = pairs[2 * i], sb = pairs[2 * i + 1];
        pr[i] = PairRec{sa, sb, sh->nprim[sa], sh->nprim[sb], sh->prim_offset[sa], sh->prim_offset[sb]};
    }
    HIP_TRY2(hipSetDevice(c->device));
    hipStream_t s = (hipStream_t)stream;
    HIP_TRY2(hipMemcpyAsync(ws, pr.data(), pr.size() * sizeof(PairRec), hipMemcpyHostToDevice, s));
    const bool cart = (flags & MDX_CARTESIAN) != 0;
    OneBodyArgs a{};
    a.pairs = (const PairRec *)ws;
    a.npair = npair;
    a.center = sh->center;
    a.expo = sh->exponent;
    a.coef = sh->coef;
    a.Ca = c->solid + c->solid_off[l[0]];
    a.Cb = c->solid + c->solid_off[l[1]];
    a.S = S;
    a.T = T;
    hipEvent_t ev1 = nullptr;
    if (c->prof_events.size() >= 2) {   // profiling hook, as for the other integral kernels
        const size_t np = c->prof_events.size() / 2, i = c->prof_count++ % np;
        ev1 = c->prof_events[2 * i + 1];
        HIP_TRY2(hipEventRecord(c->prof_events[2 * i], s));
    }
    switch (l[0] * 3 + l[1]) {
    case 0: launch_onebody<0, 0>(a, cart, s); break;
    case 1: launch_onebody<0, 1>(a, cart, s); break;
    case 2: launch_onebody<0, 2>(a, cart, s); break;
    case 3: launch_onebody<1, 0>(a, cart, s); break;
    case 4: launch_onebody<1, 1>(a, cart, s); break;
    case 5: launch_onebody<1, 2>(a, cart, s); break;
    case 6: launch_onebody<2, 0>(a, cart, s); break;
    case 7: launch_onebody<2, 1>(a, cart, s); break;
    default: launch_onebody<2, 2>(a, cart, s); break;
    }
    HIP_TRY2(hipGetLastError());
    if (ev1) HIP_TRY2(hipEventRecord(ev1, s));
    return MDX_OK;
}
