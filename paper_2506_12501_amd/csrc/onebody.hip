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
//
// The 1-particle Coulomb integrals of a set of point charges take the
// Hermite route of Eqs. (24), (26), (30), (34), with the sum over charges
// moved in front of the Hermite-to-AO transform (Eq. (37)): per primitive
// pair the lane accumulates sum_I q_I [r]_I^(0) over all charges -- Boys
// function and recursion per charge -- and only then contracts that one set
// of Hermite integrals with the pair's E coefficients.
#include <utility>

#include "eri_common.h"
#include "runtime.h"

namespace mdx {

static inline size_t al256(size_t x) { return (x + 255) & ~size_t(255); }

constexpr int ONEBODY_LMAX = 6;        // per shell, overlap / kinetic / nuclear attraction
constexpr int ONEBODY_LANE_LMAX = 3;   // one pair per lane up to here; beyond, one pair per wave
                                       // (overlap, kinetic; nuclear attraction by l_a + l_b instead)


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

// E^{ij}_t for i <= LA, j <= LB, 0 <= t <= i + j along one axis, Eqs.
// (10)-(11), with E^{00}_0 = 1 (the Gaussian factor is applied by the caller)
template <int LA, int LB>
__device__ __forceinline__ void e_axis(double i2p, double XPA, double XPB, double (&E)[LA + 1][LB + 1][LA + LB + 1])
{
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
        for (int j = 1; j <= LB; ++j)
#pragma unroll
            for (int t = 0; t <= i + j; ++t)
                E[i][j][t] = i2p * get(i, j - 1, t - 1) + XPB * get(i, j - 1, t) + (t + 1) * get(i, j - 1, t + 1);
    }
}

// the t = 0 column of e_axis (the 1-D overlaps of Eq. (8) up to (pi/p)^{1/2})
template <int LA, int LBP>
__device__ __forceinline__ void e0_axis(double p, double XPA, double XPB, double (&E0)[LA + 1][LBP + 1])
{
    double E[LA + 1][LBP + 1][LA + LBP + 1];
    e_axis<LA, LBP>(0.5 / p, XPA, XPB, E);
#pragma unroll
    for (int i = 0; i <= LA; ++i)
#pragma unroll
        for (int j = 0; j <= LBP; ++j) E0[i][j] = E[i][j][0];
}

// Cartesian values X[NA][NB] of one lane -> out[ij + npair*ab], solid
// (Eq. (18), factorised: ket index first) unless CART
template <int LA, int LB, bool CART>
__device__ __forceinline__ void store_pair(const double (&X)[ncart(LA)][ncart(LB)], const double *Ca,
                                           const double *Cb, double *out, int ij, int npair)
{
    constexpr int NA = ncart(LA), NB = ncart(LB);
    if constexpr (CART) {
#pragma unroll
        for (int i = 0; i < NA; ++i)
#pragma unroll
            for (int j = 0; j < NB; ++j) out[ij + (int64_t)npair * (i * NB + j)] = X[i][j];
    } else {
        constexpr int MA = 2 * LA + 1, MB = 2 * LB + 1;
        double U[NA][MB];
#pragma unroll
        for (int i = 0; i < NA; ++i)
#pragma unroll
            for (int n = 0; n < MB; ++n) {
                double u = 0.0;
#pragma unroll
                for (int j = 0; j < NB; ++j) u = fma(Cb[n * NB + j], X[i][j], u);
                U[i][n] = u;
            }
#pragma unroll
        for (int m = 0; m < MA; ++m)
#pragma unroll
            for (int n = 0; n < MB; ++n) {
                double v = 0.0;
#pragma unroll
                for (int i = 0; i < NA; ++i) v = fma(Ca[m * NA + i], U[i][n], v);
                out[ij + (int64_t)npair * (m * MB + n)] = v;
            }
    }
}

// PART: 0 = S and T together; 1 = S only; 2 = T only (large classes run the
// two as separate launches so that one lane holds one set of accumulators)
template <int LA, int LB, bool CART, int PART>
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
            // 1-D overlaps s1 and kinetic factors t1 per axis; each axis's E
            // table is reduced to them at once, so only one table is live
            double s1[3][LA + 1][LB + 1], t1[3][LA + 1][LB + 1];
#pragma unroll
            for (int ax = 0; ax < 3; ++ax) {
                // X_PA, X_PB from centre differences: exactly 0 on one centre
                double E0[LA + 1][LB + 3];
                e0_axis<LA, LB + 2>(p, zb / p * (B[ax] - A[ax]), za / p * (A[ax] - B[ax]), E0);
#pragma unroll
                for (int ia = 0; ia <= LA; ++ia)
#pragma unroll
                    for (int jb = 0; jb <= LB; ++jb) {
                        s1[ax][ia][jb] = E0[ia][jb];
                        double d2 = 4.0 * zb * zb * E0[ia][jb + 2] - 2.0 * zb * (2 * jb + 1) * E0[ia][jb];
                        if (jb >= 2) d2 += (double)(jb * (jb - 1)) * E0[ia][jb - 2];
                        t1[ax][ia][jb] = -0.5 * d2;
                    }
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
                        s[ax] = s1[ax][ia][jb];
                        t[ax] = t1[ax][ia][jb];
                    }
                    if constexpr (PART != 2) S[i][j] = fma(f, s[0] * s[1] * s[2], S[i][j]);
                    if constexpr (PART != 1)
                        T[i][j] = fma(f, t[0] * s[1] * s[2] + s[0] * t[1] * s[2] + s[0] * s[1] * t[2], T[i][j]);
                }
        }
    }
    if constexpr (PART != 2)
        if (a.S) store_pair<LA, LB, CART>(S, a.Ca, a.Cb, a.S, ij, a.npair);
    if constexpr (PART != 1)
        if (a.T) store_pair<LA, LB, CART>(T, a.Ca, a.Cb, a.T, ij, a.npair);
}

// Overlap and kinetic energy of shells beyond the lane kernels (l <= 6): one
// shell pair per wave.  Per primitive pair three lanes (one per axis) run the
// t = 0 column of Eqs. (10)-(11) in registers and write the 1-D overlap and
// kinetic factors to LDS; after one barrier every lane accumulates its share
// of the Cartesian function pairs.  The solid transform of Eq. (18) runs
// through LDS, ket index first.
template <int LA, int LB, bool CART>
__global__ void __launch_bounds__(64) onebody_wave_kernel(OneBodyArgs a)
{
    constexpr int NA = ncart(LA), NB = ncart(LB), NF = NA * NB, R = (NF + 63) / 64;
    constexpr int JB = LB + 3;   // kinetic needs j + 2
    constexpr int MA = CART ? NA : 2 * LA + 1, MB = CART ? NB : 2 * LB + 1;
    __shared__ double s1[3][LA + 1][LB + 1], t1[3][LA + 1][LB + 1];
    __shared__ double X[NF];
    __shared__ double U[NA * MB];
    const int ij = blockIdx.x, lane = (int)threadIdx.x;
    const PairRec pr = a.pairs[ij];
    const double A[3] = {a.center[3 * pr.sa], a.center[3 * pr.sa + 1], a.center[3 * pr.sa + 2]};
    const double B[3] = {a.center[3 * pr.sb], a.center[3 * pr.sb + 1], a.center[3 * pr.sb + 2]};
    const double AB2 = (A[0] - B[0]) * (A[0] - B[0]) + (A[1] - B[1]) * (A[1] - B[1]) + (A[2] - B[2]) * (A[2] - B[2]);
    int ex[R][3], ey[R][3];   // Cartesian exponents of this lane's function pairs (a in ex, b in ey)
#pragma unroll
    for (int r = 0; r < R; ++r) {
        const int e = min(lane + 64 * r, NF - 1), i = e / NB, j = e % NB;
#pragma unroll
        for (int ax = 0; ax < 3; ++ax) {
            ex[r][ax] = cart_exp(LA, i, ax);
            ey[r][ax] = cart_exp(LB, j, ax);
        }
    }
    double S[R], T[R];
#pragma unroll
    for (int r = 0; r < R; ++r) S[r] = T[r] = 0.0;
    for (int ka = 0; ka < pr.ka; ++ka) {
        const double za = a.expo[pr.offa + ka], ca = a.coef[pr.offa + ka];
        for (int kb = 0; kb < pr.kb; ++kb) {
            const double zb = a.expo[pr.offb + kb], cb = a.coef[pr.offb + kb];
            const double p = za + zb, i2p = 0.5 / p;
            __syncthreads();   // the previous primitive pair's readers are done
            if (lane < 3) {
                // lane = axis: the t = 0 column E^{ij}_0 of Eqs. (10)-(11), i <= l_a,
                // j <= l_b + 2, in registers.  With E^{ij}_1 = (i E^{i-1,j}_0 + j E^{i,j-1}_0)/(2p)
                // the recursion closes on t = 0:
                //   E^{i+1,j}_0 = X_PA E^{ij}_0 + (i E^{i-1,j}_0 + j E^{i,j-1}_0)/(2p), likewise for j.
                // X_PA, X_PB from centre differences: exactly 0 on one centre
                const double XPA = zb / p * (B[lane] - A[lane]), XPB = za / p * (A[lane] - B[lane]);
                double e0[LA + 1][JB];
#pragma unroll
                for (int i = 0; i <= LA; ++i) {
                    if (i == 0) e0[0][0] = 1.0;
                    else e0[i][0] = XPA * e0[i - 1][0] + (i >= 2 ? (i - 1) * i2p * e0[i - 2][0] : 0.0);
#pragma unroll
                    for (int j = 1; j < JB; ++j) {
                        double v = XPB * e0[i][j - 1];
                        if (i >= 1) v = fma(i * i2p, e0[i - 1][j - 1], v);
                        if (j >= 2) v = fma((j - 1) * i2p, e0[i][j - 2], v);
                        e0[i][j] = v;
                    }
                }
                // 1-D overlap and kinetic factors (the Laplacian on the ket Gaussian)
#pragma unroll
                for (int ia = 0; ia <= LA; ++ia)
#pragma unroll
                    for (int jb = 0; jb <= LB; ++jb) {
                        s1[lane][ia][jb] = e0[ia][jb];
                        double d2 = 4.0 * zb * zb * e0[ia][jb + 2] - 2.0 * zb * (2 * jb + 1) * e0[ia][jb];
                        if (jb >= 2) d2 += (double)(jb * (jb - 1)) * e0[ia][jb - 2];
                        t1[lane][ia][jb] = -0.5 * d2;
                    }
            }
            __syncthreads();
            // c_a c_b (pi/p)^{3/2} exp(-za zb/p |A-B|^2), Eqs. (8), (14)
            const double f = ca * cb * (M_PI / p) * sqrt(M_PI / p) * exp(-za * zb / p * AB2);
#pragma unroll
            for (int r = 0; r < R; ++r) {
                const double sx = s1[0][ex[r][0]][ey[r][0]], sy = s1[1][ex[r][1]][ey[r][1]], sz = s1[2][ex[r][2]][ey[r][2]];
                const double tx = t1[0][ex[r][0]][ey[r][0]], ty = t1[1][ex[r][1]][ey[r][1]], tz = t1[2][ex[r][2]][ey[r][2]];
                S[r] = fma(f, sx * sy * sz, S[r]);
                T[r] = fma(f, tx * sy * sz + sx * ty * sz + sx * sy * tz, T[r]);
            }
        }
    }
    for (int part = 0; part < 2; ++part) {
        double *out = part == 0 ? a.S : a.T;
        if (!out) continue;   // uniform
        const double *acc = part == 0 ? S : T;
        if constexpr (CART) {
#pragma unroll
            for (int r = 0; r < R; ++r) {
                const int e = lane + 64 * r;
                if (e < NF) out[ij + (int64_t)a.npair * e] = acc[r];
            }
        } else {
            __syncthreads();
#pragma unroll
            for (int r = 0; r < R; ++r) {
                const int e = lane + 64 * r;
                if (e < NF) X[e] = acc[r];
            }
            __syncthreads();
            for (int e = lane; e < NA * MB; e += 64) {   // U[i][n] = sum_j Cb[n][j] X[i][j]
                const int i = e / MB, n = e % MB;
                double u = 0.0;
                for (int j = 0; j < NB; ++j) u = fma(a.Cb[n * NB + j], X[i * NB + j], u);
                U[e] = u;
            }
            __syncthreads();
            for (int e = lane; e < MA * MB; e += 64) {   // out[m][n] = sum_i Ca[m][i] U[i][n]
                const int m = e / MB, n = e % MB;
                double v = 0.0;
                for (int i = 0; i < NA; ++i) v = fma(a.Ca[m * NA + i], U[i * MB + n], v);
                out[ij + (int64_t)a.npair * e] = v;
            }
        }
    }
}

struct NuclearArgs {
    const PairRec *pairs;
    int npair;
    const double *center, *expo, *coef;
    const double *charges;   // [4*ncharge]: x, y, z, q
    int ncharge;
    const double *boys;
    const double *Ca, *Cb;
    double *V;               // [ij + npair*ab]
};

// F_m(x), m <= M: the evaluation of boys_eval (Taylor series about the
// nearest 1/8 node, then downward recursion; asymptotic form for x >= 45)
// with the node rows of order M .. M + BOYS_NTERM - 1 held in LDS,
// rows[k * BOYS_NTERM + i].  Lanes of a wave read unrelated rows; from LDS
// those gathers cost a few cycles instead of a trip through the vector cache.
template <int M>
__device__ __forceinline__ void boys_eval_rows(double x, double *__restrict__ F, const double *__restrict__ rows)
{
    if (x < (double)BOYS_XMAX) {
        const int k = __double2int_rn(x * (double)BOYS_STEP_INV);
        const double d = (double)k * (1.0 / BOYS_STEP_INV) - x;
        const double *row = rows + k * BOYS_NTERM;
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
        F[0] = sqrt(0.78539816339744830962 * rx);
        if (M > 0) {
            const double e = exp(-x);
            const double hrx = 0.5 * rx;
#pragma unroll
            for (int m = 0; m < M; ++m) F[m + 1] = fma((double)(2 * m + 1), F[m], -e) * hrx;
        }
    }
}

// A workgroup takes 64 shell pairs (one per lane) and G waves: wave w sums
// the charges I = w, w + G, ... and transforms its partial Hermite sums itself
// (the transform is linear); the partial integrals are added across waves
// through LDS at the end.  Splitting the charges gives a batch of 65,536
// pairs G waves per SIMD instead of one, at the price of G transforms per
// primitive pair -- worth it where registers leave room for more waves
// (measured: 8 waves up to L = 1, 4 for L = 2 (8 were 20 % slower there),
// 2 for L = 3 and 4).  At L = 4 the kernel
// is held to 256 registers so that two waves share a SIMD ((d|d) K=5 took
// 14 % less time than with one wave of 264 registers); L = 5, 6 keep one
// wave of up to 512.  LT: Boys rows staged in LDS (else read from the
// global table; LDS was faster for every class).
template <int LA, int LB>
constexpr int nuclear_waves() { return LA + LB <= 1 ? 8 : (LA + LB == 2 ? 4 : (LA + LB <= 4 ? 2 : 1)); }
template <int LA, int LB>
constexpr int nuclear_wpe() { return LA + LB == 4 ? 2 : 1; }
template <int LA, int LB>
constexpr bool nuclear_lds_rows() { return true; }

// ---------------------------------------------------------------------------
// Hermite-to-Cartesian step of the lane kernel for L = l_a + l_b >= 3.
// The E^{ab}_{tuv} of Eq. (34) are the coefficients of x_A^a x_B^b in the
// Hermite Gaussians at P, and they factor.  With x_A = x_P + (P - A),
// x_B = x_P + (P - B) (binomial shifts) and
//   x_P^e exp(-p x_P^2) = sum_t c^e_t Lambda_t,
//   c^{e+1}_t = c^e_{t-1} / (2p) + (t + 1) c^e_{t+1}
// (Eq. (10) at X_PA = 0; closed form c^e_t = e! / (t! k! 2^k) (2p)^-(t+k)
// for e = t + 2k), the sum of Eq. (34) is taken in two stages:
//   M_e  = sum_tuv c^{e_x}_t c^{e_y}_u c^{e_z}_v [tuv]        (|e| <= L),
//   V_ab = sum_{k<=a, k'<=b} C(a,k) C(b,k') (P-A)^{a-k} (P-B)^{b-k'} M_{k+k'}.
// M replaces the Hermite table in place, one axis at a time, so a lane holds
// one table of N_H(L) values instead of the pair's three E tables next to it
// (which spilled to scratch for L >= 3).  Both shifts start from P, so the
// terms have the magnitudes of the direct sum; a shift from A to B after the
// primitive sum would multiply rounding errors by up to (|AB| / width)^l_b.
// ---------------------------------------------------------------------------
template <int LA, int LB>
constexpr bool nuclear_factored() { return LA + LB >= 3; }

__host__ __device__ constexpr int binom(int n, int k)
{
    int r = 1;
    for (int i = 1; i <= k; ++i) r = r * (n - k + i) / i;
    return r;
}

// e! / (t! k! 2^k), e = t + 2k
__host__ __device__ constexpr int mono_coef(int e, int t)
{
    const int k = (e - t) / 2;
    int r = 1;
    for (int i = t + k + 1; i <= e; ++i) r *= i;   // e! / (t+k)!
    for (int i = 2; i <= k; ++i) r /= i;           // / k!
    int num = 1;
    for (int i = t + 1; i <= t + k; ++i) num *= i; // (t+k)! / t!
    return r * num / (1 << k);
}

__host__ __device__ constexpr int tuv_axis(Tuv r, int ax) { return ax == 0 ? r.t : (ax == 1 ? r.u : r.v); }

struct MonoTerm {
    short dst, src;
    signed char e, t, first, last;
};

__host__ __device__ constexpr int mono_terms(int L, int ax)
{
    int n = 0;
    for (int k = 0; k < nherm(L); ++k) {
        const int e = tuv_axis(herm_tuv(k), ax);
        if (e > 0) n += e / 2 + 1;
    }
    return n;
}

// along axis AX, every slot with axis exponent e >= 1 becomes
// sum_{t = e, e-2, ...} c^e_t (slot with that exponent t); slots are rewritten
// in order of decreasing e, so each reads values not yet replaced
template <int L, int AX>
struct MonoPlan {
    static constexpr int N = mono_terms(L, AX);
    MonoTerm s[N > 0 ? N : 1];
    constexpr MonoPlan() : s{}
    {
        int n = 0;
        for (int e = L; e >= 1; --e)
            for (int k = 0; k < nherm(L); ++k) {
                const Tuv r = herm_tuv(k);
                if (tuv_axis(r, AX) != e) continue;
                for (int t = e; t >= 0; t -= 2) {
                    const int src = herm_index(AX == 0 ? t : r.t, AX == 1 ? t : r.u, AX == 2 ? t : r.v);
                    s[n].dst = (short)k;
                    s[n].src = (short)src;
                    s[n].e = (signed char)e;
                    s[n].t = (signed char)t;
                    s[n].first = (signed char)(t == e);
                    s[n].last = (signed char)(t < 2);
                    ++n;
                }
            }
    }
};

template <int L, int AX>
__device__ __forceinline__ void monomial_axis(double *__restrict__ W, const double (&ch)[L + 1][L + 1])
{
    constexpr MonoPlan<L, AX> plan{};
    double acc = 0.0;
#pragma unroll
    for (int i = 0; i < plan.N; ++i) {
        const MonoTerm m = plan.s[i];
        acc = m.first ? ch[m.e][m.t] * W[m.src] : fma(ch[m.e][m.t], W[m.src], acc);
        if (m.last) W[m.dst] = acc;
    }
}

// [tuv] -> M_e in place (h = 1/(2p))
template <int L>
__device__ __forceinline__ void hermite_to_monomial(double *__restrict__ W, double h)
{
    double hp[L + 1];
    hp[0] = 1.0;
#pragma unroll
    for (int n = 1; n <= L; ++n) hp[n] = hp[n - 1] * h;
    double ch[L + 1][L + 1];
#pragma unroll
    for (int e = 0; e <= L; ++e)
#pragma unroll
        for (int t = 0; t <= L; ++t) ch[e][t] = (t <= e && (e - t) % 2 == 0) ? (double)mono_coef(e, t) * hp[(e + t) / 2] : 0.0;
    monomial_axis<L, 0>(W, ch);
    monomial_axis<L, 1>(W, ch);
    monomial_axis<L, 2>(W, ch);
}

template <int L>
struct HermTab {
    signed char t[nherm(L)], u[nherm(L)], v[nherm(L)];
    constexpr HermTab() : t{}, u{}, v{}
    {
        for (int k = 0; k < nherm(L); ++k) {
            const Tuv r = herm_tuv(k);
            t[k] = (signed char)r.t;
            u[k] = (signed char)r.u;
            v[k] = (signed char)r.v;
        }
    }
};

// bra function I of the shift: U[k'] = sum_k C(a,k) (P-A)^{a-k} M_{k+k'} over
// |k'| <= l_b, then V[I][j] += f sum_{k'<=b_j} C(b_j,k') (P-B)^{b_j-k'} U[k']
template <int LA, int LB, int I>
__device__ __forceinline__ void shift_bra_function(const double *__restrict__ W, const double (&pa)[3][LA + 1],
                                                   const double (&pb)[3][LB + 1], double f,
                                                   double (&V)[ncart(LA)][ncart(LB)])
{
    constexpr int ax = cart_exp(LA, I, 0), ay = cart_exp(LA, I, 1), az = cart_exp(LA, I, 2);
    constexpr int NK = nherm(LB), NB = ncart(LB);
    constexpr HermTab<LB> hk{};
    double U[NK];
#pragma unroll
    for (int kx = 0; kx <= ax; ++kx)
#pragma unroll
        for (int ky = 0; ky <= ay; ++ky)
#pragma unroll
            for (int kz = 0; kz <= az; ++kz) {
                const double c = (double)(binom(ax, kx) * binom(ay, ky) * binom(az, kz)) * pa[0][ax - kx] *
                                 pa[1][ay - ky] * pa[2][az - kz];
#pragma unroll
                for (int q = 0; q < NK; ++q) {
                    const double w = W[herm_index(kx + hk.t[q], ky + hk.u[q], kz + hk.v[q])];
                    U[q] = (kx | ky | kz) ? fma(c, w, U[q]) : c * w;
                }
            }
#pragma unroll
    for (int j = 0; j < NB; ++j) {
        const int bx = hk.t[nherm(LB - 1) + j], by = hk.u[nherm(LB - 1) + j], bz = hk.v[nherm(LB - 1) + j];
        double s = 0.0;
#pragma unroll
        for (int kx = 0; kx <= bx; ++kx)
#pragma unroll
            for (int ky = 0; ky <= by; ++ky)
#pragma unroll
                for (int kz = 0; kz <= bz; ++kz)
                    s = fma((double)(binom(bx, kx) * binom(by, ky) * binom(bz, kz)) * pb[0][bx - kx] *
                                pb[1][by - ky] * pb[2][bz - kz],
                            U[herm_index(kx, ky, kz)], s);
        V[I][j] = fma(f, s, V[I][j]);
    }
}

// the same with the roles swapped, for l_b > l_a (the shorter intermediate):
// U[k] = sum_{k'<=b} C(b,k') (P-B)^{b-k'} M_{k+k'} over |k| <= l_a for ket function J
template <int LA, int LB, int J>
__device__ __forceinline__ void shift_ket_function(const double *__restrict__ W, const double (&pa)[3][LA + 1],
                                                   const double (&pb)[3][LB + 1], double f,
                                                   double (&V)[ncart(LA)][ncart(LB)])
{
    constexpr int bx = cart_exp(LB, J, 0), by = cart_exp(LB, J, 1), bz = cart_exp(LB, J, 2);
    constexpr int NK = nherm(LA), NA = ncart(LA);
    constexpr HermTab<LA> hk{};
    double U[NK];
#pragma unroll
    for (int kx = 0; kx <= bx; ++kx)
#pragma unroll
        for (int ky = 0; ky <= by; ++ky)
#pragma unroll
            for (int kz = 0; kz <= bz; ++kz) {
                const double c = (double)(binom(bx, kx) * binom(by, ky) * binom(bz, kz)) * pb[0][bx - kx] *
                                 pb[1][by - ky] * pb[2][bz - kz];
#pragma unroll
                for (int q = 0; q < NK; ++q) {
                    const double w = W[herm_index(kx + hk.t[q], ky + hk.u[q], kz + hk.v[q])];
                    U[q] = (kx | ky | kz) ? fma(c, w, U[q]) : c * w;
                }
            }
#pragma unroll
    for (int i = 0; i < NA; ++i) {
        const int ax = hk.t[nherm(LA - 1) + i], ay = hk.u[nherm(LA - 1) + i], az = hk.v[nherm(LA - 1) + i];
        double s = 0.0;
#pragma unroll
        for (int kx = 0; kx <= ax; ++kx)
#pragma unroll
            for (int ky = 0; ky <= ay; ++ky)
#pragma unroll
                for (int kz = 0; kz <= az; ++kz)
                    s = fma((double)(binom(ax, kx) * binom(ay, ky) * binom(az, kz)) * pa[0][ax - kx] *
                                pa[1][ay - ky] * pa[2][az - kz],
                            U[herm_index(kx, ky, kz)], s);
        V[i][J] = fma(f, s, V[i][J]);
    }
}

template <int LA, int LB, int... Is>
__device__ __forceinline__ void shift_pair(const double *__restrict__ W, const double (&pa)[3][LA + 1],
                                           const double (&pb)[3][LB + 1], double f,
                                           double (&V)[ncart(LA)][ncart(LB)], std::integer_sequence<int, Is...>)
{
    if constexpr (LB > LA) (shift_ket_function<LA, LB, Is>(W, pa, pb, f, V), ...);
    else (shift_bra_function<LA, LB, Is>(W, pa, pb, f, V), ...);
}

template <int LA, int LB, bool CART, int G, bool LT>
__global__ void __launch_bounds__(64 * G) __attribute__((amdgpu_waves_per_eu(nuclear_wpe<LA, LB>()))) nuclear_kernel(NuclearArgs a)
{
    constexpr int L = LA + LB, NH = nherm(L), NA = ncart(LA), NB = ncart(LB), NF = NA * NB;
    constexpr int NROWT = BOYS_NROW * BOYS_NTERM;
    constexpr int NLDS = LT ? NROWT : (G > 1 ? 64 * (G - 1) * (NF < 18 ? NF : 18) : 1);
    __shared__ double lds[NLDS];   // Boys rows of order L; after the charge loop, the partial sums
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
    if constexpr (LT) {
        for (int i = threadIdx.x; i < NROWT; i += 64 * G)
            lds[i] = a.boys[(i / BOYS_NTERM) * BOYS_NCOL + L + i % BOYS_NTERM];
        __syncthreads();
    }

    const int ij = blockIdx.x * 64 + lane;
    double V[NA][NB];
#pragma unroll
    for (int i = 0; i < NA; ++i)
#pragma unroll
        for (int j = 0; j < NB; ++j) V[i][j] = 0.0;
    if (ij < a.npair) {
        const PairRec pr = a.pairs[ij];
        const double A[3] = {a.center[3 * pr.sa], a.center[3 * pr.sa + 1], a.center[3 * pr.sa + 2]};
        const double B[3] = {a.center[3 * pr.sb], a.center[3 * pr.sb + 1], a.center[3 * pr.sb + 2]};
        const double AB2 =
            (A[0] - B[0]) * (A[0] - B[0]) + (A[1] - B[1]) * (A[1] - B[1]) + (A[2] - B[2]) * (A[2] - B[2]);
        for (int ka = 0; ka < pr.ka; ++ka) {
            const double za = a.expo[pr.offa + ka], ca = a.coef[pr.offa + ka];
            for (int kb = 0; kb < pr.kb; ++kb) {
                const double zb = a.expo[pr.offb + kb], cb = a.coef[pr.offb + kb];
                const double p = za + zb, rp = 1.0 / p;
                // P = A + (zeta_b/p)(B - A): exactly A on one centre
                const double P[3] = {A[0] + zb * rp * (B[0] - A[0]), A[1] + zb * rp * (B[1] - A[1]),
                                     A[2] + zb * rp * (B[2] - A[2])};
                // sum_I q_I [r]_I^(0) over this wave's charges, Eqs. (26), (30),
                // before any transform (Eq. (37))
                double Rs[NH];
#pragma unroll
                for (int k = 0; k < NH; ++k) Rs[k] = 0.0;
                const double g = 2.0 * M_PI * rp, m2p = -2.0 * p;
                for (int I = w; I < a.ncharge; I += G) {
                    const double *c = a.charges + 4 * I;   // the same charge in every lane of the wave
                    const double X = P[0] - c[0], Y = P[1] - c[1], Z = P[2] - c[2];
                    double F[L + 1];
                    if constexpr (LT) boys_eval_rows<L>(p * (X * X + Y * Y + Z * Z), F, lds);
                    else boys_eval<L>(p * (X * X + Y * Y + Z * Z), F, a.boys);
                    double S[L + 1];
                    double f = c[3] * g;
#pragma unroll
                    for (int m = 0; m <= L; ++m) {
                        S[m] = f * F[m];
                        f *= m2p;
                    }
                    r_accumulate<L>(S, X, Y, Z, Rs);
                }
                const double f = -ca * cb * exp(-za * zb * rp * AB2);
                if constexpr (nuclear_factored<LA, LB>()) {
                    // Eq. (34) in two stages: monomials at P, then the shifts to A and B
                    double pa[3][LA + 1], pb[3][LB + 1];
#pragma unroll
                    for (int ax = 0; ax < 3; ++ax) {
                        const double xa = zb * rp * (B[ax] - A[ax]), xb = za * rp * (A[ax] - B[ax]);
                        pa[ax][0] = 1.0;
                        pb[ax][0] = 1.0;
#pragma unroll
                        for (int n = 1; n <= LA; ++n) pa[ax][n] = pa[ax][n - 1] * xa;
#pragma unroll
                        for (int n = 1; n <= LB; ++n) pb[ax][n] = pb[ax][n - 1] * xb;
                    }
                    hermite_to_monomial<L>(Rs, 0.5 * rp);
                    shift_pair<LA, LB>(Rs, pa, pb, f, V, std::make_integer_sequence<int, (LB > LA ? NB : NA)>{});
                } else {
                    // E coefficients of the pair and the bra transform, Eq. (34)
                    double E[3][LA + 1][LB + 1][L + 1];
#pragma unroll
                    for (int ax = 0; ax < 3; ++ax)
                        e_axis<LA, LB>(0.5 * rp, zb * rp * (B[ax] - A[ax]), za * rp * (A[ax] - B[ax]), E[ax]);
#pragma unroll
                    for (int i = 0; i < NA; ++i)
#pragma unroll
                        for (int j = 0; j < NB; ++j) {
                            const int ix = cart_exp(LA, i, 0), iy = cart_exp(LA, i, 1), iz = cart_exp(LA, i, 2);
                            const int jx = cart_exp(LB, j, 0), jy = cart_exp(LB, j, 1), jz = cart_exp(LB, j, 2);
                            double s = 0.0;
#pragma unroll
                            for (int t = 0; t <= ix + jx; ++t)
#pragma unroll
                                for (int u = 0; u <= iy + jy; ++u) {
                                    const double etu = E[0][ix][jx][t] * E[1][iy][jy][u];
#pragma unroll
                                    for (int v = 0; v <= iz + jz; ++v)
                                        s = fma(etu * E[2][iz][jz][v], Rs[herm_index(t, u, v)], s);
                                }
                            V[i][j] = fma(f, s, V[i][j]);
                        }
                }
            }
        }
    }
    // add the waves' partial integrals, CH function pairs at a time
    if constexpr (G > 1) {
    constexpr int CH = NLDS / (64 * (G - 1)) < NF ? NLDS / (64 * (G - 1)) : NF;
    __syncthreads();   // every wave is past its charge loop: the rows are free
#pragma unroll
    for (int c0 = 0; c0 < NF; c0 += CH) {
        if (w > 0) {
#pragma unroll
            for (int k = c0; k < c0 + CH && k < NF; ++k) lds[((w - 1) * CH + k - c0) * 64 + lane] = V[k / NB][k % NB];
        }
        __syncthreads();
        if (w == 0) {
#pragma unroll
            for (int k = c0; k < c0 + CH && k < NF; ++k)
#pragma unroll
                for (int v = 0; v < G - 1; ++v) V[k / NB][k % NB] += lds[(v * CH + k - c0) * 64 + lane];
        }
        __syncthreads();
    }
    }
    if (w == 0 && ij < a.npair) store_pair<LA, LB, CART>(V, a.Ca, a.Cb, a.V, ij, a.npair);
}

template <int LA, int LB>
static void launch_nuclear(const NuclearArgs &a, bool cart, hipStream_t s)
{
    constexpr int G = nuclear_waves<LA, LB>();
    constexpr bool LT = nuclear_lds_rows<LA, LB>();
    const int nblk = (a.npair + 63) / 64;
    if (cart) hipLaunchKernelGGL((nuclear_kernel<LA, LB, true, G, LT>), dim3(nblk), dim3(64 * G), 0, s, a);
    else hipLaunchKernelGGL((nuclear_kernel<LA, LB, false, G, LT>), dim3(nblk), dim3(64 * G), 0, s, a);
}

// ---------------------------------------------------------------------------
// 1-particle Coulomb integrals of the classes with l_a + l_b >= 7: one shell
// pair per wave.
//
// The charge-summed table of one primitive pair, sum_I [tuv]_I^(0), has
// N_H(L) values (455 at L = 12), too many for one lane, so the lanes share
// it: lane c owns column (u_c, v_c), the L - u_c - v_c + 1 entries with
// those u, v.  The charges go through the wave 64 at a time, one per lane;
// a lane forms every column of its charge from the closed form of the
// recursion of Eq. (31),
//   [tuv]^(0) = sum_{i,j,k} h_{t,i} h_{u,j} h_{v,k} X^{t-2i} Y^{u-2j} Z^{v-2k} S_{t+u+v-i-j-k},
//   h_{t,i} = t! / (i! (t-2i)! 2^i),  S_n = [000]^(n) (Eq. (30) times the charge),
// (the derivative d/dX of [000]^(n) is X [000]^(n+1)), column by column with
// compile-time indices, and each entry is summed over the lanes (charges)
// into its column's owner.  After the charges, the transform of Eq. (34)
// runs through the wave's LDS table: monomials at P along x (in each lane's
// column), y and z (lanes over lines), then both binomial shifts at once as
// per-axis products G[i][j][e] (the coefficient of x_P^e in x_A^i x_B^j),
// V_ab = sum_e G_x G_y G_z M_e, with lanes over the Cartesian function pairs
// and loops of compile-time bounds over the whole table (G's zeros drop the
// terms beyond a + b; per-lane bounds would make a wave run the product of
// the lanes' maxima).  Waves synchronise only within themselves (the pairs
// of a workgroup have different primitive counts).
// ---------------------------------------------------------------------------
__device__ __forceinline__ void wave_lds_sync()
{
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

// h_{t,i} = t! / (i! (t-2i)! 2^i)
__host__ __device__ constexpr double herm_poly_coef(int t, int i)
{
    double r = 1.0;
    for (int k = 1; k <= t; ++k) r *= k;
    for (int k = 1; k <= i; ++k) r /= 2 * k;          // i! 2^i
    for (int k = 1; k <= t - 2 * i; ++k) r /= k;
    return r;
}

// compile-time tables of h_{t,i} (i <= t/2) and of the monomial coefficients
// e! / (t! k! 2^k) (e = t + 2k), both up to order L
template <int L>
struct NucCoefTab {
    double h[L + 1][L / 2 + 1], m[L + 1][L + 1];
    constexpr NucCoefTab() : h{}, m{}
    {
        for (int t = 0; t <= L; ++t)
            for (int i = 0; 2 * i <= t; ++i) h[t][i] = herm_poly_coef(t, i);
        for (int e = 0; e <= L; ++e)
            for (int t = e; t >= 0; t -= 2) m[e][t] = (double)mono_coef(e, t);
    }
};

// per-wave LDS (doubles): the Hermite/monomial table, the per-axis shift
// products G[3][l_a+1][l_b+1][L+1] and the powers [2][3][7] during the
// primitive loop; the Cartesian block and [NA][2 l_b + 1] for the solid
// transform after it
template <int LA, int LB>
struct NucWaveLds {
    static constexpr int L = LA + LB;
    static constexpr int NH = nherm(L), NGD = 3 * (LA + 1) * (LB + 1) * (L + 1), NPW = 2 * 3 * 7;
    static constexpr int NA = ncart(LA), NB = ncart(LB), NF = NA * NB;
    static constexpr int RA = NH + NGD + NPW > NF + NA * (2 * LB + 1) ? NH + NGD + NPW : NF + NA * (2 * LB + 1);
    static constexpr int OFF_M = 0, OFF_G = NH, OFF_PW = NH + NGD, OFF_V = 0;
    static constexpr int SIZE = RA;
    // pairs (waves) per workgroup: as many as 64 KB of static LDS hold
    static constexpr int WAVES_FIT = 65536 / (SIZE * 8);
    static constexpr int WAVES = WAVES_FIT >= 4 ? 4 : (WAVES_FIT < 1 ? 1 : WAVES_FIT);
};

// sum over the wave's lanes; every lane gets the total
__device__ __forceinline__ double wave_sum(double v)
{
#pragma unroll
    for (int o = 32; o >= 1; o >>= 1) v += __shfl_xor(v, o);
    return v;
}

// column C = q (q + 1) / 2 + v of the order-L table (u = q - v): each lane
// forms its own charge's [t u v] for t <= L - u - v from the closed form
//   D_d = sum_{j+k=d} h_{u,j} h_{v,k} Y^{u-2j} Z^{v-2k},  W_n = sum_d D_d S_{n+u+v-d},
//   [tuv] = sum_i h_{t,i} X^{t-2i} W_{t-i},
// the wave sums them over its charges, and the lane owning the column
// (lane C mod 64, slot C / 64) adds the sums to its table
__host__ __device__ constexpr int col_level(int c)
{
    int q = 0;
    while ((q + 1) * (q + 2) / 2 <= c) ++q;
    return q;
}

template <int L, int NCS, int C>
__device__ __forceinline__ void nuc_column(const double (&S)[L + 1], const double (&Xp)[L + 1],
                                           const double (&Yp)[L + 1], const double (&Zp)[L + 1],
                                           double (&Rs)[NCS][L + 1], int lane)
{
    constexpr int q = col_level(C), v = C - q * (q + 1) / 2, u = q - v, n = L - q;
    constexpr int DM = u / 2 + v / 2;
    constexpr NucCoefTab<L> ct{};
    double D[DM + 1];
#pragma unroll
    for (int d = 0; d <= DM; ++d) D[d] = 0.0;
#pragma unroll
    for (int j = 0; 2 * j <= u; ++j)
#pragma unroll
        for (int k = 0; 2 * k <= v; ++k) D[j + k] = fma(ct.h[u][j] * ct.h[v][k] * Yp[u - 2 * j], Zp[v - 2 * k], D[j + k]);
    double W[n + 1];
#pragma unroll
    for (int m = 0; m <= n; ++m) {
        double x = 0.0;
#pragma unroll
        for (int d = 0; d <= DM; ++d) x = fma(D[d], S[m + q - d], x);
        W[m] = x;
    }
#pragma unroll
    for (int t = 0; t <= n; ++t) {
        double x = 0.0;
#pragma unroll
        for (int i = 0; 2 * i <= t; ++i) x = fma(ct.h[t][i] * Xp[t - 2 * i], W[t - i], x);
        x = wave_sum(x);
        if (lane == C % 64) Rs[C / 64][t] += x;
    }
}

template <int L, int NCS, int... Cs>
__device__ __forceinline__ void nuc_columns(const double (&S)[L + 1], const double (&Xp)[L + 1],
                                            const double (&Yp)[L + 1], const double (&Zp)[L + 1],
                                            double (&Rs)[NCS][L + 1], int lane, std::integer_sequence<int, Cs...>)
{
    (nuc_column<L, NCS, Cs>(S, Xp, Yp, Zp, Rs, lane), ...);
}

template <int LA, int LB, bool CART>
__global__ void __launch_bounds__((64 * NucWaveLds<LA, LB>::WAVES))
__attribute__((amdgpu_waves_per_eu(2))) nuclear_wave_kernel(NuclearArgs a)
{
    constexpr int L = LA + LB, H2 = L / 2, NA = ncart(LA), NB = ncart(LB), NF = NA * NB;
    constexpr int NCOL = (L + 1) * (L + 2) / 2;   // columns (u, v), also the lines of the y and z stages
    constexpr int NCS = (NCOL + 63) / 64, NVS = (NF + 63) / 64;
    using LY = NucWaveLds<LA, LB>;
    constexpr int NWV = LY::WAVES;
    constexpr NucCoefTab<L> ct{};
    static_assert(LY::WAVES_FIT >= 1, "per-wave LDS too large");
    __shared__ double wlds[NWV][LY::SIZE];   // the waves run independently: no workgroup barrier
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;

    const int ij = blockIdx.x * NWV + w;
    if (ij >= a.npair) return;
    double *mt = wlds[w] + LY::OFF_M, *gt = wlds[w] + LY::OFF_G, *pw = wlds[w] + LY::OFF_PW,
           *vb = wlds[w] + LY::OFF_V;   // vb: after the primitive loop

    // the lane's columns: c = lane + 64 s -> (u, v), u + v = q, c = q (q + 1) / 2 + v
    int cu[NCS], cv[NCS], cn[NCS];
#pragma unroll
    for (int s = 0; s < NCS; ++s) {
        const int c = lane + 64 * s;
        int q = 0;
        while ((q + 1) * (q + 2) / 2 <= c) ++q;
        cv[s] = c - q * (q + 1) / 2;
        cu[s] = q - cv[s];
        cn[s] = c < NCOL ? L - q : -1;
    }
    double V[NVS];
#pragma unroll
    for (int s = 0; s < NVS; ++s) V[s] = 0.0;

    const PairRec pr = a.pairs[ij];
    const double A[3] = {a.center[3 * pr.sa], a.center[3 * pr.sa + 1], a.center[3 * pr.sa + 2]};
    const double B[3] = {a.center[3 * pr.sb], a.center[3 * pr.sb + 1], a.center[3 * pr.sb + 2]};
    const double AB2 = (A[0] - B[0]) * (A[0] - B[0]) + (A[1] - B[1]) * (A[1] - B[1]) + (A[2] - B[2]) * (A[2] - B[2]);
    for (int ka = 0; ka < pr.ka; ++ka) {
        const double za = a.expo[pr.offa + ka], ca = a.coef[pr.offa + ka];
        for (int kb = 0; kb < pr.kb; ++kb) {
            const double zb = a.expo[pr.offb + kb], cb = a.coef[pr.offb + kb];
            const double p = za + zb, rp = 1.0 / p;
            const double P[3] = {A[0] + zb * rp * (B[0] - A[0]), A[1] + zb * rp * (B[1] - A[1]),
                                 A[2] + zb * rp * (B[2] - A[2])};
            double Rs[NCS][L + 1];
#pragma unroll
            for (int s = 0; s < NCS; ++s)
#pragma unroll
                for (int t = 0; t <= L; ++t) Rs[s][t] = 0.0;
            const double g = 2.0 * M_PI * rp, m2p = -2.0 * p;
            // the charges 64 at a time, one per lane
            for (int I0 = 0; I0 < a.ncharge; I0 += 64) {
                const bool live = I0 + lane < a.ncharge;
                const double *ch = a.charges + 4 * (live ? I0 + lane : 0);
                const double X = P[0] - ch[0], Y = P[1] - ch[1], Z = P[2] - ch[2];
                double F[L + 1], S[L + 1];
                boys_eval<L>(p * (X * X + Y * Y + Z * Z), F, a.boys);
                double f = live ? ch[3] * g : 0.0;
#pragma unroll
                for (int m = 0; m <= L; ++m) {
                    S[m] = f * F[m];
                    f *= m2p;
                }
                double Xp[L + 1], Yp[L + 1], Zp[L + 1];
                Xp[0] = Yp[0] = Zp[0] = 1.0;
#pragma unroll
                for (int n = 1; n <= L; ++n) {
                    Xp[n] = Xp[n - 1] * X;
                    Yp[n] = Yp[n - 1] * Y;
                    Zp[n] = Zp[n - 1] * Z;
                }
                nuc_columns<L, NCS>(S, Xp, Yp, Zp, Rs, lane, std::make_integer_sequence<int, NCOL>{});
            }
            // Eq. (34), factored: monomials at P along x in each lane's column
            const double h = 0.5 * rp;
            double hp[L + 1];
            hp[0] = 1.0;
#pragma unroll
            for (int n = 1; n <= L; ++n) hp[n] = hp[n - 1] * h;
#pragma unroll
            for (int s = 0; s < NCS; ++s) {
                if (cn[s] < 0) continue;
#pragma unroll
                for (int e = L; e >= 0; --e) {
                    double v = 0.0;
#pragma unroll
                    for (int t = e; t >= 0; t -= 2) v = fma(ct.m[e][t] * hp[(e + t) / 2], Rs[s][t], v);
                    if (e <= cn[s]) mt[herm_index(e, cu[s], cv[s])] = v;
                }
            }
            // powers (P - centre)^n of this primitive pair, [side][axis][n], n <= 6
            if (lane < 6) {
                const int side = lane / 3, ax = lane % 3;
                const double d = side == 0 ? P[ax] - A[ax] : P[ax] - B[ax];
                double v = 1.0;
                for (int n = 0; n < 7; ++n) {
                    pw[(side * 3 + ax) * 7 + n] = v;
                    v *= d;
                }
            }
            wave_lds_sync();
            // y stage (lines (e_x, v) along u), then z stage (lines (e_x, e_y) along v)
#pragma unroll
            for (int stage = 1; stage <= 2; ++stage) {
#pragma unroll
                for (int s = 0; s < NCS; ++s) {
                    if (cn[s] < 0) continue;
                    const int c0 = cu[s], c1 = cv[s], n = cn[s];   // line (c0, c1): e_x = c0, and v or e_y = c1
                    double y[L + 1];
#pragma unroll
                    for (int k = 0; k <= L; ++k)
                        y[k] = k <= n ? mt[stage == 1 ? herm_index(c0, k, c1) : herm_index(c0, c1, k)] : 0.0;
#pragma unroll
                    for (int e = L; e >= 0; --e) {
                        double v = 0.0;
#pragma unroll
                        for (int t = e; t >= 0; t -= 2) v = fma(ct.m[e][t] * hp[(e + t) / 2], y[t], v);
                        if (e <= n) mt[stage == 1 ? herm_index(c0, e, c1) : herm_index(c0, c1, e)] = v;
                    }
                }
                wave_lds_sync();
            }
            // per-axis products of the two shifts,
            //   G[ax][i][j][e] = sum_{k+k'=e} C(i,k) C(j,k') (P-A)_ax^{i-k} (P-B)_ax^{j-k'}
            // (zero for e > i + j), so that V_ab = f sum_e G_x G_y G_z M_e
            for (int e = lane; e < LY::NGD; e += 64) {
                const int ax = e / ((LA + 1) * (LB + 1) * (L + 1)), i = (e / ((LB + 1) * (L + 1))) % (LA + 1),
                          j = (e / (L + 1)) % (LB + 1), q = e % (L + 1);
                double v = 0.0;
                for (int k = q - j > 0 ? q - j : 0; k <= i && k <= q; ++k)
                    v = fma((double)(binom(i, k) * binom(j, q - k)) * pw[ax * 7 + i - k], pw[(3 + ax) * 7 + j - q + k], v);
                gt[e] = v;
            }
            wave_lds_sync();
            // the contraction, lanes over Cartesian function pairs, uniform loops
            // over the whole monomial table (G's zeros drop the terms beyond a + b)
            const double f = -ca * cb * exp(-za * zb * rp * AB2);
#pragma unroll 1
            for (int s = 0; s < NVS; ++s) {
                // keeps the table's loads inside the loop (hoisted, hundreds of them stayed live and spilled)
                __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
                const int fp = lane + 64 * s < NF ? lane + 64 * s : 0;
                const int ia = fp / NB, ib = fp % NB;
                const int gi[3] = {cart_exp(LA, ia, 0), cart_exp(LA, ia, 1), cart_exp(LA, ia, 2)};
                const int gj[3] = {cart_exp(LB, ib, 0), cart_exp(LB, ib, 1), cart_exp(LB, ib, 2)};
                const double *gxp = gt + ((0 * (LA + 1) + gi[0]) * (LB + 1) + gj[0]) * (L + 1);
                const double *gyp = gt + ((1 * (LA + 1) + gi[1]) * (LB + 1) + gj[1]) * (L + 1);
                const double *gzp = gt + ((2 * (LA + 1) + gi[2]) * (LB + 1) + gj[2]) * (L + 1);
                double gz[L + 1];
#pragma unroll
                for (int e = 0; e <= L; ++e) gz[e] = gzp[e];
                double acc = 0.0;
#pragma unroll
                for (int ex = 0; ex <= L; ++ex) {
                    double sx = 0.0;
#pragma unroll
                    for (int ey = 0; ex + ey <= L; ++ey) {
                        double sy = 0.0;
#pragma unroll
                        for (int ez = 0; ex + ey + ez <= L; ++ez) sy = fma(gz[ez], mt[herm_index(ex, ey, ez)], sy);
                        sx = fma(gyp[ey], sy, sx);
                    }
                    acc = fma(gxp[ex], sx, acc);
                }
#pragma unroll
                for (int s2 = 0; s2 < NVS; ++s2)
                    if (s2 == s) V[s2] = fma(f, acc, V[s2]);
            }
            wave_lds_sync();   // the table and shift tables are rewritten by the next primitive pair
        }
    }
    // store: Cartesian directly; solid harmonics through the wave's LDS (Eq. (18), ket index first)
    if constexpr (CART) {
#pragma unroll
        for (int s = 0; s < NVS; ++s) {
            const int fp = lane + 64 * s;
            if (fp < NF) a.V[ij + (int64_t)a.npair * fp] = V[s];
        }
    } else {
        constexpr int MA = 2 * LA + 1, MB = 2 * LB + 1;
        double *ub = vb + NF;   // [NA][MB]
#pragma unroll
        for (int s = 0; s < NVS; ++s) {
            const int fp = lane + 64 * s;
            if (fp < NF) vb[fp] = V[s];
        }
        wave_lds_sync();
        for (int e = lane; e < NA * MB; e += 64) {
            const int i = e / MB, n = e % MB;
            double u = 0.0;
            for (int j = 0; j < NB; ++j) u = fma(a.Cb[n * NB + j], vb[i * NB + j], u);
            ub[e] = u;
        }
        wave_lds_sync();
        for (int e = lane; e < MA * MB; e += 64) {
            const int m = e / MB, n = e % MB;
            double v = 0.0;
            for (int i = 0; i < NA; ++i) v = fma(a.Ca[m * NA + i], ub[i * MB + n], v);
            a.V[ij + (int64_t)a.npair * e] = v;
        }
    }
}

template <int LA, int LB>
static void launch_nuclear_wave(const NuclearArgs &a, bool cart, hipStream_t s)
{
    constexpr int NWV = NucWaveLds<LA, LB>::WAVES;
    const int nblk = (a.npair + NWV - 1) / NWV;
    if (cart) hipLaunchKernelGGL((nuclear_wave_kernel<LA, LB, true>), dim3(nblk), dim3(64 * NWV), 0, s, a);
    else hipLaunchKernelGGL((nuclear_wave_kernel<LA, LB, false>), dim3(nblk), dim3(64 * NWV), 0, s, a);
}

template <int LA, int LB, int PART>
static void launch_onebody_part(const OneBodyArgs &a, bool cart, hipStream_t s)
{
    const int nblk = (a.npair + 63) / 64;
    if (cart) hipLaunchKernelGGL((onebody_kernel<LA, LB, true, PART>), dim3(nblk), dim3(64), 0, s, a);
    else hipLaunchKernelGGL((onebody_kernel<LA, LB, false, PART>), dim3(nblk), dim3(64), 0, s, a);
}

template <int LA, int LB>
static void launch_onebody(const OneBodyArgs &a, bool cart, hipStream_t s)
{
    if constexpr (LA > ONEBODY_LANE_LMAX || LB > ONEBODY_LANE_LMAX) {   // one pair per wave
        if (cart) hipLaunchKernelGGL((onebody_wave_kernel<LA, LB, true>), dim3(a.npair), dim3(64), 0, s, a);
        else hipLaunchKernelGGL((onebody_wave_kernel<LA, LB, false>), dim3(a.npair), dim3(64), 0, s, a);
    } else if constexpr (LA + LB >= 5) {   // S and T apart: one set of accumulators per lane
        if (a.S) launch_onebody_part<LA, LB, 1>(a, cart, s);
        if (a.T) launch_onebody_part<LA, LB, 2>(a, cart, s);
    } else {
        launch_onebody_part<LA, LB, 0>(a, cart, s);
    }
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
    if (npair > 0 && (l[0] < 0 || l[1] < 0 || l[0] > ONEBODY_LMAX || l[1] > ONEBODY_LMAX))
        return fail(MDX_EUNSUPPORTED, "one-body integrals for l_a = %d, l_b = %d (compiled for l <= %d)", l[0], l[1],
                    ONEBODY_LMAX);
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

namespace mdx {

void onebody_records(const mdx_shells *sh, int32_t npair, const int32_t *pairs, std::vector<PairRec> &pr)
{
    pr.resize((size_t)npair);
    for (int32_t i = 0; i < npair; ++i) {
        const int32_t sa = pairs[2 * i], sb = pairs[2 * i + 1];
        pr[i] = PairRec{sa, sb, sh->nprim[sa], sh->nprim[sb], sh->prim_offset[sa], sh->prim_offset[sb]};
    }
}

// the lane records of a validated batch, uploaded to the head of ws
static mdx_status stage_pairs(mdx_ctx *c, const mdx_shells *sh, int32_t npair, const int32_t *pairs, void *ws,
                              size_t ws_bytes, hipStream_t s, const char *who)
{
    if (!ws) return fail(MDX_EINVAL, "%s: null workspace", who);
    if ((uintptr_t)ws & 255) return fail(MDX_EINVAL, "%s: workspace not 256-byte aligned", who);
    const size_t need = al256((size_t)npair * sizeof(PairRec));
    if (ws_bytes < need) return fail(MDX_EWORKSPACE, "workspace %zu bytes < %zu required", ws_bytes, need);
    MDX_TRY(refuse_capture(s, "the call copies its pair records from host memory"));
    std::vector<PairRec> pr;
    onebody_records(sh, npair, pairs, pr);
    HIP_TRY2(hipSetDevice(c->device));
    HIP_TRY2(hipMemcpyAsync(ws, pr.data(), pr.size() * sizeof(PairRec), hipMemcpyHostToDevice, s));
    return MDX_OK;
}

// profiling hook, as for the other integral kernels: records the opening
// event; *ev1 is the event to record after the launch (null without the hook)
static mdx_status prof_open(mdx_ctx *c, hipStream_t s, hipEvent_t *ev1)
{
    *ev1 = nullptr;
    if (c->prof_events.size() >= 2) {
        const size_t np = c->prof_events.size() / 2, i = c->prof_count++ % np;
        *ev1 = c->prof_events[2 * i + 1];
        HIP_TRY2(hipEventRecord(c->prof_events[2 * i], s));
    }
    return MDX_OK;
}

}  // namespace mdx

// one case per (l_a, l_b): l <= ONEBODY_LANE_LMAX (MDX_ONEBODY_SWITCH) or
// l <= ONEBODY_LMAX (MDX_ONEBODY_SWITCH7)
#define MDX_ONEBODY_SWITCH(LAUNCH, la, lb, ...)          \
    switch ((la) * 4 + (lb)) {                           \
    case 0: LAUNCH<0, 0>(__VA_ARGS__); break;            \
    case 1: LAUNCH<0, 1>(__VA_ARGS__); break;            \
    case 2: LAUNCH<0, 2>(__VA_ARGS__); break;            \
    case 3: LAUNCH<0, 3>(__VA_ARGS__); break;            \
    case 4: LAUNCH<1, 0>(__VA_ARGS__); break;            \
    case 5: LAUNCH<1, 1>(__VA_ARGS__); break;            \
    case 6: LAUNCH<1, 2>(__VA_ARGS__); break;            \
    case 7: LAUNCH<1, 3>(__VA_ARGS__); break;            \
    case 8: LAUNCH<2, 0>(__VA_ARGS__); break;            \
    case 9: LAUNCH<2, 1>(__VA_ARGS__); break;            \
    case 10: LAUNCH<2, 2>(__VA_ARGS__); break;           \
    case 11: LAUNCH<2, 3>(__VA_ARGS__); break;           \
    case 12: LAUNCH<3, 0>(__VA_ARGS__); break;           \
    case 13: LAUNCH<3, 1>(__VA_ARGS__); break;           \
    case 14: LAUNCH<3, 2>(__VA_ARGS__); break;           \
    default: LAUNCH<3, 3>(__VA_ARGS__); break;           \
    }

// one case per (l_a, l_b) with l_a + l_b <= 6 (the classes of the 1-particle
// Coulomb lane kernel)
#define MDX_NUCLEAR_LANE_SWITCH(LAUNCH, la, lb, ...)    \
    switch ((la) * 7 + (lb)) {                           \
    case 0: LAUNCH<0, 0>(__VA_ARGS__); break; \
    case 1: LAUNCH<0, 1>(__VA_ARGS__); break; \
    case 7: LAUNCH<1, 0>(__VA_ARGS__); break; \
    case 2: LAUNCH<0, 2>(__VA_ARGS__); break; \
    case 8: LAUNCH<1, 1>(__VA_ARGS__); break; \
    case 14: LAUNCH<2, 0>(__VA_ARGS__); break; \
    case 3: LAUNCH<0, 3>(__VA_ARGS__); break; \
    case 9: LAUNCH<1, 2>(__VA_ARGS__); break; \
    case 15: LAUNCH<2, 1>(__VA_ARGS__); break; \
    case 21: LAUNCH<3, 0>(__VA_ARGS__); break; \
    case 4: LAUNCH<0, 4>(__VA_ARGS__); break; \
    case 10: LAUNCH<1, 3>(__VA_ARGS__); break; \
    case 16: LAUNCH<2, 2>(__VA_ARGS__); break; \
    case 22: LAUNCH<3, 1>(__VA_ARGS__); break; \
    case 28: LAUNCH<4, 0>(__VA_ARGS__); break; \
    case 5: LAUNCH<0, 5>(__VA_ARGS__); break; \
    case 11: LAUNCH<1, 4>(__VA_ARGS__); break; \
    case 17: LAUNCH<2, 3>(__VA_ARGS__); break; \
    case 23: LAUNCH<3, 2>(__VA_ARGS__); break; \
    case 29: LAUNCH<4, 1>(__VA_ARGS__); break; \
    case 35: LAUNCH<5, 0>(__VA_ARGS__); break; \
    case 6: LAUNCH<0, 6>(__VA_ARGS__); break; \
    case 12: LAUNCH<1, 5>(__VA_ARGS__); break; \
    case 18: LAUNCH<2, 4>(__VA_ARGS__); break; \
    case 24: LAUNCH<3, 3>(__VA_ARGS__); break; \
    case 30: LAUNCH<4, 2>(__VA_ARGS__); break; \
    case 36: LAUNCH<5, 1>(__VA_ARGS__); break; \
    default: LAUNCH<6, 0>(__VA_ARGS__); break; \
    }

// one case per (l_a, l_b) with l_a + l_b >= 7, l <= 6 (the one-pair-per-wave
// 1-particle Coulomb kernel)
#define MDX_NUCLEAR_WAVE_SWITCH(LAUNCH, la, lb, ...)    \
    switch ((la) * 7 + (lb)) {                           \
    case 13: LAUNCH<1, 6>(__VA_ARGS__); break; \
    case 19: LAUNCH<2, 5>(__VA_ARGS__); break; \
    case 20: LAUNCH<2, 6>(__VA_ARGS__); break; \
    case 25: LAUNCH<3, 4>(__VA_ARGS__); break; \
    case 26: LAUNCH<3, 5>(__VA_ARGS__); break; \
    case 27: LAUNCH<3, 6>(__VA_ARGS__); break; \
    case 31: LAUNCH<4, 3>(__VA_ARGS__); break; \
    case 32: LAUNCH<4, 4>(__VA_ARGS__); break; \
    case 33: LAUNCH<4, 5>(__VA_ARGS__); break; \
    case 34: LAUNCH<4, 6>(__VA_ARGS__); break; \
    case 37: LAUNCH<5, 2>(__VA_ARGS__); break; \
    case 38: LAUNCH<5, 3>(__VA_ARGS__); break; \
    case 39: LAUNCH<5, 4>(__VA_ARGS__); break; \
    case 40: LAUNCH<5, 5>(__VA_ARGS__); break; \
    case 41: LAUNCH<5, 6>(__VA_ARGS__); break; \
    case 43: LAUNCH<6, 1>(__VA_ARGS__); break; \
    case 44: LAUNCH<6, 2>(__VA_ARGS__); break; \
    case 45: LAUNCH<6, 3>(__VA_ARGS__); break; \
    case 46: LAUNCH<6, 4>(__VA_ARGS__); break; \
    case 47: LAUNCH<6, 5>(__VA_ARGS__); break; \
    default: LAUNCH<6, 6>(__VA_ARGS__); break; \
    }

#define MDX_ONEBODY_SWITCH7(LAUNCH, la, lb, ...)         \
    switch ((la) * 7 + (lb)) {                           \
    case 0: LAUNCH<0, 0>(__VA_ARGS__); break; \
    case 1: LAUNCH<0, 1>(__VA_ARGS__); break; \
    case 2: LAUNCH<0, 2>(__VA_ARGS__); break; \
    case 3: LAUNCH<0, 3>(__VA_ARGS__); break; \
    case 4: LAUNCH<0, 4>(__VA_ARGS__); break; \
    case 5: LAUNCH<0, 5>(__VA_ARGS__); break; \
    case 6: LAUNCH<0, 6>(__VA_ARGS__); break; \
    case 7: LAUNCH<1, 0>(__VA_ARGS__); break; \
    case 8: LAUNCH<1, 1>(__VA_ARGS__); break; \
    case 9: LAUNCH<1, 2>(__VA_ARGS__); break; \
    case 10: LAUNCH<1, 3>(__VA_ARGS__); break; \
    case 11: LAUNCH<1, 4>(__VA_ARGS__); break; \
    case 12: LAUNCH<1, 5>(__VA_ARGS__); break; \
    case 13: LAUNCH<1, 6>(__VA_ARGS__); break; \
    case 14: LAUNCH<2, 0>(__VA_ARGS__); break; \
    case 15: LAUNCH<2, 1>(__VA_ARGS__); break; \
    case 16: LAUNCH<2, 2>(__VA_ARGS__); break; \
    case 17: LAUNCH<2, 3>(__VA_ARGS__); break; \
    case 18: LAUNCH<2, 4>(__VA_ARGS__); break; \
    case 19: LAUNCH<2, 5>(__VA_ARGS__); break; \
    case 20: LAUNCH<2, 6>(__VA_ARGS__); break; \
    case 21: LAUNCH<3, 0>(__VA_ARGS__); break; \
    case 22: LAUNCH<3, 1>(__VA_ARGS__); break; \
    case 23: LAUNCH<3, 2>(__VA_ARGS__); break; \
    case 24: LAUNCH<3, 3>(__VA_ARGS__); break; \
    case 25: LAUNCH<3, 4>(__VA_ARGS__); break; \
    case 26: LAUNCH<3, 5>(__VA_ARGS__); break; \
    case 27: LAUNCH<3, 6>(__VA_ARGS__); break; \
    case 28: LAUNCH<4, 0>(__VA_ARGS__); break; \
    case 29: LAUNCH<4, 1>(__VA_ARGS__); break; \
    case 30: LAUNCH<4, 2>(__VA_ARGS__); break; \
    case 31: LAUNCH<4, 3>(__VA_ARGS__); break; \
    case 32: LAUNCH<4, 4>(__VA_ARGS__); break; \
    case 33: LAUNCH<4, 5>(__VA_ARGS__); break; \
    case 34: LAUNCH<4, 6>(__VA_ARGS__); break; \
    case 35: LAUNCH<5, 0>(__VA_ARGS__); break; \
    case 36: LAUNCH<5, 1>(__VA_ARGS__); break; \
    case 37: LAUNCH<5, 2>(__VA_ARGS__); break; \
    case 38: LAUNCH<5, 3>(__VA_ARGS__); break; \
    case 39: LAUNCH<5, 4>(__VA_ARGS__); break; \
    case 40: LAUNCH<5, 5>(__VA_ARGS__); break; \
    case 41: LAUNCH<5, 6>(__VA_ARGS__); break; \
    case 42: LAUNCH<6, 0>(__VA_ARGS__); break; \
    case 43: LAUNCH<6, 1>(__VA_ARGS__); break; \
    case 44: LAUNCH<6, 2>(__VA_ARGS__); break; \
    case 45: LAUNCH<6, 3>(__VA_ARGS__); break; \
    case 46: LAUNCH<6, 4>(__VA_ARGS__); break; \
    case 47: LAUNCH<6, 5>(__VA_ARGS__); break; \
    default: LAUNCH<6, 6>(__VA_ARGS__); break; \
    }

namespace mdx {

mdx_status onebody_launch(mdx_ctx *c, const mdx_shells *sh, const PairRec *pairs, int32_t npair, int la, int lb,
                          bool cart, double *S, double *T, hipStream_t s)
{
    if (npair == 0 || (!S && !T)) return MDX_OK;
    hipEvent_t ev1;
    MDX_TRY(prof_open(c, s, &ev1));
    OneBodyArgs a{};
    a.pairs = pairs;
    a.npair = npair;
    a.center = sh->center;
    a.expo = sh->exponent;
    a.coef = sh->coef;
    a.Ca = c->solid + c->solid_off[la];
    a.Cb = c->solid + c->solid_off[lb];
    a.S = S;
    a.T = T;
    MDX_ONEBODY_SWITCH7(launch_onebody, la, lb, a, cart, s)
    HIP_TRY2(hipGetLastError());
    if (ev1) HIP_TRY2(hipEventRecord(ev1, s));
    return MDX_OK;
}

mdx_status nuclear_lane_launch(mdx_ctx *c, const mdx_shells *sh, const PairRec *pairs, int32_t npair, int la,
                               int lb, bool cart, int32_t ncharge, const double *charges, double *V, hipStream_t s)
{
    if (npair == 0) return MDX_OK;
    hipEvent_t ev1;
    MDX_TRY(prof_open(c, s, &ev1));
    NuclearArgs a{};
    a.pairs = pairs;
    a.npair = npair;
    a.center = sh->center;
    a.expo = sh->exponent;
    a.coef = sh->coef;
    a.charges = charges;
    a.ncharge = ncharge;
    a.boys = c->boys;
    a.Ca = c->solid + c->solid_off[la];
    a.Cb = c->solid + c->solid_off[lb];
    a.V = V;
    if (la + lb <= 6) {
        MDX_NUCLEAR_LANE_SWITCH(launch_nuclear, la, lb, a, cart, s)
    } else {
        MDX_NUCLEAR_WAVE_SWITCH(launch_nuclear_wave, la, lb, a, cart, s)
    }
    HIP_TRY2(hipGetLastError());
    if (ev1) HIP_TRY2(hipEventRecord(ev1, s));
    return MDX_OK;
}

}  // namespace mdx

extern "C" mdx_status mdx_one_body_batch(mdx_ctx *c, const mdx_shells *sh, int32_t npair, const int32_t *pairs,
                                         int flags, double *S, double *T, void *ws, size_t ws_bytes,
                                         mdx_stream_t stream)
{
    int l[2];
    mdx_status st = check_pairs(c, sh, npair, pairs, flags, l);
    if (st != MDX_OK) return st;
    if (npair == 0 || (!S && !T)) return MDX_OK;
    hipStream_t s = (hipStream_t)stream;
    MDX_TRY(stage_pairs(c, sh, npair, pairs, ws, ws_bytes, s, "mdx_one_body_batch"));
    return onebody_launch(c, sh, (const PairRec *)ws, npair, l[0], l[1], (flags & MDX_CARTESIAN) != 0, S, T, s);
}

extern "C" size_t mdx_nuclear_workspace_size(mdx_ctx *c, const mdx_shells *sh, int32_t npair, const int32_t *pairs,
                                             int32_t ncharge, int flags)
{
    int l[2];
    if (check_pairs(c, sh, npair, pairs, flags, l) != MDX_OK) return 0;
    if (ncharge < 0) {
        fail(MDX_EINVAL, "negative charge count");
        return 0;
    }
    return al256((size_t)npair * sizeof(PairRec)) + 256;
}

extern "C" mdx_status mdx_nuclear_batch(mdx_ctx *c, const mdx_shells *sh, int32_t npair, const int32_t *pairs,
                                        int32_t ncharge, const double *charges, int flags, double *V, void *ws,
                                        size_t ws_bytes, mdx_stream_t stream)
{
    int l[2];
    mdx_status st = check_pairs(c, sh, npair, pairs, flags, l);
    if (st != MDX_OK) return st;
    if (ncharge < 0) return fail(MDX_EINVAL, "negative charge count");
    if (ncharge > 0 && !charges) return fail(MDX_EINVAL, "null charge array");
    if (npair == 0) return MDX_OK;
    hipStream_t s = (hipStream_t)stream;
    if (!V) return fail(MDX_EINVAL, "mdx_nuclear_batch: null output");
    MDX_TRY(stage_pairs(c, sh, npair, pairs, ws, ws_bytes, s, "mdx_nuclear_batch"));
    return nuclear_lane_launch(c, sh, (const PairRec *)ws, npair, l[0], l[1], (flags & MDX_CARTESIAN) != 0, ncharge,
                               charges, V, s);
}

extern "C" mdx_status mdx_one_body_prepare(mdx_ctx *c, const mdx_shells *sh, int32_t npair, const int32_t *pairs,
                                           int flags, mdx_batch **out)
{
    if (!out) return fail(MDX_EINVAL, "mdx_one_body_prepare: null handle pointer");
    *out = nullptr;
    int l[2];
    MDX_TRY(check_pairs(c, sh, npair, pairs, flags, l));
    mdx_batch *b = new mdx_batch;
    mdx_status st = batch_init(b, c, sh, B_ONEBODY, flags);
    b->la = l[0];
    b->lb = l[1];
    b->npair = npair;
    const bool cart = (flags & MDX_CARTESIAN) != 0;
    b->out_doubles = npair > 0 ? (int64_t)npair * nfunc(l[0], cart) * nfunc(l[1], cart) : 0;
    if (st == MDX_OK && npair > 0) {
        std::vector<PairRec> pr;
        onebody_records(sh, npair, pairs, pr);
        st = batch_tables(b, pr.size() * sizeof(PairRec));
        if (st == MDX_OK && hipMemcpy(b->dtab, pr.data(), pr.size() * sizeof(PairRec), hipMemcpyHostToDevice) !=
                                hipSuccess)
            st = fail(MDX_EDEVICE, "mdx_one_body_prepare: copy of the pair records failed");
    }
    if (st != MDX_OK) {
        mdx_batch_destroy(b);
        return st;
    }
    *out = b;
    return MDX_OK;
}

extern "C" mdx_status mdx_one_body_run(const mdx_batch *b, const mdx_shells *sh, double *S, double *T, void *ws,
                                       size_t ws_bytes, mdx_stream_t stream)
{
    MDX_TRY(batch_check(b, sh, B_ONEBODY, ws, ws_bytes, "mdx_one_body_run"));
    return onebody_launch(b->c, sh, (const PairRec *)b->dtab, b->npair, b->la, b->lb,
                          (b->flags & MDX_CARTESIAN) != 0, S, T, (hipStream_t)stream);
}

extern "C" mdx_status mdx_nuclear_prepare(mdx_ctx *c, const mdx_shells *sh, int32_t npair, const int32_t *pairs,
                                          int32_t ncharge, int flags, mdx_batch **out)
{
    if (!out) return fail(MDX_EINVAL, "mdx_nuclear_prepare: null handle pointer");
    *out = nullptr;
    int l[2];
    MDX_TRY(check_pairs(c, sh, npair, pairs, flags, l));
    if (ncharge < 0) return fail(MDX_EINVAL, "negative charge count");
    const bool cart = (flags & MDX_CARTESIAN) != 0;
    mdx_batch *b = new mdx_batch;
    mdx_status st = batch_init(b, c, sh, B_NUC, flags);
    b->la = l[0];
    b->lb = l[1];
    b->npair = npair;
    b->ncharge = ncharge;
    b->out_doubles = npair > 0 ? (int64_t)npair * nfunc(l[0], cart) * nfunc(l[1], cart) : 0;
    if (st == MDX_OK && npair > 0) {
        std::vector<PairRec> pr;
        onebody_records(sh, npair, pairs, pr);
        st = batch_tables(b, pr.size() * sizeof(PairRec));
        if (st == MDX_OK && hipMemcpy(b->dtab, pr.data(), pr.size() * sizeof(PairRec), hipMemcpyHostToDevice) !=
                                hipSuccess)
            st = fail(MDX_EDEVICE, "mdx_nuclear_prepare: copy of the pair records failed");
    }
    if (st != MDX_OK) {
        mdx_batch_destroy(b);
        return st;
    }
    *out = b;
    return MDX_OK;
}

extern "C" mdx_status mdx_nuclear_run(const mdx_batch *b, const mdx_shells *sh, const double *charges, double *V,
                                      void *ws, size_t ws_bytes, mdx_stream_t stream)
{
    MDX_TRY(batch_check(b, sh, B_NUC, ws, ws_bytes, "mdx_nuclear_run"));
    if (b->npair == 0) return MDX_OK;
    if (b->ncharge > 0 && !charges) return fail(MDX_EINVAL, "mdx_nuclear_run: null charge array");
    if (!V) return fail(MDX_EINVAL, "mdx_nuclear_run: null output");
    hipStream_t s = (hipStream_t)stream;
    return nuclear_lane_launch(b->c, sh, (const PairRec *)b->dtab, b->npair, b->la, b->lb,
                               (b->flags & MDX_CARTESIAN) != 0, b->ncharge, charges, V, s);
}
