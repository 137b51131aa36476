// mfma_common.h -- pieces shared by the matrix-core integral kernels:
// the FP64 MFMA wrapper and the one-axis sweeps of the Hermite recursion
// (Eq. (31)) over a dense (L+1)^3 cube in LDS.
#pragma once

#include <utility>

#include "eri_common.h"
#include "kernels.h"

namespace mdx {

typedef double d4 __attribute__((ext_vector_type(4)));

__device__ __forceinline__ d4 mfma(double a, double b, d4 c)
{
    return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0);
}

// cube offset of Hermite k (t*D*D + u*D + v)
template <int D>
__host__ __device__ constexpr int cube_off(int k)
{
    const Tuv r = herm_tuv(k);
    return (r.t * D + r.u) * D + r.v;
}

template <int L, int LK>
struct KetOffsets {
    static constexpr int D = L + 1;
    static constexpr int NKN = nherm(LK - 1);
    static constexpr int NTPAD = round_up(NKN, 4);
    static constexpr int NKT = ncart(LK);
    static constexpr int NKTP = round_up(NKT, 4);
    int q[NTPAD > 0 ? NTPAD : 1];   // non-terminal ket Hermites (0 for padding)
    int t[NKTP];                    // terminal ket Hermites (0 for padding)
    constexpr KetOffsets() : q{}, t{}
    {
        for (int k = 0; k < NTPAD; ++k) q[k] = k < NKN ? cube_off<D>(k) : 0;
        for (int k = 0; k < NKTP; ++k) t[k] = k < NKT ? cube_off<D>(NKN + k) : 0;
    }
};

template <int N>
__device__ __forceinline__ int pick4(const int (&v)[N], int base, int g)
{
    // v[base + g] for a wave-varying g in 0..3 with compile-time base
    const int a0 = v[base], a1 = v[base + 1], a2 = v[base + 2], a3 = v[base + 3];
    return (g & 2) ? ((g & 1) ? a3 : a2) : ((g & 1) ? a1 : a0);
}

// [r]^(0) of one primitive quartet, Eq. (31), as three one-axis sweeps over
// the table cube[(t*D + u)*D + v] (D = L+1).  Each sweep handles columns of a
// compile-time length, so it is fully unrolled: no predication, no wasted
// work on short columns, recursion state in registers.
//   z, y sweep: per v, raise z to v in registers, then y:
//               [0 u v]^(m), m <= M-u (M = L-v) -> cube position (m, u, v)
//   x sweep:  per (u, v), [t u v]^(0), t <= M (M = L-u-v) -> (t, u, v)
// Intermediate columns are stored at (m, u, v) and overwritten in place by
// the lane that owns them.
template <int D, int M>
__device__ __forceinline__ void ysweep(double *__restrict__ cv /* cube + v */, const double *__restrict__ S, double Y,
                                       double Z)
{
    // z first: [0 0 v]^(m), m <= M, for v = L - M, from [0]^(m) (registers only)
    constexpr int L = D - 1, V = L - M;
    double c[D], p[D];
#pragma unroll
    for (int m = 0; m < D; ++m) {
        c[m] = S[m];
        p[m] = 0.0;
    }
#pragma unroll
    for (int v = 1; v <= V; ++v) {
        double n[D];
#pragma unroll
        for (int m = 0; m <= L - v; ++m) n[m] = v > 1 ? fma((double)(v - 1), p[m + 1], Z * c[m + 1]) : Z * c[m + 1];
#pragma unroll
        for (int m = 0; m <= L - v; ++m) {
            p[m] = c[m];
            c[m] = n[m];
        }
        p[L - v + 1] = c[L - v + 1];
    }
    // then y: [0 u v]^(m), m <= M - u
#pragma unroll
    for (int m = 0; m <= M; ++m) {
        cv[(m * D) * D] = c[m];
        p[m] = 0.0;
    }
#pragma unroll
    for (int u = 1; u <= M; ++u) {
        double n[M + 1];
#pragma unroll
        for (int m = 0; m <= M - u; ++m) n[m] = u > 1 ? fma((double)(u - 1), p[m + 1], Y * c[m + 1]) : Y * c[m + 1];
#pragma unroll
        for (int m = 0; m <= M - u; ++m) cv[(m * D + u) * D] = n[m];
#pragma unroll
        for (int m = 0; m <= M - u; ++m) {
            p[m] = c[m];
            c[m] = n[m];
        }
        p[M - u + 1] = c[M - u + 1];
    }
}

template <int D, int M>
__device__ __forceinline__ void xsweep(double *__restrict__ cuv /* cube + u*D + v */, double X)
{
    double c[M + 1], p[M + 1];
#pragma unroll
    for (int m = 0; m <= M; ++m) {
        c[m] = cuv[(m * D) * D];
        p[m] = 0.0;
    }
#pragma unroll
    for (int t = 1; t <= M; ++t) {
        double n[M + 1];
#pragma unroll
        for (int m = 0; m <= M - t; ++m) n[m] = t > 1 ? fma((double)(t - 1), p[m + 1], X * c[m + 1]) : X * c[m + 1];
        cuv[(t * D) * D] = n[0];
#pragma unroll
        for (int m = 0; m <= M - t; ++m) {
            p[m] = c[m];
            c[m] = n[m];
        }
        p[M - t + 1] = c[M - t + 1];
    }
}

// Sweep work of one wave.  Wave W owns the z/y columns v with v % NW == W and
// the x passes of order M with (L - M) % NW == W; lanes take quartets (y) or
// (quartet, column) pairs (x).  All z/y columns of a wave sit in one block
// under a single lane guard, so the scheduler can interleave their independent
// recursion chains; idle lanes stay masked (a fully masked 16-lane group costs
// no FP64 pipe time).  Requires NQ <= 64.
template <int D, int NW, int W, int M>
__device__ __forceinline__ void ycol(double *cq, const double *Sq, double Y, double Z)
{
    constexpr int v = D - 1 - M;
    if constexpr (v % NW == W) ysweep<D, M>(cq + v, Sq, Y, Z);
}

template <int D, int NW, int W, int... Ms>
__device__ __forceinline__ void ywave(double *cube, const double *S, const double *PQ, int NQ, int lane,
                                      std::integer_sequence<int, Ms...>)
{
    constexpr int CUBE = D * D * D;
    if (lane >= NQ) return;
    double *cq = cube + lane * CUBE;
    const double *Sq = S + lane * D;
    const double Y = PQ[lane * 4 + 1], Z = PQ[lane * 4 + 2];
    (ycol<D, NW, W, Ms>(cq, Sq, Y, Z), ...);
}

template <int D, int NW, int W, int NQCT, int M>
__device__ __forceinline__ void xcols(double *cube, const double *PQ, int NQ, int lane)
{
    constexpr int L = D - 1, s = L - M, CUBE = D * D * D;
    if constexpr (M > 0 && s % NW == W) {   // order 0 columns are complete after the y sweep
        constexpr int R = (NQCT * (s + 1) + 63) / 64;
        const int n = NQ * (s + 1);
#pragma unroll
        for (int r = 0; r < R; ++r) {
            const int e = lane + 64 * r;
            if (e < n) {
                const int q = e / (s + 1), v = e - q * (s + 1), u = s - v;
                xsweep<D, M>(cube + q * CUBE + u * D + v, PQ[q * 4]);
            }
        }
    }
}

template <int D, int NW, int W, int NQCT, int... Ms>
__device__ __forceinline__ void xwave(double *cube, const double *PQ, int NQ, int lane,
                                      std::integer_sequence<int, Ms...>)
{
    (xcols<D, NW, W, NQCT, Ms>(cube, PQ, NQ, lane), ...);
}

// One z/y column per branch region: the chains of a wave run one after the
// other, which keeps fewer registers live next to a large accumulator set.
template <int D, int NW, int M>
__device__ __forceinline__ void ycol_branch(double *cube, const double *S, const double *PQ, int NQ, int w, int lane)
{
    constexpr int v = D - 1 - M, CUBE = D * D * D;
    if (w == v % NW && lane < NQ)
        ysweep<D, M>(cube + lane * CUBE + v, S + lane * D, PQ[lane * 4 + 1], PQ[lane * 4 + 2]);
}

template <int D, int NW, int... Ms>
__device__ __forceinline__ void ysweeps_serial(double *cube, const double *S, const double *PQ, int NQ, int w,
                                               int lane, std::integer_sequence<int, Ms...>)
{
    (ycol_branch<D, NW, Ms>(cube, S, PQ, NQ, w, lane), ...);
}

// z/y sweeps of all live quartets (every wave calls this; wave w does its
// share).  SER selects the column-per-branch form for register-heavy kernels.
template <int D, int NW, bool SER, int... Ws>
__device__ __forceinline__ void ysweeps(double *cube, const double *S, const double *PQ, int NQ, int w,
                                        int lane, std::integer_sequence<int, Ws...>)
{
    if constexpr (SER)
        ysweeps_serial<D, NW>(cube, S, PQ, NQ, w, lane, std::make_integer_sequence<int, D>{});
    else
        ((w == Ws ? ywave<D, NW, Ws>(cube, S, PQ, NQ, lane, std::make_integer_sequence<int, D>{}) : void()), ...);
}

// x sweep of all columns of order M in a branch region of its own
template <int D, int NW, int M>
__device__ __forceinline__ void xorder_branch(double *cube, const double *PQ, int NQ, int w, int lane)
{
    constexpr int L = D - 1, s = L - M, CUBE = D * D * D;
    if (M > 0 && w == s % NW)
        for (int e = lane; e < NQ * (s + 1); e += 64) {
            const int q = e / (s + 1), v = e - q * (s + 1), u = s - v;
            xsweep<D, M>(cube + q * CUBE + u * D + v, PQ[q * 4]);
        }
}

template <int D, int NW, int... Ms>
__device__ __forceinline__ void xsweeps_serial(double *cube, const double *PQ, int NQ, int w, int lane,
                                               std::integer_sequence<int, Ms...>)
{
    (xorder_branch<D, NW, Ms>(cube, PQ, NQ, w, lane), ...);
}

// x sweeps (after the z/y sweeps of all waves are visible); SER as for ysweeps
template <int D, int NW, int NQCT, bool SER, int... Ws>
__device__ __forceinline__ void xsweeps(double *cube, const double *PQ, int NQ, int w, int lane,
                                        std::integer_sequence<int, Ws...>)
{
    if constexpr (SER)
        xsweeps_serial<D, NW>(cube, PQ, NQ, w, lane, std::make_integer_sequence<int, D>{});
    else
        ((w == Ws ? xwave<D, NW, Ws, NQCT>(cube, PQ, NQ, lane, std::make_integer_sequence<int, D>{}) : void()), ...);
}

}  // namespace mdx
