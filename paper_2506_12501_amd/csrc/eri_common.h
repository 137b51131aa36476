// eri_common.h -- compile-time tables for the integral kernels.
#pragma once

#include "boys_device.h"
#include "mdx_internal.h"

namespace mdx {

// ---------------------------------------------------------------------------
// Hermite auxiliary recursion, Eq. (31):
//   [r+1_i]^(m) = r_i [r-1_i]^(m+1) + (P_i - Q_i) [r]^(m+1)
// Values live in slots  slot(k, m) = m*nherm(L) + k  (k = Hermite index).
// The plan lists, level by level, every (k, m) with |r_k| + m <= L and the
// slots it reads; level 0 holds [0]^(m) (Eq. (27)).
// ---------------------------------------------------------------------------
struct RStep {
    short dst, src1, src2;   // src2 < 0: no r_i term
    signed char axis;        // i
    signed char coef;        // r_i - 1 ... i.e. the r_i of the lowered index
};

__host__ __device__ constexpr int rplan_count(int L)
{
    int n = 0;
    for (int lev = 1; lev <= L; ++lev) n += ncart(lev) * (L - lev + 1);
    return n;
}

template <int L>
struct RPlan {
    static constexpr int NH = nherm(L);
    static constexpr int N = rplan_count(L);
    RStep s[N > 0 ? N : 1];
    constexpr RPlan() : s{}
    {
        int n = 0;
        for (int lev = 1; lev <= L; ++lev)
            for (int k = nherm(lev - 1); k < nherm(lev); ++k) {
                const Tuv r = herm_tuv(k);
                const int ax = r.t > 0 ? 0 : (r.u > 0 ? 1 : 2);
                const int ri = ax == 0 ? r.t : (ax == 1 ? r.u : r.v);
                const int k1 = herm_index(r.t - (ax == 0), r.u - (ax == 1), r.v - (ax == 2));
                const int k2 = ri > 1 ? herm_index(r.t - 2 * (ax == 0), r.u - 2 * (ax == 1), r.v - 2 * (ax == 2)) : -1;
                for (int m = 0; m <= L - lev; ++m) {
                    s[n].dst = (short)(m * NH + k);
                    s[n].src1 = (short)((m + 1) * NH + k1);
                    s[n].src2 = (short)(k2 >= 0 ? (m + 1) * NH + k2 : -1);
                    s[n].axis = (signed char)ax;
                    s[n].coef = (signed char)(ri - 1);
                    ++n;
                }
            }
    }
};

template <int L>
__device__ __forceinline__ void r_recursion(const double *__restrict__ S, double X, double Y, double Z,
                                            double *__restrict__ R /*[(L+1)*nherm(L)]*/)
{
    constexpr RPlan<L> plan{};
    constexpr int NH = nherm(L);
#pragma unroll
    for (int m = 0; m <= L; ++m) R[m * NH] = S[m];
    const double XPQ[3] = {X, Y, Z};
#pragma unroll
    for (int i = 0; i < plan.N; ++i) {
        const RStep e = plan.s[i];
        double v = XPQ[e.axis] * R[e.src1];
        if (e.src2 >= 0) v = fma((double)e.coef, R[e.src2], v);
        R[e.dst] = v;
    }
}

// Rs[k] += [r_k]^(0) for every |r_k| <= L: the recursion of Eq. (31) taken
// order by order, m = L-1 down to 0, in one table T of the order-(m+1)
// values.  Within an order the entries are rewritten in decreasing |r|, so
// each step reads order-(m+1) values that are still in place; the order-0
// values go straight into Rs.  A lane holds N_H(L-1) values instead of the
// (L+1) N_H(L) of r_recursion.
struct RAccStep {
    short dst, src1, src2;   // src2 < 0: no r_i term; kind 1: dst = 0, src1 = m
    signed char axis, coef, kind;   // kind 0: T[dst] = ..., 1: T[0] = S[m], 2: Rs[dst] += ...
};

__host__ __device__ constexpr int racc_count(int L)
{
    int n = 0;
    for (int m = L - 1; m >= 1; --m) n += nherm(L - m) - 1 + 1;
    return n + nherm(L) - 1;
}

template <int L>
struct RAccPlan {
    static constexpr int N = racc_count(L);
    RAccStep s[N > 0 ? N : 1];
    constexpr RAccPlan() : s{}
    {
        int n = 0;
        auto step = [&](int k, int kind) {
            const Tuv r = herm_tuv(k);
            const int ax = r.t > 0 ? 0 : (r.u > 0 ? 1 : 2);
            const int ri = ax == 0 ? r.t : (ax == 1 ? r.u : r.v);
            s[n].dst = (short)k;
            s[n].src1 = (short)herm_index(r.t - (ax == 0), r.u - (ax == 1), r.v - (ax == 2));
            s[n].src2 = (short)(ri > 1 ? herm_index(r.t - 2 * (ax == 0), r.u - 2 * (ax == 1), r.v - 2 * (ax == 2)) : -1);
            s[n].axis = (signed char)ax;
            s[n].coef = (signed char)(ri - 1);
            s[n].kind = (signed char)kind;
            ++n;
        };
        for (int m = L - 1; m >= 1; --m) {
            for (int lev = L - m; lev >= 1; --lev)
                for (int k = nherm(lev - 1); k < nherm(lev); ++k) step(k, 0);
            s[n].dst = 0;
            s[n].src1 = (short)m;
            s[n].src2 = -1;
            s[n].axis = 0;
            s[n].coef = 0;
            s[n].kind = 1;
            ++n;
        }
        for (int k = 1; k < nherm(L); ++k) step(k, 2);
    }
};

template <int L>
__device__ __forceinline__ void r_accumulate(const double *__restrict__ S, double X, double Y, double Z,
                                             double *__restrict__ Rs /*[nherm(L)]*/)
{
    Rs[0] += S[0];
    if constexpr (L > 0) {
        constexpr RAccPlan<L> plan{};
        double T[nherm(L - 1)];
        T[0] = S[L];
        const double XPQ[3] = {X, Y, Z};
#pragma unroll
        for (int i = 0; i < plan.N; ++i) {
            const RAccStep e = plan.s[i];
            if (e.kind == 1) {
                T[0] = S[e.src1];
            } else {
                double v = XPQ[e.axis] * T[e.src1];
                if (e.src2 >= 0) v = fma((double)e.coef, T[e.src2], v);
                if (e.kind == 0) T[e.dst] = v;
                else Rs[e.dst] += v;
            }
        }
    }
}

// Hermite index of the sum of two Hermite triples, as a table [ka][kb]
template <int LA, int LB>
struct SumTab {
    short idx[nherm(LA) > 0 ? nherm(LA) : 1][nherm(LB) > 0 ? nherm(LB) : 1];
    constexpr SumTab() : idx{}
    {
        for (int a = 0; a < nherm(LA); ++a)
            for (int b = 0; b < nherm(LB); ++b) {
                const Tuv x = herm_tuv(a), y = herm_tuv(b);
                idx[a][b] = (short)herm_index(x.t + y.t, x.u + y.u, x.v + y.v);
            }
    }
};

}  // namespace mdx
