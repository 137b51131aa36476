// grad_mfma.h -- backward kernel: centre derivatives of a class of shellsets
// contracted with an adjoint W (the paper has no derivatives; this follows
// from differentiating the Gaussian of Eq. (1)).
//
// For one side (the "derivative side", pair ab with centres A and B)
//   d/dA_i phi_a = 2 zeta_a phi_{a+1_i} - a_i phi_{a-1_i},
// and the product of that with phi_b is again a Hermite expansion about the
// same P, of order l_a + l_b + 1.  The pair-data kernel stores these six
// expansions (A_x, A_y, A_z, B_x, B_y, B_z) as matrices Hd[d][ab][(kb, p)].
// For a shellset (I, J) with adjoint block W[ab][cd] the six derivatives are
//   g_d = sum_{ab,cd} W[ab][cd] sum_p Hd[d][ab][p] X[p][cd],
//   X[(kb,p)][cd] = sum_{kk,q} [p+q]_{kb,kk} H_ket[kk][q][cd],
// X being the ket transform of Eq. (32) for bra Hermite rows up to order
// l_a + l_b + 1 ([r] of Eq. (31) to L + 1), with the partial early
// contraction of the terminal ket Hermites (Eqs. (38)-(40)).  The kernel
// forms X transposed on the FP64 matrix cores, X^T = H_ket^T [p+q]^T: the
// accumulator tiles of X^T are then, element for element, the right operand
// of the adjoint fold X'^T = W X^T, which runs once per shellset after the
// ket primitives; the six Frobenius products of X' with Hd are VALU dot
// products over its accumulator tiles.  A second launch with the roles
// swapped gives the other pair's centres.
#pragma once

#include <algorithm>

#include "mfma_common.h"

namespace mdx {

// NTN / NTW: 16-function tiles of the derivative side / the other side;
// MTW: 16-row tiles per wave per chunk; NW waves; LAY: table layout; KP: ket
// primitives per sweep round
template <int LD, int LW, int NTN, int NTW, int MTW, int NW, int WPE, int LAY, int KP>
__global__ void __launch_bounds__(64 * NW) __attribute__((amdgpu_waves_per_eu(WPE)))
eri_grad_kernel(GradArgs a)
{
    constexpr int L = LD + LW + 1;   // the derivative side reaches order LD + 1
    typedef Cube<L + 1, LAY> CB;
    constexpr int D = L + 1, CUBE = CB::SIZE;
    constexpr int NHD = nherm(LD + 1);   // derivative-side rows per primitive pair
    constexpr int NKN = nherm(LW - 1);
    constexpr int NTPAD = round_up(NKN, 4);
    constexpr int KS = NTPAD / 4;
    constexpr int NKT = ncart(LW);
    constexpr int KT = round_up(NKT, 4) / 4;
    constexpr int RPB = NTPAD + NKT;
    constexpr int NP = NTN * 16;       // derivative-side functions, padded
    constexpr int NQW = NTW * 16;      // other side's functions, padded (= its column stride)
    constexpr int WLD = NQW + 1;       // adjoint row stride in LDS (odd: rows spread over banks)
    constexpr int NT = 64 * NW;
    constexpr int HKR = (NTPAD * NQW + NT - 1) / NT;
    constexpr int TKR = (4 * KT * NQW + NT - 1) / NT;
    // large accumulator set or long columns: sweep the columns one branch each
    constexpr bool YSER = MTW * NTW * 4 + MTW * KT > 48 || D > 12;
    constexpr int NQCT = (NW * MTW * 16) / NHD + 2;         // bound on quartets per chunk (host: nqmax)
    static_assert(KP >= 1 && KP * NQCT <= 64 && KP * NQCT <= CB::QMAX, "tables of one sweep round");
    const int tid = threadIdx.x;
    const int w = tid >> 6, lane = tid & 63, g = lane >> 4, c = lane & 15;

    // one shellset per workgroup; derivative-side pair I changes slowest so
    // that the workgroups resident on an XCD share its Hd in L2
    const int t = xcd_tile(blockIdx.x, gridDim.x);
    const int I = t / a.nJ, J = t - I * a.nJ;

    const int npb = a.dside.nprim[I];
    const int nkk = a.wside.nprim[J];
    const int nrows = npb * NHD;
    const int MT = (nrows + 15) >> 4;
    const int nch = (MT + NW * MTW - 1) / (NW * MTW);
    const int nqmax = a.nqmax;
    const int kkmax = a.wside.kmax;
    const int nw = a.nw;

    extern __shared__ double smem[];
    double *cube = smem;                          // KP blocks of nqmax tables
    double *S = cube + CB::words(KP * nqmax);     // [kkmax][nqmax][D]
    double *PQ = S + kkmax * nqmax * D;           // [kkmax][nqmax][4]
    double *Wt = PQ + kkmax * nqmax * 4;          // [kkmax]
    double *Hk = Wt + kkmax;                      // [KP][NTPAD][NQW]  ket rows of a sweep round
    double *Tk = Hk + KP * NTPAD * NQW;           // [4*KT][NQW]       terminal matrix of the other side
    double *Wl = Tk + 4 * KT * NQW;               // [NP][WLD]         adjoint block W[ab][cd]
    double *red = Wl + NP * WLD;                  // [NW][6]
    int *kq = (int *)(red + NW * 6);              // [NTPAD]
    int *kt = kq + NTPAD;                         // [4*KT]
    int *rowt = kt + 4 * KT;                      // [NHD] table offsets of the derivative-side rows

    for (int k = tid; k < NHD; k += NT) rowt[k] = CB::off(k);
    for (int k = tid; k < NTPAD; k += NT) kq[k] = k < NKN ? CB::off(k) : 0;
    for (int k = tid; k < 4 * KT; k += NT) kt[k] = k < NKT ? CB::off(NKN + k) : 0;
    {
        const double *Wg = a.W + (int64_t)I * a.wsI + (int64_t)J * a.wsJ;
        for (int e = tid; e < NP * WLD; e += NT) {
            const int i = e / WLD, j = e - i * WLD;
            Wl[e] = (i < a.nd && j < nw) ? Wg[(int64_t)i * a.wsd + (int64_t)j * a.wsw] : 0.0;
        }
#pragma unroll
        for (int i = 0; i < TKR; ++i) {
            const int e = tid + i * NT;
            if (e < 4 * KT * NQW) Tk[e] = a.Tw[e];
        }
    }

    const PrimRec *bp = a.dside.prim + (int64_t)I * a.dside.kmax;
    const PrimRec *kp = a.wside.prim + (int64_t)J * a.wside.kmax;
    const double *HkG = a.wside.H + (int64_t)J * a.wside.pair_stride;
    const double *Hd = a.dside.H + (int64_t)I * a.dside.pair_stride;
    const int64_t dstride = a.dside.pair_stride / 6;
    const int rpbd = (int)(dstride / NP);   // row stride of Hd[d][ab][.]

    double gacc[6];
#pragma unroll
    for (int d = 0; d < 6; ++d) gacc[d] = 0.0;

    for (int ch = 0; ch < nch; ++ch) {
        const int tile0 = ch * NW * MTW + w * MTW;
        const int row_lo = ch * NW * MTW * 16;
        const int row_hi = min(nrows, row_lo + NW * MTW * 16);
        const int kb_lo = row_lo / NHD, kb_hi = (row_hi - 1) / NHD;
        const int NQ = kb_hi - kb_lo + 1;

        __syncthreads();   // tables visible; previous chunk done with LDS
        int abase[MTW];
#pragma unroll
        for (int tt = 0; tt < MTW; ++tt) {
            const int row = 16 * (tile0 + tt) + c;
            int off = 0;
            if (row < nrows) {
                const int kb = row / NHD, h = row - kb * NHD;
                off = (kb - kb_lo) * CUBE + rowt[h];
            }
            abase[tt] = off;
        }
        d4 acc[MTW][NTW];   // X^T tiles: [cd][row]
        double Y[MTW][KT];
#pragma unroll
        for (int tt = 0; tt < MTW; ++tt) {
#pragma unroll
            for (int n = 0; n < NTW; ++n) acc[tt][n] = d4{0.0, 0.0, 0.0, 0.0};
#pragma unroll
            for (int s = 0; s < KT; ++s) Y[tt][s] = 0.0;
        }

        // [0]^(m) of every primitive quartet of the chunk, Eq. (27)
        for (int e = tid; e < NQ * nkk; e += NT) {
            const int kk = e / NQ, q = e - kk * NQ;
            const PrimRec B = bp[kb_lo + q];
            const PrimRec K = kp[kk];
            const double pq = B.p + K.p;
            const double ypq = rsqrt_d(pq);   // 1/sqrt(p+q)
            const double rho = B.p * K.p * (ypq * ypq);
            const double X = B.Px - K.Px, Yv = B.Py - K.Py, Z = B.Pz - K.Pz;
            double F[D];
            boys_eval<L>(rho * (X * X + Yv * Yv + Z * Z), F, a.boys);
            double f = B.ws * K.ws * ypq;
            const double m2r = -2.0 * rho;
            double *Sq = S + (kk * nqmax + q) * D;
#pragma unroll
            for (int m = 0; m <= L; ++m) {
                Sq[m] = f * F[m];
                f *= m2r;
            }
            double *pq4 = PQ + (kk * nqmax + q) * 4;
            pq4[0] = X;
            pq4[1] = Yv;
            pq4[2] = Z;
            if (q == 0) Wt[kk] = K.wt;
        }

        // rounds of KP ket primitives: one set of sweeps fills the tables of all of them
        for (int kk0 = 0; kk0 < nkk; kk0 += KP) {
            const int nk = min(KP, nkk - kk0);
            __syncthreads();   // previous round's reads of the tables and Hk are complete
            // ket rows of this round (non-terminal rows are contiguous): global
            // loads now, LDS stores after the recursion
            double hv[KP][HKR];
#pragma unroll
            for (int j = 0; j < KP; ++j)
#pragma unroll
                for (int i = 0; i < HKR; ++i) {
                    const int e = tid + i * NT;
                    hv[j][i] = (j < nk && e < NTPAD * NQW) ? HkG[(int64_t)(kk0 + j) * RPB * NQW + e] : 0.0;
                }
            {
                // the sweeps gate the whole workgroup: raised wave priority, as in the
                // forward kernel
                __builtin_amdgcn_s_setprio(2);
                const double *Sk = S + kk0 * nqmax * D, *PQk = PQ + kk0 * nqmax * 4;
                ysweeps<CB, NW, YSER>(cube, Sk, PQk, NQ, nk * nqmax, nqmax, w, lane,
                                      std::make_integer_sequence<int, NW>{});
                __syncthreads();
                xsweeps<CB, NW, KP * NQCT, YSER>(cube, PQk, NQ, nk * nqmax, nqmax, w, lane,
                                                 std::make_integer_sequence<int, NW>{});
                __builtin_amdgcn_s_setprio(0);
            }
#pragma unroll
            for (int j = 0; j < KP; ++j)
#pragma unroll
                for (int i = 0; i < HKR; ++i) {
                    const int e = tid + i * NT;
                    if (j < nk && e < NTPAD * NQW) Hk[j * NTPAD * NQW + e] = hv[j][i];
                }
            __syncthreads();

#pragma unroll
            for (int j = 0; j < KP; ++j) {
                if (j >= nk) break;   // uniform
                const double *cj = cube + j * nqmax * CUBE;
                const double *Hj = Hk + j * NTPAD * NQW;
                // X^T += H_ket^T [p+q]^T over the non-terminal Hermites: the ket
                // rows are the left operand (M = cd), the table gather the right (N = rows)
#pragma unroll 2
                for (int s = 0; s < KS; ++s) {
                    const int qo = kq[4 * s + g];
                    double bv[NTW];
#pragma unroll
                    for (int n = 0; n < NTW; ++n) bv[n] = Hj[(4 * s + g) * NQW + 16 * n + c];
#pragma unroll
                    for (int tt = 0; tt < MTW; ++tt) {
                        const double av = cj[abase[tt] + qo];
#pragma unroll
                        for (int n = 0; n < NTW; ++n) acc[tt][n] = mfma(bv[n], av, acc[tt][n]);
                    }
                }
                // terminal Hermites: early contraction over the ket primitives
                const double wt = Wt[kk0 + j];
#pragma unroll
                for (int s = 0; s < KT; ++s) {
                    const int to = kt[4 * s + g];
#pragma unroll
                    for (int tt = 0; tt < MTW; ++tt) Y[tt][s] = fma(wt, cj[abase[tt] + to], Y[tt][s]);
                }
            }
        }

        // terminal block: X^T += T^T Y^T
#pragma unroll
        for (int s = 0; s < KT; ++s) {
            double bv[NTW];
#pragma unroll
            for (int n = 0; n < NTW; ++n) bv[n] = Tk[(4 * s + g) * NQW + 16 * n + c];
#pragma unroll
            for (int tt = 0; tt < MTW; ++tt)
#pragma unroll
                for (int n = 0; n < NTW; ++n) acc[tt][n] = mfma(bv[n], Y[tt][s], acc[tt][n]);
        }

        // per row tile: adjoint fold X'^T = W X^T on MFMA -- lane (c, g) holds
        // X^T[16n + 4r + g][row c] in acc[tt][n][r], which is the right operand
        // of K step 4n + r -- then the Frobenius products with the six
        // derivative expansions (rows past the last primitive are zero in Hd).
        // The Hd values of a group of HG function tiles (all of them for up to
        // two tiles; one at a time beyond, for registers) are loaded together
        // before any is used.
        constexpr int HG = NTN <= 2 ? NTN : 1;
#pragma unroll
        for (int tt = 0; tt < MTW; ++tt) {
            const int T = tile0 + tt;
            if (T < MT) {
                const double *h0 = Hd + (int64_t)g * rpbd + 16 * T + c;
#pragma unroll
                for (int m0 = 0; m0 < NTN; m0 += HG) {
                    double hv[HG][4][6];
#pragma unroll
                    for (int mm = 0; mm < HG; ++mm)
#pragma unroll
                        for (int r = 0; r < 4; ++r)
#pragma unroll
                            for (int d = 0; d < 6; ++d)
                                hv[mm][r][d] = h0[d * dstride + (int64_t)(16 * (m0 + mm) + 4 * r) * rpbd];
                    d4 O[HG];
#pragma unroll
                    for (int mm = 0; mm < HG; ++mm) {
                        O[mm] = d4{0.0, 0.0, 0.0, 0.0};
#pragma unroll
                        for (int n = 0; n < NTW; ++n)
#pragma unroll
                            for (int r = 0; r < 4; ++r)
                                O[mm] = mfma(Wl[(16 * (m0 + mm) + c) * WLD + 16 * n + 4 * r + g], acc[tt][n][r], O[mm]);
                    }
#pragma unroll
                    for (int mm = 0; mm < HG; ++mm)
#pragma unroll
                        for (int r = 0; r < 4; ++r)
#pragma unroll
                            for (int d = 0; d < 6; ++d) gacc[d] = fma(hv[mm][r][d], O[mm][r], gacc[d]);
                }
            }
        }
    }

    // workgroup sum of the six derivatives, then the caller's twelve slots
#pragma unroll
    for (int d = 0; d < 6; ++d) {
        double v = gacc[d];
#pragma unroll
        for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off);
        gacc[d] = v;
    }
    if (lane == 0)
#pragma unroll
        for (int d = 0; d < 6; ++d) red[w * 6 + d] = gacc[d];
    __syncthreads();
    if (tid < 12 && ((a.wmask >> tid) & 1)) {
        double v = 0.0;
        for (int k = 0; k < 6; ++k) {
            double gk = 0.0;
            for (int ww = 0; ww < NW; ++ww) gk += red[ww * 6 + k];
            v += (double)a.M[tid][k] * gk;
        }
        a.G[(int64_t)I * a.gsI + (int64_t)J * a.gsJ + (int64_t)tid * a.gss] = v;
    }
}

template <int LD, int LW, int NTN, int NTW, int MTW, int NW, int LAY, int KP>
static size_t grad_lds_bytes(int nqmax, int kkmax)
{
    constexpr int L = LD + LW + 1, D = L + 1;
    constexpr int NTPAD = round_up(nherm(LW - 1), 4);
    constexpr int KT = round_up(ncart(LW), 4) / 4;
    constexpr int NP = NTN * 16, NQW = NTW * 16;
    const size_t dbl = (size_t)Cube<D, LAY>::words(KP * nqmax) + (size_t)kkmax * nqmax * (D + 4) + kkmax +
                       (size_t)KP * NTPAD * NQW + (size_t)4 * KT * NQW + (size_t)NP * (NQW + 1) + (size_t)NW * 6;
    return dbl * 8 + (size_t)(NTPAD + 4 * KT + nherm(LD + 1)) * 4;
}

template <int LD, int LW, int NTN, int NTW, int MTW, int NW, int WPE, int LAY, int KP>
static bool launch_grad(const GradArgs &a0, int nblocks, hipStream_t s)
{
    GradArgs a = a0;
    constexpr int NHD = nherm(LD + 1);
    if (a.nwp != NTW * 16 || a.nw > NTW * 16 || a.nd > NTN * 16) return false;
    a.nqmax = std::min(a.dside.kmax, (NW * MTW * 16) / NHD + 2);
    const size_t lds = grad_lds_bytes<LD, LW, NTN, NTW, MTW, NW, LAY, KP>(a.nqmax, a.wside.kmax);
    if (lds > 160 * 1024) return false;
    auto kern = eri_grad_kernel<LD, LW, NTN, NTW, MTW, NW, WPE, LAY, KP>;
    static size_t lds_set = 0;   // largest dynamic LDS granted to this instance so far
    if (lds > 64 * 1024 && lds > lds_set) {
        if (hipFuncSetAttribute((const void *)kern, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds) != hipSuccess)
            return false;
        lds_set = lds;
    }
    hipLaunchKernelGGL(kern, dim3(nblocks), dim3(64 * NW), lds, s, a);
    return true;
}

// Dispatch over an instance list X(LD, LW, NTN, NTW, MTW, NW, WPE, LAY, KP);
// several tile shapes, table layouts or sweep rounds for one key are variants
// 1, 2, ... in listing order.
#define MDX_GRAD_DISPATCH(SUFFIX, LIST)                                                          \
    int eri_grad_variants_##SUFFIX(const GradKey &k)                                             \
    {                                                                                            \
        int n = 0;                                                                               \
        LIST(MDX_GRAD_COUNT)                                                                     \
        return n;                                                                                \
    }                                                                                            \
    bool eri_grad_launch_##SUFFIX(const GradKey &k, const GradArgs &a, int nblocks, int variant, \
                                  hipStream_t s)                                                 \
    {                                                                                            \
        int n = 0;                                                                               \
        LIST(MDX_GRAD_TRY)                                                                       \
        return false;                                                                            \
    }
#define MDX_GRAD_COUNT(ld, lw, ntn, ntw, mtw, nw, wpe, lay, kp) \
    if (k.LD == ld && k.LW == lw && k.NTN == ntn && k.NTW == ntw) ++n;
#define MDX_GRAD_TRY(ld, lw, ntn, ntw, mtw, nw, wpe, lay, kp)                           \
    if (k.LD == ld && k.LW == lw && k.NTN == ntn && k.NTW == ntw && ++n == variant)     \
        return launch_grad<ld, lw, ntn, ntw, mtw, nw, wpe, lay, kp>(a, nblocks, s);

}  // namespace mdx
