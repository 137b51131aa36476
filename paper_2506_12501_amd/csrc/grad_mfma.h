// grad_mfma.h -- backward kernel: centre derivatives of a class of shellsets
// contracted with an adjoint W (the paper has no derivatives; this follows
// from differentiating the Gaussian of Eq. (1)).
//
// For one side (the "derivative side", pair ab with centres A and B)
//   d/dA_i phi_a = 2 zeta_a phi_{a+1_i} - a_i phi_{a-1_i},
// and the product of that with phi_b is again a Hermite expansion about the
// same P, of order l_a + l_b + 1.  The pair-data kernel stores these six
// expansions (A_x, A_y, A_z, B_x, B_y, B_z) as matrices Hd[d][(kb, p)][ab].
// For a shellset (I, J) with adjoint block W[ab][cd] the six derivatives are
//   g_d = sum_{ab,cd} W[ab][cd] sum_p Hd[d][p][ab] sum_q [p+q] H_ket[q][cd]
//       = sum_{(kb,p), ab} Hd[d][(kb,p)][ab] X'[(kb,p)][ab],
//   X'[(kb,p)][ab] = sum_{kk,q} [p+q]_{kb,kk} H'[kk][q][ab],
//   H'[kk][q][ab]  = sum_cd H_ket[kk][q][cd] W[ab][cd]   (adjoint folded into the ket).
// X' is the ket transform of Eq. (32) with the adjoint-folded ket, for bra
// Hermite rows up to order l_a + l_b + 1 ([r] of Eq. (31) to L + 1), with
// the partial early contraction of the terminal ket Hermites (Eqs. (38)-(40)).
// The fold and the ket transform run on the FP64 matrix cores; the six
// Frobenius products with Hd are VALU dot products over the accumulator tiles.
// A second launch with the roles swapped gives the other pair's centres.
#pragma once

#include <algorithm>

#include "mfma_common.h"

namespace mdx {

constexpr int GRAD_NWP_MAX = 48;   // other side's column stride bound (36 Cartesian functions)

template <int LD, int LW, int NTN, int MTW, int NW, int WPE, int LAY>
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
    constexpr int NP = NTN * 16;
    constexpr int NT = 64 * NW;
    constexpr int MK = (NTPAD + 15) / 16;   // 16-row tiles of the adjoint fold
    constexpr int HKR = (NTPAD * GRAD_NWP_MAX + NT - 1) / NT;
    constexpr bool YSER = MTW * NTN * 4 + MTW * KT > 48;   // large accumulator set: sweep columns one branch each
    constexpr int NQCT = (NW * MTW * 16) / NHD + 2;   // bound on quartets per chunk (host: nqmax)
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
    const int nw = a.nw, nwq = (nw + 3) & ~3, nwp = a.nwp;

    extern __shared__ double smem[];
    double *cube = smem;                       // nqmax tables
    double *S = cube + CB::words(nqmax);       // [kkmax][nqmax][D]
    double *PQ = S + kkmax * nqmax * D;        // [kkmax][nqmax][4]
    double *Wt = PQ + kkmax * nqmax * 4;       // [kkmax]
    double *Hk = Wt + kkmax;                   // [NTPAD][NP]   adjoint-folded ket block
    double *Tk = Hk + NTPAD * NP;              // [4*KT][NP]    adjoint-folded terminal matrix
    double *Wl = Tk + 4 * KT * NP;             // [NP][nwq]     adjoint block W[i][j]
    double *Hr = Wl + NP * nwq;                // [NTPAD][nwp]  raw ket block
    double *red = Hr + NTPAD * nwp;            // [NW][6]
    int *kq = (int *)(red + NW * 6);           // [NTPAD]
    int *kt = kq + NTPAD;                      // [4*KT]
    int *rowt = kt + 4 * KT;                   // [NHD] table offsets of the derivative-side rows

    for (int k = tid; k < NHD; k += NT) rowt[k] = CB::off(k);
    for (int k = tid; k < NTPAD; k += NT) kq[k] = k < NKN ? CB::off(k) : 0;
    for (int k = tid; k < 4 * KT; k += NT) kt[k] = k < NKT ? CB::off(NKN + k) : 0;
    {
        const double *Wg = a.W + (int64_t)I * a.wsI + (int64_t)J * a.wsJ;
        for (int e = tid; e < NP * nwq; e += NT) {
            const int i = e / nwq, j = e - i * nwq;
            Wl[e] = (i < a.nd && j < nw) ? Wg[(int64_t)i * a.wsd + (int64_t)j * a.wsw] : 0.0;
        }
    }
    __syncthreads();
    // terminal matrix folded with the adjoint: Tk[q][i] = sum_j T[q][j] W[i][j]
    for (int e = tid; e < 4 * KT * NP; e += NT) {
        const int q = e / NP, i = e - q * NP;
        double v = 0.0;
        for (int j = 0; j < nw; ++j) v = fma(a.Tw[q * nwp + j], Wl[i * nwq + j], v);
        Tk[e] = v;
    }

    const PrimRec *bp = a.dside.prim + (int64_t)I * a.dside.kmax;
    const PrimRec *kp = a.wside.prim + (int64_t)J * a.wside.kmax;
    const double *HkG = a.wside.H + (int64_t)J * a.wside.pair_stride;
    const double *Hd = a.dside.H + (int64_t)I * a.dside.pair_stride;
    const int64_t dstride = a.dside.pair_stride / 6;

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
        d4 acc[MTW][NTN];
        double Y[MTW][KT];
#pragma unroll
        for (int tt = 0; tt < MTW; ++tt) {
#pragma unroll
            for (int n = 0; n < NTN; ++n) acc[tt][n] = d4{0.0, 0.0, 0.0, 0.0};
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

        for (int kk = 0; kk < nkk; ++kk) {
            __syncthreads();   // previous reads of the table, Hr and Hk are complete
            double hv[HKR > 0 ? HKR : 1];
            {
                const double *src = HkG + (int64_t)kk * RPB * nwp;   // non-terminal rows are contiguous
#pragma unroll
                for (int i = 0; i < HKR; ++i) {
                    const int e = tid + i * NT;
                    hv[i] = e < NTPAD * nwp ? src[e] : 0.0;
                }
            }
            {
                const double *Sk = S + kk * nqmax * D, *PQk = PQ + kk * nqmax * 4;
                ysweeps<CB, NW, YSER>(cube, Sk, PQk, NQ, NQ, nqmax, w, lane, std::make_integer_sequence<int, NW>{});
                __syncthreads();
                xsweeps<CB, NW, NQCT, YSER>(cube, PQk, NQ, NQ, nqmax, w, lane, std::make_integer_sequence<int, NW>{});
            }
#pragma unroll
            for (int i = 0; i < HKR; ++i) {
                const int e = tid + i * NT;
                if (e < NTPAD * nwp) Hr[e] = hv[i];
            }
            __syncthreads();
            // adjoint fold on MFMA: Hk[q][i] = sum_j Hr[q][j] W[i][j]  (M = q, K = j, N = i)
            for (int it = w; it < MK * NTN; it += NW) {
                const int m = it / NTN, n = it - m * NTN;
                const int qa = 16 * m + c;
                d4 f = d4{0.0, 0.0, 0.0, 0.0};
                for (int s = 0; s < (nwq >> 2); ++s) {
                    const int j = 4 * s + g;
                    const double av = qa < NTPAD ? Hr[qa * nwp + j] : 0.0;
                    f = mfma(av, Wl[(16 * n + c) * nwq + j], f);
                }
#pragma unroll
                for (int r = 0; r < 4; ++r) {
                    const int q = 16 * m + 4 * r + g;
                    if (q < NTPAD) Hk[q * NP + 16 * n + c] = f[r];
                }
            }
            __syncthreads();

            // ket transform on MFMA over the non-terminal Hermites
#pragma unroll 2
            for (int s = 0; s < KS; ++s) {
                const int qo = kq[4 * s + g];
                double bv[NTN];
#pragma unroll
                for (int n = 0; n < NTN; ++n) bv[n] = Hk[(4 * s + g) * NP + 16 * n + c];
#pragma unroll
                for (int tt = 0; tt < MTW; ++tt) {
                    const double av = cube[abase[tt] + qo];
#pragma unroll
                    for (int n = 0; n < NTN; ++n) acc[tt][n] = mfma(av, bv[n], acc[tt][n]);
                }
            }
            // terminal Hermites: early contraction over the ket primitives
            const double wt = Wt[kk];
#pragma unroll
            for (int s = 0; s < KT; ++s) {
                const int to = kt[4 * s + g];
#pragma unroll
                for (int tt = 0; tt < MTW; ++tt) Y[tt][s] = fma(wt, cube[abase[tt] + to], Y[tt][s]);
            }
        }

        // terminal block: X' += Y T'
#pragma unroll
        for (int s = 0; s < KT; ++s) {
            double bv[NTN];
#pragma unroll
            for (int n = 0; n < NTN; ++n) bv[n] = Tk[(4 * s + g) * NP + 16 * n + c];
#pragma unroll
            for (int tt = 0; tt < MTW; ++tt)
#pragma unroll
                for (int n = 0; n < NTN; ++n) acc[tt][n] = mfma(Y[tt][s], bv[n], acc[tt][n]);
        }

        // Frobenius products with the six derivative expansions (rows past the
        // last primitive are zero in Hd)
#pragma unroll
        for (int tt = 0; tt < MTW; ++tt) {
            const int T = tile0 + tt;
            if (T < MT) {
#pragma unroll
                for (int n = 0; n < NTN; ++n)
#pragma unroll
                    for (int r = 0; r < 4; ++r) {
                        const double x = acc[tt][n][r];
                        const double *h = Hd + (int64_t)(16 * T + 4 * r + g) * NP + 16 * n + c;
#pragma unroll
                        for (int d = 0; d < 6; ++d) gacc[d] = fma(h[d * dstride], x, gacc[d]);
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

template <int LD, int LW, int NTN, int MTW, int NW, int LAY>
static size_t grad_lds_bytes(int nqmax, int kkmax, int nwq, int nwp)
{
    constexpr int L = LD + LW + 1, D = L + 1;
    constexpr int NTPAD = round_up(nherm(LW - 1), 4);
    constexpr int KT = round_up(ncart(LW), 4) / 4;
    constexpr int NP = NTN * 16;
    const size_t dbl = (size_t)Cube<D, LAY>::words(nqmax) + (size_t)kkmax * nqmax * (D + 4) + kkmax + (size_t)NTPAD * NP +
                       (size_t)4 * KT * NP + (size_t)NP * nwq + (size_t)NTPAD * nwp + (size_t)NW * 6;
    return dbl * 8 + (size_t)(NTPAD + 4 * KT + nherm(LD + 1)) * 4;
}

template <int LD, int LW, int NTN, int MTW, int NW, int WPE, int LAY>
static bool launch_grad(const GradArgs &a0, int nblocks, hipStream_t s)
{
    GradArgs a = a0;
    constexpr int NHD = nherm(LD + 1);
    if (a.nwp > GRAD_NWP_MAX || a.nd > NTN * 16) return false;
    a.nqmax = std::min(a.dside.kmax, (NW * MTW * 16) / NHD + 2);
    const size_t lds = grad_lds_bytes<LD, LW, NTN, MTW, NW, LAY>(a.nqmax, a.wside.kmax, (a.nw + 3) & ~3, a.nwp);
    if (lds > 160 * 1024) return false;
    auto kern = eri_grad_kernel<LD, LW, NTN, MTW, NW, WPE, LAY>;
    static size_t lds_set = 0;   // largest dynamic LDS granted to this instance so far
    if (lds > 64 * 1024 && lds > lds_set) {
        if (hipFuncSetAttribute((const void *)kern, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds) != hipSuccess)
            return false;
        lds_set = lds;
    }
    hipLaunchKernelGGL(kern, dim3(nblocks), dim3(64 * NW), lds, s, a);
    return true;
}

// Dispatch over an instance list X(LD, LW, NTN, MTW, NW, WPE, LAY); several
// tile shapes or table layouts for one key are variants 1, 2, ... in listing
// order.
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
#define MDX_GRAD_COUNT(ld, lw, ntn, mtw, nw, wpe, lay) \
    if (k.LD == ld && k.LW == lw && k.NTN == ntn) ++n;
#define MDX_GRAD_TRY(ld, lw, ntn, mtw, nw, wpe, lay)                            \
    if (k.LD == ld && k.LW == lw && k.NTN == ntn && ++n == variant)             \
        return launch_grad<ld, lw, ntn, mtw, nw, wpe, lay>(a, nblocks, s);

}  // namespace mdx
