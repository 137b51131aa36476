// eri_mfma.h -- the matrix-core integral kernel body (one shellset per
// workgroup), its LDS footprint and its instance list; shared by the plain
// launches and the persistent work-queue launches.
//
// One workgroup of NW waves evaluates one shellset (bra pair I, ket pair J).
// The Hermite-to-AO transforms of the paper's Eq. (36) chain are dense
// contractions and run as MFMA GEMMs:
//
//  ket transform (Eq. (32), with the partial early contraction of Sec. 2.2.2,
//  Eqs. (38)-(40)):
//     X[(kb,p)][cd] = sum_{kk, q non-terminal} [p+q]^(0)_{kb,kk} H_ket[kk][q][cd]
//                   + sum_{q terminal} Y[(kb,p)][q] T[q][cd],
//     Y[(kb,p)][q]  = sum_kk w_kk [p+q]^(0)_{kb,kk}          (VALU, registers)
//  M = rows (bra primitive, bra Hermite), K = (ket primitive, ket Hermite),
//  N = ket functions.  The A operand is gathered from [r]^(0) held in LDS
//  (Eq. (25): [p|q] is never stored, the sign lives in H_ket).
//
//  bra transform (Eq. (33)):  out[ab][cd] = sum_rows H_bra[ab][row] X[row][cd]
//  The accumulator tile of X is used directly as the B operand: register r of
//  lane (c, g) holds X[row 4r+g][col c], which is B[k=g][n=c] of k-step r, so
//  the K order of the bra GEMM is permuted to match (no data movement).
//
// [r]^(0) follows the recursion of Eq. (31) in three one-axis sweeps (z, then
// y per column v, then x per column (u, v)), each of compile-time length and
// unrolled in registers.  The table is an (L+1)^3 cube indexed (t,u,v) with
// bank-padded strides, so [p+q] sits at offset(p) + offset(q): per-lane row
// offsets plus compile-time ket offsets.
#pragma once

#include <algorithm>

#include "mfma_common.h"

namespace mdx {

// One shellset (bra pair I, ket pair J) per workgroup; every thread of the
// workgroup calls this with the same (I, J); nI = bra pairs of ket J.
template <int LB, int LK, int NTAB, int NTCD, int NTG, int MTW, int NW, bool GB, int LAY, int KP, bool DIG = false>
__device__ __forceinline__ void eri_mfma_shellset(const EriArgs &a, const int I, const int J, const int nI)
{
    constexpr int L = LB + LK;
    typedef Cube<L + 1, LAY> CB;
    constexpr int D = L + 1, CUBE = CB::SIZE;
    constexpr int NUV = (L + 1) * (L + 2) / 2;
    constexpr int NHB = GB ? ncart(LB) : nherm(LB);
    constexpr int HB0 = GB ? nherm(LB - 1) : 0;
    constexpr int NKN = nherm(LK - 1);
    constexpr int NTPAD = round_up(NKN, 4);
    constexpr int KS = NTPAD / 4;
    constexpr int NKT = ncart(LK);
    constexpr int KT = round_up(NKT, 4) / 4;
    constexpr int RPB = NTPAD + NKT;
    constexpr int NCDP = NTCD * 16, NABP = NTAB * 16;
    constexpr int NG = NTCD / NTG;
    constexpr int GW = NTG * 16;
    constexpr int NT = 64 * NW;
    constexpr int HKR = (NTPAD * GW + NT - 1) / NT;   // staged ket values per thread
    constexpr int TKR = (4 * KT * GW + NT - 1) / NT;  // staged terminal-matrix values per thread
    constexpr bool YSER = MTW * NTG * 4 + MTW * KT > 48;   // large accumulator set: sweep columns one branch each
    constexpr int NQCT = GB ? 1 : (NW * MTW * 16) / NHB + 2;   // bound on quartets per chunk (host: nqmax)
    static_assert(NTCD % NTG == 0, "cd tiles must split into groups");
    static_assert(KP >= 1 && KP * NQCT <= 64 && KP * NQCT <= CB::QMAX, "tables of one sweep round");
    const int tid = threadIdx.x;
    const int w = tid >> 6, lane = tid & 63, g = lane >> 4, c = lane & 15;


    const int npb = a.bra.nprim[I];
    const int nkk = a.ket.nprim[J];
    const int nbk = GB ? 1 : npb;
    const int nrows = nbk * NHB;
    const int MT = (nrows + 15) >> 4;
    const int nch = (MT + NW * MTW - 1) / (NW * MTW);
    const int nqmax = a.nqmax;

    // With several column groups the [r]^(0) table may stay resident across
    // groups, so the cross-wave reduction gets a region of its own.
    constexpr bool SEPRED = NG > 1;
    // reduction buffer: with one column group every wave's whole partial bra
    // transform (overlaying the free cube), else waves 1.. one output tile at a time
    constexpr int RED = SEPRED ? (NW - 1) * NTG * 256 : NW * NTAB * NTG * 256;
    extern __shared__ double smem[];
    double *cube = smem;   // KP blocks of nqmax tables: ket primitive kk0 + j, bra primitive q at slot j*nqmax + q
    const int tabs = CB::words(KP * nqmax);
    const int cube_words = (SEPRED || tabs > RED) ? tabs : RED;
    double *red = SEPRED ? smem + cube_words : cube;
    const int kkmax = a.ket.kmax;
    double *S = smem + cube_words + (SEPRED ? RED : 0);   // [kkmax][nqmax][D]
    double *PQ = S + kkmax * nqmax * D;                  // [kkmax][nqmax][4]
    double *Wt = PQ + kkmax * nqmax * 4;                 // [kkmax] terminal weights
    double *Hk = Wt + kkmax;                             // [KP][NTPAD][GW]
    double *Tk = Hk + KP * NTPAD * GW;                   // [4*KT][GW]
    int *kq = (int *)(Tk + 4 * KT * GW);                 // [NTPAD] table offsets, non-terminal ket
    int *kt = kq + NTPAD;                                // [4*KT] table offsets, terminal ket
    int *oab = kt + 4 * KT;                              // [NABP] output offsets (copies of a.om)
    int *ocd = oab + NABP;                               // [NCDP]
    int *rowt = ocd + NCDP;                              // [NHB] table offsets of the bra Hermite rows
    double *dgb = (double *)(rowt + round_up(NHB, 2));   // DIG: [NABP] Db of bra pair I, [NCDP] Dk of ket pair J
    double *dgk = dgb + NABP;

    if constexpr (DIG) {   // the densities of this shellset, read at the store (after many barriers)
        for (int k = tid; k < NABP; k += NT) dgb[k] = (a.dig.Jk && k < a.nab) ? a.dig.Db[I + a.dig.nb * k] : 0.0;
        for (int k = tid; k < NCDP; k += NT) dgk[k] = (a.dig.Jb && k < a.ncd) ? a.dig.Dk[J + a.dig.nk * k] : 0.0;
    }
    for (int k = tid; k < NHB; k += NT) rowt[k] = CB::off(HB0 + k);
    for (int k = tid; k < NTPAD; k += NT) kq[k] = k < NKN ? CB::off(k) : 0;
    for (int k = tid; k < 4 * KT; k += NT) kt[k] = k < NKT ? CB::off(NKN + k) : 0;
    if constexpr (NW > 1) {   // the cross-wave epilogues look output offsets up in LDS
        for (int k = tid; k < NABP; k += NT) oab[k] = k < a.nab ? a.om.oab[k] : 0;
        for (int k = tid; k < NCDP; k += NT) ocd[k] = k < a.ncd ? a.om.ocd[k] : 0;
    }

    const PrimRec *bp = a.bra.prim + (int64_t)I * a.bra.kmax;
    const PrimRec *kp = a.ket.prim + (int64_t)J * a.ket.kmax;
    const double *Hb = a.bra.H + (int64_t)I * a.bra.pair_stride;
    const double *HkG = a.ket.H + (int64_t)J * a.ket.pair_stride;

    const bool resident = (nkk == 1 && nch == 1);
    const int64_t obase = a.om.count ? a.om.obase[J] : (int64_t)J * a.om.sJ;
    const int64_t omult = a.om.count ? (int64_t)nI : a.om.mult;

    for (int grp = 0; grp < NG; ++grp) {
        for (int ch = 0; ch < nch; ++ch) {
            const int tile0 = ch * NW * MTW + w * MTW;
            const int row_lo = ch * NW * MTW * 16;
            const int row_hi = min(nrows, row_lo + NW * MTW * 16);
            const int kb_lo = GB ? 0 : row_lo / NHB;
            const int kb_hi = GB ? 0 : (row_hi - 1) / NHB;
            const int NQ = kb_hi - kb_lo + 1;

            __syncthreads();   // Hermite table visible; previous users of LDS done
            // terminal ket matrix of this column group; with several groups the
            // loads are issued now and stored after [0]^(m), hiding their latency
            double tv[TKR];
#pragma unroll
            for (int i = 0; i < TKR; ++i) {
                const int e = tid + i * NT;
                tv[i] = e < 4 * KT * GW ? a.Tket[(e / GW) * NCDP + grp * GW + (e % GW)] : 0.0;
                if constexpr (NG == 1)
                    if (e < 4 * KT * GW) Tk[e] = tv[i];
            }
            int abase[MTW];
#pragma unroll
            for (int tt = 0; tt < MTW; ++tt) {
                const int row = 16 * (tile0 + tt) + c;
                int off = 0;
                if (row < nrows) {
                    const int kb = GB ? 0 : row / NHB;
                    const int h = GB ? row : row - kb * NHB;
                    off = (kb - kb_lo) * CUBE + rowt[h];
                }
                abase[tt] = off;
            }
            d4 acc[MTW][NTG];
            double Y[MTW][KT];
#pragma unroll
            for (int tt = 0; tt < MTW; ++tt) {
#pragma unroll
                for (int n = 0; n < NTG; ++n) acc[tt][n] = d4{0.0, 0.0, 0.0, 0.0};
#pragma unroll
                for (int s = 0; s < KT; ++s) Y[tt][s] = 0.0;
            }

            const bool fresh = !(resident && grp > 0);
            if (fresh) {
                // [0]^(m) of every primitive quartet of the chunk, Eq. (27), times the
                // primitive weights; a single-function solid bra sums its primitives here
                for (int e = tid; e < NQ * nkk; e += NT) {
                    const int kk = e / NQ, q = e - kk * NQ;
                    double Sm[D];
#pragma unroll
                    for (int m = 0; m <= L; ++m) Sm[m] = 0.0;
                    const PrimRec K = kp[kk];
                    double X = 0.0, Yv = 0.0, Z = 0.0;
                    const int b0 = GB ? 0 : kb_lo + q, b1 = GB ? npb : kb_lo + q + 1;
                    for (int ib = b0; ib < b1; ++ib) {
                        const PrimRec B = bp[ib];
                        const double pq = B.p + K.p;
                        const double ypq = rsqrt_d(pq);   // 1/sqrt(p+q)
                        const double rho = B.p * K.p * (ypq * ypq);
                        X = B.Px - K.Px;
                        Yv = B.Py - K.Py;
                        Z = B.Pz - K.Pz;
                        double F[D];
                        boys_eval<L, false>(rho * (X * X + Yv * Yv + Z * Z), F, a.boys);
                        double f = B.ws * K.ws * ypq;
                        const double m2r = -2.0 * rho;
#pragma unroll
                        for (int m = 0; m <= L; ++m) {
                            Sm[m] = fma(f, F[m], Sm[m]);
                            f *= m2r;
                        }
                    }
                    double *Sq = S + (kk * nqmax + q) * D;
#pragma unroll
                    for (int m = 0; m <= L; ++m) Sq[m] = Sm[m];
                    double *pq4 = PQ + (kk * nqmax + q) * 4;
                    pq4[0] = X;
                    pq4[1] = Yv;
                    pq4[2] = Z;
                    if (q == 0) Wt[kk] = K.wt;
                }
            }

            if constexpr (NG > 1) {
#pragma unroll
                for (int i = 0; i < TKR; ++i) {
                    const int e = tid + i * NT;
                    if (e < 4 * KT * GW) Tk[e] = tv[i];
                }
            }

            // rounds of KP ket primitives: one set of sweeps fills the tables of
            // all of them (more busy lanes per instruction, fewer barriers)
            for (int kk0 = 0; kk0 < nkk; kk0 += KP) {
                const int nk = min(KP, nkk - kk0);
                __syncthreads();   // previous round's reads of the tables / Hk are complete
                // ket blocks of this round: global loads now, LDS stores after the recursion
                double hv[KP][HKR];
#pragma unroll
                for (int j = 0; j < KP; ++j) {
#pragma unroll
                    for (int i = 0; i < HKR; ++i) {
                        const int e = tid + i * NT;
                        hv[j][i] = (j < nk && e < NTPAD * GW)
                                       ? HkG[(int64_t)(kk0 + j) * RPB * NCDP + grp * GW + (e / GW) * NCDP + (e % GW)]
                                       : 0.0;
                    }
                }
                if (fresh) {
                    // one-axis sweeps of Eq. (31): z and y per column v, then x per (u, v).
                    // The whole workgroup waits for them at the next barrier, while the
                    // other resident workgroup's matrix instructions can wait: the sweeps
                    // issue at a raised wave priority.
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
                        if (j < nk && e < NTPAD * GW) Hk[j * NTPAD * GW + e] = hv[j][i];
                    }
                __syncthreads();

#pragma unroll
                for (int j = 0; j < KP; ++j) {
                    if (j >= nk) break;   // uniform
                    const double *cj = cube + j * nqmax * CUBE;
                    const double *Hj = Hk + j * NTPAD * GW;
                    // ket transform on MFMA over the non-terminal Hermites
#pragma unroll 2
                    for (int s = 0; s < KS; ++s) {
                        const int qo = kq[4 * s + g];
                        double bv[NTG];
#pragma unroll
                        for (int n = 0; n < NTG; ++n) bv[n] = Hj[(4 * s + g) * GW + 16 * n + c];
#pragma unroll
                        for (int tt = 0; tt < MTW; ++tt) {
                            const double av = cj[abase[tt] + qo];
#pragma unroll
                            for (int n = 0; n < NTG; ++n) acc[tt][n] = mfma(av, bv[n], acc[tt][n]);
                        }
                    }
                    // terminal Hermites: early contraction over ket primitives
                    const double wt = Wt[kk0 + j];
#pragma unroll
                    for (int s = 0; s < KT; ++s) {
                        const int to = kt[4 * s + g];
#pragma unroll
                        for (int tt = 0; tt < MTW; ++tt) Y[tt][s] = fma(wt, cj[abase[tt] + to], Y[tt][s]);
                    }
                }
            }

            // terminal block: X += Y T
#pragma unroll
            for (int s = 0; s < KT; ++s) {
                double bv[NTG];
#pragma unroll
                for (int n = 0; n < NTG; ++n) bv[n] = Tk[(4 * s + g) * GW + 16 * n + c];
#pragma unroll
                for (int tt = 0; tt < MTW; ++tt)
#pragma unroll
                    for (int n = 0; n < NTG; ++n) acc[tt][n] = mfma(Y[tt][s], bv[n], acc[tt][n]);
            }

            d4 O[NTAB][NTG];
#pragma unroll
            for (int mm = 0; mm < NTAB; ++mm)
#pragma unroll
                for (int n = 0; n < NTG; ++n) O[mm][n] = d4{0.0, 0.0, 0.0, 0.0};
            // bra transform: O += H_bra X, K order permuted to the accumulator layout;
            // the next tile's H_bra values are fetched while this tile multiplies
            double hb[2][4][NTAB];
            {
                const int T = min(tile0, MT - 1);
#pragma unroll
                for (int r = 0; r < 4; ++r)
#pragma unroll
                    for (int mm = 0; mm < NTAB; ++mm) hb[0][r][mm] = Hb[(int64_t)(16 * T + 4 * r + g) * NABP + 16 * mm + c];
            }
#pragma unroll
            for (int tt = 0; tt < MTW; ++tt) {
                const int cur = tt & 1, nxt = cur ^ 1;
                if (tt + 1 < MTW) {
                    const int T = min(tile0 + tt + 1, MT - 1);
#pragma unroll
                    for (int r = 0; r < 4; ++r)
#pragma unroll
                        for (int mm = 0; mm < NTAB; ++mm)
                            hb[nxt][r][mm] = Hb[(int64_t)(16 * T + 4 * r + g) * NABP + 16 * mm + c];
                }
                if (tile0 + tt < MT) {
#pragma unroll
                    for (int r = 0; r < 4; ++r)
#pragma unroll
                        for (int mm = 0; mm < NTAB; ++mm)
#pragma unroll
                            for (int n = 0; n < NTG; ++n) O[mm][n] = mfma(hb[cur][r][mm], acc[tt][n][r], O[mm][n]);
                }
            }

            // sum the waves' partial bra transforms and store this column group
            // (a shellset with several row chunks accumulates through the output)
            if constexpr (NW == 1) {   // one wave: nothing to reduce
#pragma unroll
                for (int mm = 0; mm < NTAB; ++mm)
#pragma unroll
                    for (int n = 0; n < NTG; ++n)
#pragma unroll
                        for (int r = 0; r < 4; ++r) {
                            const int ab = 16 * mm + 4 * r + g;
                            const int cd = grp * GW + 16 * n + c;
                            if constexpr (DIG)
                                digest_block(a.dig, I, J, ab, cd, ab < a.nab, cd < a.ncd, O[mm][n][r], g, c, dgk[cd], dgb[ab]);
                            else if (ab < a.nab && cd < a.ncd) {   // one wave: offsets from the arguments
                                double *dst = a.om.out + obase + (int64_t)I * a.om.sI +
                                              omult * (int64_t)(a.om.oab[ab] + a.om.ocd[cd]);
                                *dst = ch == 0 ? O[mm][n][r] : *dst + O[mm][n][r];
                            }
                        }
            } else if constexpr (!SEPRED) {
                __syncthreads();   // every wave is past its last read of the cube
#pragma unroll
                for (int mm = 0; mm < NTAB; ++mm)
#pragma unroll
                    for (int n = 0; n < NTG; ++n)
#pragma unroll
                        for (int r = 0; r < 4; ++r) red[(((w * NTAB + mm) * NTG + n) * 4 + r) * 64 + lane] = O[mm][n][r];
                __syncthreads();
                // wave w sums and stores the slots s = w, w + NW, ...
                for (int sl = w; sl < NTAB * NTG * 4; sl += NW) {
                    const int mm = sl / (NTG * 4), n = (sl >> 2) % NTG, r = sl & 3;
                    double v = 0.0;
                    for (int ww = 0; ww < NW; ++ww) v += red[(((ww * NTAB + mm) * NTG + n) * 4 + r) * 64 + lane];
                    const int ab = 16 * mm + 4 * r + g;
                    const int cd = grp * GW + 16 * n + c;
                    if constexpr (DIG)
                        digest_block(a.dig, I, J, ab, cd, ab < a.nab, cd < a.ncd, v, g, c, dgk[cd], dgb[ab]);
                    else if (ab < a.nab && cd < a.ncd) {
                        double *dst = a.om.out + obase + (int64_t)I * a.om.sI + omult * (int64_t)(oab[ab] + ocd[cd]);
                        *dst = ch == 0 ? v : *dst + v;
                    }
                }
            } else
#pragma unroll
            for (int mm = 0; mm < NTAB; ++mm) {
                __syncthreads();
                if (w > 0) {
#pragma unroll
                    for (int n = 0; n < NTG; ++n)
#pragma unroll
                        for (int r = 0; r < 4; ++r) red[(((w - 1) * NTG + n) * 4 + r) * 64 + lane] = O[mm][n][r];
                }
                __syncthreads();
                if (w == 0) {
#pragma unroll
                    for (int n = 0; n < NTG; ++n)
#pragma unroll
                        for (int r = 0; r < 4; ++r) {
                            double v = O[mm][n][r];
                            for (int ww = 1; ww < NW; ++ww) v += red[(((ww - 1) * NTG + n) * 4 + r) * 64 + lane];
                            const int ab = 16 * mm + 4 * r + g;
                            const int cd = grp * GW + 16 * n + c;
                            if constexpr (DIG)
                                digest_block(a.dig, I, J, ab, cd, ab < a.nab, cd < a.ncd, v, g, c, dgk[cd], dgb[ab]);
                            else if (ab < a.nab && cd < a.ncd) {
                                double *dst = a.om.out + obase + (int64_t)I * a.om.sI +
                                              omult * (int64_t)(oab[ab] + ocd[cd]);
                                *dst = ch == 0 ? v : *dst + v;
                            }
                        }
                }
            }
        }
    }
}


struct MfmaShape {
    int NTAB, NTCD, NTG, MTW, NW;
};

template <int LB, int LK, int NTAB, int NTCD, int NTG, int MTW, int NW, bool GB, int LAY, int KP, bool DIG = false>
__host__ __device__ inline size_t mfma_lds_bytes(int nqmax, int kkmax)
{
    constexpr int L = LB + LK, D = L + 1;
    constexpr int NTPAD = round_up(nherm(LK - 1), 4);
    constexpr int KT = round_up(ncart(LK), 4) / 4;
    constexpr bool SEPRED = NTCD / NTG > 1;
    constexpr size_t RED = SEPRED ? (size_t)(NW - 1) * NTG * 256 : (size_t)NW * NTAB * NTG * 256;
    const size_t tabs = (size_t)Cube<D, LAY>::words(KP * nqmax);
    const size_t cube_words = SEPRED ? tabs + RED : std::max(tabs, RED);
    constexpr int NHB = GB ? ncart(LB) : nherm(LB);
    return (cube_words + (size_t)kkmax * nqmax * (D + 4) + kkmax + (size_t)(KP * NTPAD + 4 * KT) * NTG * 16) * 8 +
           (size_t)(NTPAD + 4 * KT + (NTAB + NTCD) * 16 + (DIG ? round_up(NHB, 2) : NHB)) * 4 +
           (DIG ? (size_t)(NTAB + NTCD) * 16 * 8 : 0);
}

// Instances: class key (LB, LK, NAB, NCD, GB), tile shape
// (NTAB, NTCD, NTG, MTW, NW, WPE), table layout LAY (see Cube; C = compact)
// and ket primitives per sweep round KP.  Several instances per key are
// variants 1, 2, ... in listing order; the autotuner picks one per class.
#define MDX_MFMA_INSTANCES(X)                                                                      \
    X(4, 4, 25, 25, false, 2, 2, 2, 5, 4, 2, CUBE_LAY_COMPACT, 2)  /* (dd|dd)                 */   \
    X(4, 4, 25, 25, false, 2, 2, 2, 5, 4, 2, 141, 1)                                               \
    X(4, 4, 25, 25, false, 2, 2, 2, 3, 4, 2, 141, 1)                                               \
    X(4, 4, 25, 25, false, 2, 2, 2, 5, 4, 1, 141, 1)                                               \
    X(4, 4, 25, 25, false, 2, 2, 1, 5, 4, 2, 141, 1)                                               \
    X(4, 4, 25, 25, false, 2, 2, 2, 3, 2, 3, 141, 1)                                               \
    X(4, 3, 25, 15, false, 2, 1, 1, 5, 4, 2, CUBE_LAY_COMPACT, 3)  /* (dd|dp), (pd|dd) swapped*/   \
    X(4, 3, 25, 15, false, 2, 1, 1, 5, 4, 2, CUBE_LAY_COMPACT, 2)                                  \
    X(4, 3, 25, 15, false, 2, 1, 1, 5, 4, 2, 141, 1)                                               \
    X(4, 3, 25, 15, false, 2, 1, 1, 3, 4, 2, 141, 1)                                               \
    X(4, 3, 25, 15, false, 2, 1, 1, 5, 4, 1, 141, 1)                                               \
    X(4, 3, 25, 15, false, 2, 1, 1, 3, 2, 3, 141, 1)                                               \
    X(4, 2, 25, 9, false, 2, 1, 1, 5, 4, 2, 141, 1)             /* (dd|pp)                   */    \
    X(4, 2, 25, 9, false, 2, 1, 1, 5, 4, 2, CUBE_LAY_COMPACT, 2)                                   \
    X(4, 2, 25, 9, false, 2, 1, 1, 5, 4, 2, CUBE_LAY_COMPACT, 3)                                   \
    X(4, 2, 25, 5, false, 2, 1, 1, 5, 4, 2, 141, 1)             /* (dd|ds)                   */    \
    X(4, 2, 25, 5, false, 2, 1, 1, 5, 4, 2, CUBE_LAY_COMPACT, 2)                                   \
    X(4, 2, 25, 5, false, 2, 1, 1, 5, 4, 2, CUBE_LAY_COMPACT, 3)                                   \
    X(3, 3, 15, 15, false, 1, 1, 1, 5, 4, 2, 141, 1)            /* (dp|dp)                   */    \
    X(3, 3, 15, 15, false, 1, 1, 1, 3, 4, 2, CUBE_LAY_COMPACT, 2)                                  \
    X(3, 3, 15, 15, false, 1, 1, 1, 3, 4, 2, CUBE_LAY_COMPACT, 3)                                  \
    X(3, 2, 15, 9, false, 1, 1, 1, 5, 4, 2, 141, 1)             /* (dp|pp)                   */    \
    X(3, 2, 15, 9, false, 1, 1, 1, 3, 4, 2, CUBE_LAY_COMPACT, 2)                                   \
    X(3, 2, 15, 9, false, 1, 1, 1, 3, 4, 2, CUBE_LAY_COMPACT, 3)                                   \
    X(3, 2, 15, 5, false, 1, 1, 1, 5, 4, 2, 141, 1)             /* (dp|ds)                   */    \
    X(3, 2, 15, 5, false, 1, 1, 1, 3, 4, 2, CUBE_LAY_COMPACT, 2)                                   \
    X(2, 2, 9, 9, false, 1, 1, 1, 5, 4, 2, 141, 1)              /* (pp|pp)                   */    \
    X(2, 2, 9, 9, false, 1, 1, 1, 2, 4, 2, CUBE_LAY_COMPACT, 2)                                    \
    X(4, 4, 36, 36, false, 3, 3, 3, 5, 4, 2, CUBE_LAY_COMPACT, 2)  /* (dd|dd) Cartesian       */   \
    X(4, 4, 36, 36, false, 3, 3, 3, 5, 4, 2, 141, 1)                                               \
    X(4, 3, 36, 18, false, 3, 2, 2, 5, 4, 2, CUBE_LAY_COMPACT, 2)  /* (dd|dp) Cartesian       */   \
    X(4, 3, 36, 18, false, 3, 2, 2, 5, 4, 2, 141, 1)                                               \
    X(6, 6, 49, 49, false, 4, 4, 2, 2, 3, 2, 10, 1)             /* (ff|ff)                   */    \
    X(6, 6, 49, 49, false, 4, 4, 2, 2, 3, 2, 141, 1)                                               \
    X(6, 6, 49, 49, false, 4, 4, 1, 2, 3, 2, 141, 1)                                               \
    X(6, 6, 49, 49, false, 4, 4, 2, 2, 3, 1, 141, 1)                                               \
    X(8, 8, 81, 81, false, 6, 6, 1, 3, 4, 2, 141, 1)            /* (gg|gg)                   */    \
    X(8, 8, 81, 81, false, 6, 6, 2, 3, 4, 2, 141, 1)                                               \
    X(8, 8, 81, 81, false, 6, 6, 2, 3, 4, 1, 141, 1)                                               \
    X(10, 10, 121, 121, false, 8, 8, 1, 2, 4, 1, CUBE_LAY_COMPACT, 1)  /* (hh|hh)            */   \
    X(2, 4, 5, 25, true, 1, 2, 2, 1, 1, 2, 0, 1)                /* (d|dd)                    */    \
    X(3, 4, 7, 25, true, 1, 2, 2, 1, 1, 2, 0, 1)                /* (f|dd)                    */    \
    X(4, 4, 9, 25, true, 1, 2, 2, 1, 1, 2, 0, 1)                /* (g|dd)                    */    \
    X(5, 4, 11, 25, true, 1, 2, 2, 2, 1, 2, 0, 1)               /* (h|dd)                    */    \
    X(6, 4, 13, 25, true, 1, 2, 2, 2, 1, 2, 0, 1)               /* (i|dd)                    */    \
    X(0, 4, 1, 25, true, 1, 2, 2, 1, 1, 2, 0, 1)                /* (s|dd)                    */    \
    X(1, 4, 3, 25, true, 1, 2, 2, 1, 1, 2, 0, 1)                /* (p|dd)                    */    \
    /* one wave per shellset for small, lightly contracted shellsets (screened molecules) */      \
    X(4, 4, 25, 25, false, 2, 2, 2, 3, 1, 4, CUBE_LAY_COMPACT, 2)  /* (dd|dd)                 */   \
    X(4, 3, 25, 15, false, 2, 1, 1, 3, 1, 4, CUBE_LAY_COMPACT, 3)  /* (dd|dp)                 */   \
    X(4, 2, 25, 9, false, 2, 1, 1, 3, 1, 4, CUBE_LAY_COMPACT, 3)   /* (dd|pp)                 */   \
    X(3, 3, 15, 15, false, 1, 1, 1, 4, 1, 4, CUBE_LAY_COMPACT, 2)  /* (dp|dp)                 */   \
    X(2, 2, 9, 9, false, 1, 1, 1, 2, 1, 4, CUBE_LAY_COMPACT, 4)    /* (pp|pp)                 */   \
    X(2, 1, 9, 3, false, 1, 1, 1, 2, 1, 4, CUBE_LAY_COMPACT, 4)    /* (pp|ps)                 */   \
    X(2, 2, 5, 9, false, 1, 1, 1, 2, 1, 4, CUBE_LAY_COMPACT, 4)    /* (ds|pp)                 */   \
    X(2, 2, 5, 5, false, 1, 1, 1, 2, 1, 4, CUBE_LAY_COMPACT, 4)    /* (ds|ds)                 */   \
    X(2, 1, 5, 3, false, 1, 1, 1, 2, 1, 4, CUBE_LAY_COMPACT, 4)    /* (ds|ps)                 */   \
    X(3, 2, 15, 9, false, 1, 1, 1, 2, 1, 4, CUBE_LAY_COMPACT, 4)   /* (dp|pp)                 */   \
    X(3, 1, 15, 3, false, 1, 1, 1, 2, 1, 4, CUBE_LAY_COMPACT, 4)   /* (dp|ps)                 */   \
    X(3, 2, 15, 5, false, 1, 1, 1, 2, 1, 4, CUBE_LAY_COMPACT, 4)   /* (dp|ds)                 */   \
    X(4, 1, 25, 3, false, 2, 1, 1, 3, 1, 4, CUBE_LAY_COMPACT, 4)   /* (dd|ps)                 */   \
    X(4, 2, 25, 5, false, 2, 1, 1, 3, 1, 4, CUBE_LAY_COMPACT, 4)   /* (dd|ds)                 */

// The instance rows of the general kernel; digestion (and its persistent
// form) is compiled for the first row of each class only.
struct MfmaRow {
    int lb, lk, nab, ncd;
    bool gb;
    int ntab, ntcd, ntg, mtw, nw, wpe, lay, kp;
};
constexpr MfmaRow kMfmaRows[] = {
#define MDX_ROW(lb, lk, nab, ncd, gb, ntab, ntcd, ntg, mtw, nw, wpe, lay, kp) \
    {lb, lk, nab, ncd, gb, ntab, ntcd, ntg, mtw, nw, wpe, lay, kp},
    MDX_MFMA_INSTANCES(MDX_ROW)
#undef MDX_ROW
};
constexpr bool first_of_class(MfmaRow x)
{
    for (const MfmaRow &r : kMfmaRows)
        if (r.lb == x.lb && r.lk == x.lk && r.nab == x.nab && r.ncd == x.ncd && r.gb == x.gb)
            return r.ntab == x.ntab && r.ntcd == x.ntcd && r.ntg == x.ntg && r.mtw == x.mtw && r.nw == x.nw &&
                   r.wpe == x.wpe && r.lay == x.lay && r.kp == x.kp;
    return false;
}
}  // namespace mdx
