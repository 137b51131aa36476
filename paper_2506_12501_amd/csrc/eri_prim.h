// eri_prim.h -- matrix-core kernel for shellsets whose bra and ket pairs are
// single primitive pairs (uncontracted shells; the high angular momentum
// classes).
//
// One workgroup evaluates NB shellsets (bra pairs I0 .. I0+NB-1 against one
// ket pair J), each from one [r]^(0) table (Eq. (31)); the tables are built
// together, one quartet per lane.
// With a single primitive quartet the partial early contraction of
// Sec. 2.2.2 saves nothing, so the ket transform of Eq. (32) runs over every
// ket Hermite, terminal ones included, with B read straight from the ket pair
// data, and the bra transform of Eq. (33) follows:
//     X[p][cd]   = sum_q [p+q]^(0) H_ket[q][cd]
//     out[ab][cd] = sum_p H_bra[p][ab] X[p][cd]
// The waves split the ket functions: wave w owns the 16-column tiles
// w, w + NW, ... and, one tile at a time, accumulates the whole column tile of
// X (every bra Hermite row) in registers, applies the bra transform and
// stores.  No partial sums cross waves, so after the table is built there is
// no barrier and no LDS traffic other than the operand gathers.
// TAIL: the function counts are 16k+1 ((ff|ff): 49, (gg|gg): 81), so the last
// column tile and the last output-row tile would each carry one function in
// 16.  That function's column of X, its output row and its output column are
// instead accumulated on the VALU inside the matrix-core loops, from the same
// operands (one wave's first pass takes the column of X and the output
// column; every pass takes its part of the output row), which removes a fifth
// to a quarter of the matrix-core work.
// Row parts: the bra Hermite rows of a column tile in RS parts, each accumulating
// its own tiles of X and adding its share of the bra transform to the
// output tiles, so that only MT/RS tiles of X are live at once ((ii|ii) has
// 455 bra Hermite rows, 29 tiles).
#pragma once

#include "mfma_common.h"

namespace mdx {

template <int LB, int LK, int NTAB, int NTCD, int NW, int NB, bool TAIL, int LAY>
__device__ __forceinline__ void eri_prim_unit(const EriArgs &a, const int I0, const int J, const int nI)
{
    constexpr int L = LB + LK, D = L + 1;
    typedef Cube<D, LAY> CB;
    constexpr int NHB = nherm(LB);              // bra Hermite rows of the one primitive pair
    constexpr int MT = (NHB + 15) / 16;         // row tiles
    constexpr int NKN = nherm(LK - 1);          // non-terminal ket Hermites
    constexpr int NTPAD = round_up(NKN, 4);
    constexpr int NKT = ncart(LK);              // terminal ket Hermites
    constexpr int RPB = NTPAD + NKT;            // ket rows stored per primitive pair
    constexpr int KS = round_up(RPB, 4) / 4;    // k-steps over all ket rows
    constexpr int NCDP = NTCD * 16, NABP = NTAB * 16;
    constexpr int NT = 64 * NW;
    constexpr int NTABM = TAIL ? NTAB - 1 : NTAB;   // output-row tiles on the matrix cores
    constexpr int NTCDM = TAIL ? NTCD - 1 : NTCD;   // column tiles on the matrix cores
    constexpr int ABT = 16 * (NTAB - 1), CDT = 16 * (NTCD - 1);   // the tail functions (TAIL)
    static_assert(!TAIL || NB == 1, "tail functions with one shellset per workgroup");
    constexpr int RS = MT > 24 ? 2 : 1;         // row parts (only where a column tile of X would not fit)
    static_assert(!TAIL || RS == 1, "row parts without the VALU tail");
    constexpr int MTP = (MT + RS - 1) / RS;     // row tiles per part
    const int tid = threadIdx.x;
    const int w = tid >> 6, lane = tid & 63, g = lane >> 4, c = lane & 15;
    static_assert(NB <= 64 && NB <= CB::QMAX, "tables of one workgroup");
    const int nv = min(NB, nI - I0);           // shellsets of this workgroup

    extern __shared__ double smem[];
    double *cube = smem;                        // NB tables, slot q = bra pair I0 + q
    double *S = cube + CB::words(NB);           // [NB][D]  [0]^(m) times the primitive weights
    double *PQ = S + NB * D;                    // [NB][4]  P - Q
    double *Xt = PQ + 4 * NB;                   // [16*MT] (TAIL) column CDT of X
    int *oab = (int *)(Xt + (TAIL ? 16 * MT : 0));   // [NABP] output offsets
    int *ocd = oab + NABP;                      // [NCDP]

    for (int k = tid; k < NABP; k += NT) oab[k] = k < a.nab ? a.om.oab[k] : 0;
    for (int k = tid; k < NCDP; k += NT) ocd[k] = k < a.ncd ? a.om.ocd[k] : 0;
    for (int q = tid; q < nv; q += NT) {
        // [0]^(m) of the primitive quartet of slot q, Eq. (27), with the primitive weights
        const PrimRec B = a.bra.prim[(int64_t)(I0 + q) * a.bra.kmax];
        const PrimRec K = a.ket.prim[(int64_t)J * a.ket.kmax];
        const double pq = B.p + K.p;
        const double ypq = rsqrt_d(pq);   // 1/sqrt(p+q)
        const double rho = B.p * K.p * (ypq * ypq);
        const double X = B.Px - K.Px, Y = B.Py - K.Py, Z = B.Pz - K.Pz;
        double F[D];
        boys_eval<L>(rho * (X * X + Y * Y + Z * Z), F, a.boys);
        double f = B.ws * K.ws * ypq;
        const double m2r = -2.0 * rho;
#pragma unroll
        for (int m = 0; m <= L; ++m) {
            S[q * D + m] = f * F[m];
            f *= m2r;
        }
        PQ[q * 4 + 0] = X;
        PQ[q * 4 + 1] = Y;
        PQ[q * 4 + 2] = Z;
    }
    __syncthreads();
    // one-axis sweeps of Eq. (31), one table per lane, split over the waves, one
    // recursion column per branch region (long columns at high L)
    ysweeps<CB, NW, true>(cube, S, PQ, nv, NB, NB, w, lane, std::make_integer_sequence<int, NW>{});
    __syncthreads();
    xsweeps<CB, NW, NB, true>(cube, PQ, nv, NB, NB, w, lane, std::make_integer_sequence<int, NW>{});
    __syncthreads();

    int abase[MT];   // table offset of the bra Hermite of row 16T + c (rows past NHB: 0; their H_bra is read as 0)
#pragma unroll
    for (int T = 0; T < MT; ++T) {
        const int row = 16 * T + c;
        abase[T] = row < NHB ? CB::off(row) : 0;
    }
    const double *Hk = a.ket.H + (int64_t)J * a.ket.pair_stride;
    const int64_t obase = a.om.count ? a.om.obase[J] : (int64_t)J * a.om.sJ;
    const int64_t omult = a.om.count ? (int64_t)nI : a.om.mult;
    constexpr KetRowOffsets<CB, LK, 4 * KS> KO{};
    // primitive expansion: later primitive combinations add to the first one's output
    const bool acc_out = a.accumulate != 0;
    auto put = [acc_out](double *p, double v) { *p = acc_out ? *p + v : v; };

    constexpr int NP = (NTCDM + NW - 1) / NW;   // column passes of a wave per shellset
#pragma unroll 1
    for (int it = 0; it < NB * NP; ++it) {
        const int q = it / NP, jt = w + (it - q * NP) * NW;
        if (q >= nv) break;   // uniform
        if (jt >= NTCDM) continue;
        const bool tpass = TAIL && w == NW - 1 && it == 0;   // uniform: this pass also takes the tail column
        const double *Hb = a.bra.H + (int64_t)(I0 + q) * a.bra.pair_stride;
        double *out = a.om.out + obase + (int64_t)(I0 + q) * a.om.sI;
        const int qb = q * CB::SIZE;   // this shellset's table
        // the gathers and the H_bra loads are the same in every pass; an opaque
        // zero offset keeps them inside the pass instead of being hoisted out of
        // the loop and held live across it
        int zo = 0;
        asm volatile("" : "+v"(zo));
        const double *hb = Hb + zo;
        d4 O[NTABM];
#pragma unroll
        for (int i = 0; i < NTABM; ++i) O[i] = d4{0.0, 0.0, 0.0, 0.0};
        double trow = 0.0, ocol[NTAB];
#pragma unroll
        for (int i = 0; i < NTAB; ++i) ocol[i] = 0.0;
#pragma unroll 1
        for (int part = 0; part < RS; ++part) {
        const int T0 = part * MTP;                                   // first row tile of this part
        const int MTN = (part + 1) * MTP < MT ? MTP : MT - T0;       // row tiles of this part
        int ab0[MTP];   // table offsets of this part's bra rows (row 16(T0 + T) + c)
#pragma unroll
        for (int T = 0; T < MTP; ++T) {
            if constexpr (RS == 1) {
                ab0[T] = abase[T];
            } else {
                const int row = 16 * (T0 + T) + c;
                ab0[T] = row < NHB ? CB::off(row) : 0;
            }
        }
        // ket transform of column tile jt: M = bra rows, K = ket rows, N = 16 ket functions
        // (gathers of step s + 1 and ket rows of step s + 3 are issued while step s
        // multiplies)
        const double *hk = Hk + 16 * jt + c;
        d4 X[MTP];
#pragma unroll
        for (int T = 0; T < MTP; ++T) X[T] = d4{0.0, 0.0, 0.0, 0.0};
        double av[2][MTP], bq[4], tq[4], xt[MTP];
#pragma unroll
        for (int T = 0; T < MTP; ++T) xt[T] = 0.0;
        const double *hkt = Hk + CDT;   // TAIL: ket column CDT
#pragma unroll
        for (int k = 0; k < 3 && k < KS; ++k) {
            bq[k] = 4 * k + g < RPB ? hk[(int64_t)(4 * k + g) * NCDP] : 0.0;
            if constexpr (TAIL) tq[k] = (tpass && 4 * k + g < RPB) ? hkt[(int64_t)(4 * k + g) * NCDP] : 0.0;
        }
        {
            const int qo = sel4(KO.o[0], KO.o[1], KO.o[2], KO.o[3], g) + zo + qb;
#pragma unroll
            for (int T = 0; T < MTP; ++T)
                if (T < MTN) av[0][T] = cube[ab0[T] + qo];
        }
#pragma unroll
        for (int s = 0; s < KS; ++s) {
            if (s + 1 < KS) {
                const int qo = sel4(KO.o[4 * s + 4], KO.o[4 * s + 5], KO.o[4 * s + 6], KO.o[4 * s + 7], g) + zo + qb;
#pragma unroll
                for (int T = 0; T < MTP; ++T)
                    if (T < MTN) av[(s + 1) & 1][T] = cube[ab0[T] + qo];
            }
            if (s + 3 < KS) {
                bq[(s + 3) & 3] = 4 * (s + 3) + g < RPB ? hk[(int64_t)(4 * (s + 3) + g) * NCDP] : 0.0;
                if constexpr (TAIL)
                    tq[(s + 3) & 3] = (tpass && 4 * (s + 3) + g < RPB) ? hkt[(int64_t)(4 * (s + 3) + g) * NCDP] : 0.0;
            }
#pragma unroll
            for (int T = 0; T < MTP; ++T)
                if (T < MTN) X[T] = mfma(av[s & 1][T], bq[s & 3], X[T]);
            if constexpr (TAIL)
                if (tpass)
#pragma unroll
                    for (int T = 0; T < MTP; ++T) xt[T] = fma(av[s & 1][T], tq[s & 3], xt[T]);
            __builtin_amdgcn_sched_barrier(0);
        }
        if constexpr (TAIL) {
            if (tpass) {
                // column CDT of X: sum the four lane groups, rows past NHB are 0
#pragma unroll
                for (int T = 0; T < MTP; ++T) {
                    double v = xt[T];
                    v += __shfl_xor(v, 16);
                    v += __shfl_xor(v, 32);
                    if (g == 0) Xt[16 * T + c] = 16 * T + c < NHB ? v : 0.0;
                }
            }
        }
        // bra transform: out = H_bra^T X, the accumulator tile of X used as the
        // B operand (register r of lane (c, g) holds X[16T + 4r + g][c])
        // K steps (T, r) in order; H_bra rows of step k + 2 are loaded while step k
        // multiplies (scheduling barriers keep the loads from all being hoisted)
        // (TAIL: output row ABT from the same accumulators on the VALU: each lane
        // multiplies its own rows, the four lane groups are summed after)
        const double *hbp = hb + (int64_t)(16 * T0) * NABP;   // H_bra rows of this part
        // rows past NHB are read as 0 (with primitive expansion the pair data
        // there hold the next primitive's rows, not zero padding)
        const int nrow_p = NHB - 16 * T0;
        double hq[3][NTAB];
#pragma unroll
        for (int k = 0; k < 2; ++k)
#pragma unroll
            for (int i = 0; i < NTAB; ++i)
                hq[k][i] = 4 * k + g < nrow_p ? hbp[(int64_t)(4 * k + g) * NABP + (i < NTABM ? 16 * i + c : ABT)] : 0.0;
#pragma unroll
        for (int k = 0; k < 4 * MTP; ++k) {
            if (k < 4 * MTN) {
                if (k + 2 < 4 * MTN) {
#pragma unroll
                    for (int i = 0; i < NTAB; ++i)
                        hq[(k + 2) % 3][i] = 4 * (k + 2) + g < nrow_p
                                                 ? hbp[(int64_t)(4 * (k + 2) + g) * NABP + (i < NTABM ? 16 * i + c : ABT)]
                                                 : 0.0;
                }
#pragma unroll
                for (int i = 0; i < NTABM; ++i) O[i] = mfma(hq[k % 3][i], X[k >> 2][k & 3], O[i]);
                if constexpr (TAIL) {
                    trow = fma(hq[k % 3][NTAB - 1], X[k >> 2][k & 3], trow);
                    if (tpass) {   // output column CDT: H_bra rows times the column of X
                        const double xv = Xt[4 * k + g];
#pragma unroll
                        for (int i = 0; i < NTAB; ++i) ocol[i] = fma(hq[k % 3][i], xv, ocol[i]);
                    }
                }
            }
            __builtin_amdgcn_sched_barrier(0);
        }
        }   // row parts
        const int cd = 16 * jt + c;
#pragma unroll
        for (int i = 0; i < NTABM; ++i)
#pragma unroll
            for (int r = 0; r < 4; ++r) {
                const int ab = 16 * i + 4 * r + g;
                if (ab < a.nab && cd < a.ncd) put(out + omult * (int64_t)(oab[ab + zo] + ocd[cd]), O[i][r]);
            }
        if constexpr (TAIL) {
            trow += __shfl_xor(trow, 16);
            trow += __shfl_xor(trow, 32);
            if (g == 0 && cd < a.ncd) put(out + omult * (int64_t)(oab[ABT] + ocd[cd]), trow);
            if (tpass) {
#pragma unroll
                for (int i = 0; i < NTAB; ++i) {
                    double v = ocol[i];
                    v += __shfl_xor(v, 16);
                    v += __shfl_xor(v, 32);
                    // i < NTABM: function 16i + c; the last slot holds column ABT (the corner)
                    const int ab = i < NTABM ? 16 * i + c : ABT;
                    if (g == 0 && (i < NTABM || c == 0) && ab < a.nab) put(out + omult * (int64_t)(oab[ab] + ocd[CDT]), v);
                }
            }
        }
    }
}

template <int LB, int LK, int NTAB, int NTCD, int NW, int NB, bool TAIL, int LAY>
__host__ __device__ inline size_t prim_lds_bytes()
{
    constexpr int L = LB + LK, D = L + 1;
    return ((size_t)Cube<D, LAY>::words(NB) + (size_t)NB * (D + 4) + (TAIL ? round_up(nherm(LB), 16) : 0)) * 8 +
           (size_t)((NTAB + NTCD) * 16) * 4;
}

// Instances: class key (LB, LK, NAB, NCD) -- four-centre, both sides pairs --
// tile counts (NTAB, NTCD), waves NW, waves per SIMD WPE, bra pairs per
// workgroup NB, the VALU tail TAIL (function counts 16k+1) and table layout LAY.  They follow the matrix-core kernel's variants of the same
// key in the variant numbering and serve only batches whose pairs are single
// primitive pairs.
#define MDX_PRIM_INSTANCES(X)                                                                      \
    X(6, 6, 49, 49, 4, 4, 3, 3, 1, true, CUBE_LAY_COMPACT)        /* (ff|ff)                 */    \
    X(6, 6, 49, 49, 4, 4, 2, 3, 2, false, CUBE_LAY_COMPACT)                                        \
    X(6, 6, 49, 49, 4, 4, 2, 3, 1, false, CUBE_LAY_COMPACT)                                        \
    X(6, 6, 49, 49, 4, 4, 4, 3, 1, false, CUBE_LAY_COMPACT)                                        \
    X(8, 8, 81, 81, 6, 6, 2, 2, 1, false, CUBE_LAY_COMPACT)       /* (gg|gg)                 */    \
    X(8, 8, 81, 81, 6, 6, 3, 2, 1, false, CUBE_LAY_COMPACT)                                        \
    X(8, 8, 81, 81, 6, 6, 6, 3, 1, false, CUBE_LAY_COMPACT)                                        \
    X(10, 10, 121, 121, 8, 8, 2, 1, 1, false, CUBE_LAY_COMPACT)   /* (hh|hh)                 */    \
    X(10, 10, 121, 121, 8, 8, 4, 1, 1, false, CUBE_LAY_COMPACT)                                    \
    X(10, 10, 121, 121, 8, 8, 3, 1, 1, false, CUBE_LAY_COMPACT)                                    \
    X(12, 12, 169, 169, 11, 11, 2, 1, 1, false, CUBE_LAY_COMPACT) /* (ii|ii)                 */    \
    X(12, 12, 169, 169, 11, 11, 4, 1, 1, false, CUBE_LAY_COMPACT)                                  \
    /* mixed high-L classes (their only kernels: contracted pairs by primitive expansion) */       \
    X(8, 6, 81, 49, 6, 4, 2, 2, 1, false, CUBE_LAY_COMPACT)       /* (gg|ff)                 */    \
    X(8, 4, 81, 25, 6, 2, 2, 2, 1, false, CUBE_LAY_COMPACT)       /* (gg|dd)                 */    \
    X(10, 8, 121, 81, 8, 6, 2, 1, 1, false, CUBE_LAY_COMPACT)     /* (hh|gg)                 */    \
    X(10, 6, 121, 49, 8, 4, 2, 1, 1, false, CUBE_LAY_COMPACT)     /* (hh|ff)                 */    \
    X(10, 4, 121, 25, 8, 2, 2, 1, 1, false, CUBE_LAY_COMPACT)     /* (hh|dd)                 */    \
    X(12, 10, 169, 121, 11, 8, 2, 1, 1, false, CUBE_LAY_COMPACT)  /* (ii|hh)                 */    \
    X(12, 8, 169, 81, 11, 6, 2, 1, 1, false, CUBE_LAY_COMPACT)    /* (ii|gg)                 */    \
    X(12, 6, 169, 49, 11, 4, 2, 1, 1, false, CUBE_LAY_COMPACT)    /* (ii|ff)                 */    \
    X(12, 4, 169, 25, 11, 2, 2, 1, 1, false, CUBE_LAY_COMPACT)    /* (ii|dd)                 */

}  // namespace mdx
