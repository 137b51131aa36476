// eri_multi.h -- matrix-core kernel for 3-centre shellsets (X|cd) of a
// single-function solid bra X and a ket pair of single primitive pairs, several
// shellsets per workgroup.
//
// A 3-centre shellset is small: the solid bra keeps only its terminal
// Hermites (Sec. 2.2.3) and one primitive quartet per ket primitive pair
// feeds the transforms, so per shellset the [r]^(0) recursion of Eq. (31)
// -- a chain of dependent steps -- outweighs the contractions.  One workgroup
// therefore takes NBI = NW*SPW bra functions I0 .. I0+NBI-1 against one ket
// pair J.  Their tables are built together, one shellset per lane, in an
// interleaved LDS block; then wave w evaluates shellsets w*SPW .. w*SPW+SPW-1
// one after the other:
//     X[p][cd]    = sum_q [p+q]^(0) H_ket[q][cd]      (Eq. (32), all ket rows)
//     out[ab][cd] = sum_p H_bra[p][ab] X[p][cd]       (Eq. (33), p terminal)
// The ket rows of J are loaded once per wave and kept in registers for all of
// its shellsets; no partial sum crosses waves.
#pragma once

#include "mfma_common.h"

namespace mdx {

template <int LB, int LK, int NTAB, int NTCD, int NW, int SPW, int LAY>
__device__ __forceinline__ void eri_multi_unit(const EriArgs &a, const int I0, const int J, const int nI)
{
    constexpr int L = LB + LK, D = L + 1;
    typedef Cube<D, LAY> CB;
    constexpr int NBI = NW * SPW;               // shellsets (bra functions) per workgroup
    constexpr int NHB = ncart(LB);              // terminal bra Hermites (the solid bra's rows)
    constexpr int HB0 = nherm(LB - 1);          // Hermite index of the first of them
    constexpr int MT = (NHB + 15) / 16;         // row tiles
    constexpr int NKN = nherm(LK - 1);
    constexpr int NTPAD = round_up(NKN, 4);
    constexpr int RPB = NTPAD + ncart(LK);      // ket rows stored per primitive pair
    constexpr int KS = round_up(RPB, 4) / 4;    // k-steps over all ket rows
    constexpr int NCDP = NTCD * 16, NABP = NTAB * 16;
    constexpr int NT = 64 * NW;
    static_assert(NBI <= 64 && NBI <= CB::QMAX, "tables of one workgroup");
    const int tid = threadIdx.x;
    const int w = tid >> 6, lane = tid & 63, g = lane >> 4, c = lane & 15;
    const int nv = min(NBI, nI - I0);           // shellsets of this workgroup

    extern __shared__ double smem[];
    double *cube = smem;                        // NBI tables, slot q = bra function I0 + q
    double *S = cube + CB::words(NBI);          // [NBI][D]
    double *PQ = S + NBI * D;                   // [NBI][4]

    const PrimRec K = a.ket.prim[(int64_t)J * a.ket.kmax];
    for (int q = tid; q < nv; q += NT) {
        // [0]^(m) of slot q, Eq. (27); the solid bra's primitives share its centre
        // and are summed here with their weights (Sec. 2.2.3)
        const int I = I0 + q;
        const PrimRec *bp = a.bra.prim + (int64_t)I * a.bra.kmax;
        const int npb = a.bra.nprim[I];
        double Sm[D];
#pragma unroll
        for (int m = 0; m <= L; ++m) Sm[m] = 0.0;
        double X = 0.0, Y = 0.0, Z = 0.0;
        for (int ib = 0; ib < npb; ++ib) {
            const PrimRec B = bp[ib];
            const double pq = B.p + K.p;
            const double ypq = rsqrt_d(pq);   // 1/sqrt(p+q)
            const double rho = B.p * K.p * (ypq * ypq);
            X = B.Px - K.Px;
            Y = B.Py - K.Py;
            Z = B.Pz - K.Pz;
            double F[D];
            boys_eval<L>(rho * (X * X + Y * Y + Z * Z), F, a.boys);
            double f = B.ws * K.ws * ypq;
            const double m2r = -2.0 * rho;
#pragma unroll
            for (int m = 0; m <= L; ++m) {
                Sm[m] = fma(f, F[m], Sm[m]);
                f *= m2r;
            }
        }
#pragma unroll
        for (int m = 0; m <= L; ++m) S[q * D + m] = Sm[m];
        PQ[q * 4 + 0] = X;
        PQ[q * 4 + 1] = Y;
        PQ[q * 4 + 2] = Z;
    }
    __syncthreads();
    // one-axis sweeps of Eq. (31), one shellset per lane
    ysweeps<CB, NW, true>(cube, S, PQ, nv, NBI, NBI, w, lane, std::make_integer_sequence<int, NW>{});
    __syncthreads();
    xsweeps<CB, NW, NBI, true>(cube, PQ, nv, NBI, NBI, w, lane, std::make_integer_sequence<int, NW>{});
    __syncthreads();

    // ket rows of J, kept in registers for every shellset of the wave
    constexpr KetRowOffsets<CB, LK, 4 * KS> KO{};
    const double *Hk = a.ket.H + (int64_t)J * a.ket.pair_stride;
    double bk[KS][NTCD];
#pragma unroll
    for (int s = 0; s < KS; ++s)
#pragma unroll
        for (int n = 0; n < NTCD; ++n) bk[s][n] = 4 * s + g < RPB ? Hk[(int64_t)(4 * s + g) * NCDP + 16 * n + c] : 0.0;
    int rofs[MT];   // table offset of the bra Hermite of row 16T + c (rows past NHB: 0, H_bra is 0 there)
#pragma unroll
    for (int T = 0; T < MT; ++T) rofs[T] = 16 * T + c < NHB ? CB::off(HB0 + 16 * T + c) : 0;
    const int64_t obase = a.om.count ? a.om.obase[J] : (int64_t)J * a.om.sJ;
    const int64_t omult = a.om.count ? (int64_t)nI : a.om.mult;

#pragma unroll 1
    for (int i = 0; i < SPW; ++i) {
        const int q = w * SPW + i;
        if (q >= nv) break;   // uniform over the wave
        const int I = I0 + q;
        // ket transform: M = bra rows, K = ket rows, N = ket functions
        d4 X[MT][NTCD];
#pragma unroll
        for (int T = 0; T < MT; ++T)
#pragma unroll
            for (int n = 0; n < NTCD; ++n) X[T][n] = d4{0.0, 0.0, 0.0, 0.0};
        const double *cq = cube + q * CB::SIZE;
#pragma unroll
        for (int s = 0; s < KS; ++s) {
            const int qo = sel4(KO.o[4 * s], KO.o[4 * s + 1], KO.o[4 * s + 2], KO.o[4 * s + 3], g);
#pragma unroll
            for (int T = 0; T < MT; ++T) {
                const double av = cq[rofs[T] + qo];
#pragma unroll
                for (int n = 0; n < NTCD; ++n) X[T][n] = mfma(av, bk[s][n], X[T][n]);
            }
        }
        // bra transform with the accumulator tiles as the B operand
        const double *Hb = a.bra.H + (int64_t)I * a.bra.pair_stride;
        d4 O[NTAB][NTCD];
#pragma unroll
        for (int mm = 0; mm < NTAB; ++mm)
#pragma unroll
            for (int n = 0; n < NTCD; ++n) O[mm][n] = d4{0.0, 0.0, 0.0, 0.0};
#pragma unroll
        for (int T = 0; T < MT; ++T)
#pragma unroll
            for (int r = 0; r < 4; ++r)
#pragma unroll
                for (int mm = 0; mm < NTAB; ++mm) {
                    const double h = Hb[(int64_t)(16 * T + 4 * r + g) * NABP + 16 * mm + c];
#pragma unroll
                    for (int n = 0; n < NTCD; ++n) O[mm][n] = mfma(h, X[T][n][r], O[mm][n]);
                }
        double *out = a.om.out + obase + (int64_t)I * a.om.sI;
#pragma unroll
        for (int mm = 0; mm < NTAB; ++mm)
#pragma unroll
            for (int n = 0; n < NTCD; ++n)
#pragma unroll
                for (int r = 0; r < 4; ++r) {
                    const int ab = 16 * mm + 4 * r + g, cd = 16 * n + c;
                    if (ab < a.nab && cd < a.ncd) out[omult * (int64_t)(a.om.oab[ab] + a.om.ocd[cd])] = O[mm][n][r];
                }
    }
}

template <int LB, int LK, int NTAB, int NTCD, int NW, int SPW, int LAY>
__host__ __device__ inline size_t multi_lds_bytes()
{
    constexpr int D = LB + LK + 1, NBI = NW * SPW;
    return ((size_t)Cube<D, LAY>::words(NBI) + (size_t)NBI * (D + 4)) * 8;
}

// Instances: class key (LB, LK, NAB, NCD) -- 3-centre, single-function solid
// bra, ket pair -- tile counts (NTAB, NTCD), waves NW, shellsets per wave SPW
// and table layout LAY.  They follow the class's other matrix-core variants in the
// variant numbering and serve ket pairs of single primitive pairs.
#define MDX_MULTI_INSTANCES(X)                                                                     \
    X(2, 4, 5, 25, 1, 2, 4, 2, CUBE_LAY_COMPACT)               /* (d|dd)                    */    \
    X(3, 4, 7, 25, 1, 2, 4, 4, CUBE_LAY_COMPACT)               /* (f|dd)                    */    \
    X(3, 4, 7, 25, 1, 2, 4, 2, CUBE_LAY_COMPACT)                                                   \
    X(4, 4, 9, 25, 1, 2, 4, 4, CUBE_LAY_COMPACT)               /* (g|dd)                    */    \
    X(4, 4, 9, 25, 1, 2, 4, 2, CUBE_LAY_COMPACT)                                                   \
    X(5, 4, 11, 25, 1, 2, 4, 2, CUBE_LAY_COMPACT)              /* (h|dd)                    */    \
    X(5, 4, 11, 25, 1, 2, 2, 4, CUBE_LAY_COMPACT)                                                  \
    X(6, 4, 13, 25, 1, 2, 4, 2, CUBE_LAY_COMPACT)              /* (i|dd)                    */    \
    X(6, 4, 13, 25, 1, 2, 2, 4, CUBE_LAY_COMPACT)

}  // namespace mdx
