// eri_prim.h -- matrix-core kernel for shellsets whose bra and ket pairs are
// single primitive pairs (uncontracted shells; the high angular momentum
// classes).
//
// One workgroup evaluates one shellset from one [r]^(0) table (Eq. (31)).
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
#pragma once

#include "mfma_common.h"

namespace mdx {

template <int LB, int LK, int NTAB, int NTCD, int NW, int LAY>
__device__ __forceinline__ void eri_prim_shellset(const EriArgs &a, const int I, const int J, const int nI)
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
    const int tid = threadIdx.x;
    const int w = tid >> 6, lane = tid & 63, g = lane >> 4, c = lane & 15;

    extern __shared__ double smem[];
    double *cube = smem;                        // one table
    double *S = cube + CB::words(1);            // [D]  [0]^(m) times the primitive weights
    double *PQ = S + D;                         // [4]  P - Q
    int *oab = (int *)(PQ + 4);                 // [NABP] output offsets
    int *ocd = oab + NABP;                      // [NCDP]

    for (int k = tid; k < NABP; k += NT) oab[k] = k < a.nab ? a.om.oab[k] : 0;
    for (int k = tid; k < NCDP; k += NT) ocd[k] = k < a.ncd ? a.om.ocd[k] : 0;
    if (tid == 0) {
        // [0]^(m) of the primitive quartet, Eq. (27), with the primitive weights
        const PrimRec B = a.bra.prim[(int64_t)I * a.bra.kmax];
        const PrimRec K = a.ket.prim[(int64_t)J * a.ket.kmax];
        const double pq = B.p + K.p;
        const double rho = B.p * K.p / pq;
        const double X = B.Px - K.Px, Y = B.Py - K.Py, Z = B.Pz - K.Pz;
        double F[D];
        boys_eval<L>(rho * (X * X + Y * Y + Z * Z), F, a.boys);
        double f = B.ws * K.ws * rsqrt_d(pq);
        const double m2r = -2.0 * rho;
#pragma unroll
        for (int m = 0; m <= L; ++m) {
            S[m] = f * F[m];
            f *= m2r;
        }
        PQ[0] = X;
        PQ[1] = Y;
        PQ[2] = Z;
    }
    __syncthreads();
    // one-axis sweeps of Eq. (31) over the one table, split over the waves, one
    // recursion column per branch region (long columns at high L)
    ysweeps<CB, NW, true>(cube, S, PQ, 1, 1, 1, w, lane, std::make_integer_sequence<int, NW>{});
    __syncthreads();
    xsweeps<CB, NW, 1, true>(cube, PQ, 1, 1, 1, w, lane, std::make_integer_sequence<int, NW>{});
    __syncthreads();

    int abase[MT];   // table offset of the bra Hermite of row 16T + c (rows past NHB: 0, H_bra is 0 there)
#pragma unroll
    for (int T = 0; T < MT; ++T) {
        const int row = 16 * T + c;
        abase[T] = row < NHB ? CB::off(row) : 0;
    }
    const double *Hb = a.bra.H + (int64_t)I * a.bra.pair_stride;
    const double *Hk = a.ket.H + (int64_t)J * a.ket.pair_stride;
    const int64_t obase = a.om.count ? a.om.obase[J] : (int64_t)J * a.om.sJ;
    const int64_t omult = a.om.count ? (int64_t)nI : a.om.mult;
    double *out = a.om.out + obase + (int64_t)I * a.om.sI;

    static_assert(NTCD % NW == 0, "column tiles split evenly over the waves");
#pragma unroll 1
    for (int pass = 0; pass < NTCD / NW; ++pass) {
        const int jt = w + pass * NW;
        // the gathers and the H_bra loads are the same in every pass; an opaque
        // zero offset keeps them inside the pass instead of being hoisted out of
        // the loop and held live across it
        int zo = 0;
        asm volatile("" : "+v"(zo));
        const double *hb = Hb + zo;
        // ket transform of column tile jt: M = bra rows, K = ket rows, N = 16 ket functions
        // (gathers of step s + 1 and ket rows of step s + 3 are issued while step s
        // multiplies)
        constexpr KetRowOffsets<CB, LK, 4 * KS> KO{};
        const double *hk = Hk + 16 * jt + c;
        d4 X[MT];
#pragma unroll
        for (int T = 0; T < MT; ++T) X[T] = d4{0.0, 0.0, 0.0, 0.0};
        double av[2][MT], bq[4];
#pragma unroll
        for (int k = 0; k < 3 && k < KS; ++k) bq[k] = 4 * k + g < RPB ? hk[(int64_t)(4 * k + g) * NCDP] : 0.0;
        {
            const int qo = sel4(KO.o[0], KO.o[1], KO.o[2], KO.o[3], g) + zo;
#pragma unroll
            for (int T = 0; T < MT; ++T) av[0][T] = cube[abase[T] + qo];
        }
#pragma unroll
        for (int s = 0; s < KS; ++s) {
            if (s + 1 < KS) {
                const int qo = sel4(KO.o[4 * s + 4], KO.o[4 * s + 5], KO.o[4 * s + 6], KO.o[4 * s + 7], g) + zo;
#pragma unroll
                for (int T = 0; T < MT; ++T) av[(s + 1) & 1][T] = cube[abase[T] + qo];
            }
            if (s + 3 < KS) bq[(s + 3) & 3] = 4 * (s + 3) + g < RPB ? hk[(int64_t)(4 * (s + 3) + g) * NCDP] : 0.0;
#pragma unroll
            for (int T = 0; T < MT; ++T) X[T] = mfma(av[s & 1][T], bq[s & 3], X[T]);
            __builtin_amdgcn_sched_barrier(0);
        }
        // bra transform: out = H_bra^T X, the accumulator tile of X used as the
        // B operand (register r of lane (c, g) holds X[16T + 4r + g][c])
        // K steps (T, r) in order; H_bra rows of step k + 2 are loaded while step k
        // multiplies (scheduling barriers keep the loads from all being hoisted)
        d4 O[NTAB];
#pragma unroll
        for (int i = 0; i < NTAB; ++i) O[i] = d4{0.0, 0.0, 0.0, 0.0};
        double hq[3][NTAB];
#pragma unroll
        for (int k = 0; k < 2; ++k)
#pragma unroll
            for (int i = 0; i < NTAB; ++i) hq[k][i] = hb[(int64_t)(4 * k + g) * NABP + 16 * i + c];
#pragma unroll
        for (int k = 0; k < 4 * MT; ++k) {
            if (k + 2 < 4 * MT) {
#pragma unroll
                for (int i = 0; i < NTAB; ++i) hq[(k + 2) % 3][i] = hb[(int64_t)(4 * (k + 2) + g) * NABP + 16 * i + c];
            }
#pragma unroll
            for (int i = 0; i < NTAB; ++i) O[i] = mfma(hq[k % 3][i], X[k >> 2][k & 3], O[i]);
            __builtin_amdgcn_sched_barrier(0);
        }
        const int cd = 16 * jt + c;
#pragma unroll
        for (int i = 0; i < NTAB; ++i)
#pragma unroll
            for (int r = 0; r < 4; ++r) {
                const int ab = 16 * i + 4 * r + g;
                if (ab < a.nab && cd < a.ncd) out[omult * (int64_t)(oab[ab + zo] + ocd[cd])] = O[i][r];
            }
    }
}

template <int LB, int LK, int NTAB, int NTCD, int NW, int LAY>
__host__ __device__ inline size_t prim_lds_bytes()
{
    constexpr int L = LB + LK, D = L + 1;
    return ((size_t)Cube<D, LAY>::words(1) + D + 4) * 8 + (size_t)((NTAB + NTCD) * 16) * 4;
}

// Instances: class key (LB, LK, NAB, NCD) -- four-centre, both sides pairs --
// tile counts (NTAB, NTCD), waves NW (dividing NTCD), waves per SIMD WPE and
// table layout LAY.  They follow the matrix-core kernel's variants of the same
// key in the variant numbering and serve only batches whose pairs are single
// primitive pairs.
#define MDX_PRIM_INSTANCES(X)                                                                      \
    X(6, 6, 49, 49, 4, 4, 4, 3, CUBE_LAY_COMPACT)              /* (ff|ff)                   */    \
    X(6, 6, 49, 49, 4, 4, 2, 3, CUBE_LAY_COMPACT)                                                  \
    X(6, 6, 49, 49, 4, 4, 2, 4, CUBE_LAY_COMPACT)                                                  \
    X(6, 6, 49, 49, 4, 4, 1, 3, CUBE_LAY_COMPACT)                                                  \
    X(8, 8, 81, 81, 6, 6, 2, 2, CUBE_LAY_COMPACT)              /* (gg|gg)                   */    \
    X(8, 8, 81, 81, 6, 6, 3, 2, CUBE_LAY_COMPACT)                                                  \
    X(8, 8, 81, 81, 6, 6, 6, 3, CUBE_LAY_COMPACT)                                                  \
    X(8, 8, 81, 81, 6, 6, 1, 2, CUBE_LAY_COMPACT)

}  // namespace mdx
