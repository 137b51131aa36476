// eri_valu.h -- the register integral kernel body (one lane per shellset)
// and its instance list; shared by the plain and the persistent launches.
//
// Per primitive quartet the lane follows the MD chain of Eq. (36):
//   [0]^(m) (Eq. (27), Boys of Eq. (28))  ->  [r]^(0) (Eq. (31))
//   -> [p|q] = (-1)^{l_q} [p+q]^(0) (Eq. (25); the sign sits in the ket H)
//   -> ket transform (Eq. (32)), accumulated over ket primitives
// and, once per bra primitive, the bra transform (Eq. (33)).  Lanes of a wave
// take consecutive bra pairs of one ket pair, so ket data are wave-uniform
// (scalar loads) and stores of the [ij,ab,cd,kl] layout are coalesced.
// A single-function solid side sums its primitives into [0]^(m) before the
// recursion (Sec. 2.2.3).
#pragma once

#include "eri_common.h"
#include "kernels.h"

namespace mdx {

// Shellset (bra pair I, ket pair J) of the calling lane into out[ab][cd],
// for the ket functions cd = C0 .. C0 + NCS - 1 (all of them by default).
// UJ: J is the same for the whole wave, so its ket data are scalar loads
// (false only for paired batches, one quartet per lane).
template <int LB, int LK, int NAB, int NCD, bool GB, bool GK, bool UJ = true, int C0 = 0, int NCS = NCD>
__device__ __forceinline__ void eri_valu_compute(const EriArgs &a, const int I, const int J, double (&out)[NAB][NCS])
{
    static_assert(C0 >= 0 && NCS >= 1 && C0 + NCS <= NCD, "ket function range");
    constexpr int L = LB + LK;
    constexpr int NH = nherm(L);
    constexpr int NHB = GB ? ncart(LB) : nherm(LB);           // bra rows per primitive
    constexpr int HB0 = GB ? nherm(LB - 1) : 0;               // Hermite index of bra row 0
    constexpr int NKN = GK ? 0 : nherm(LK - 1);               // ket non-terminal rows
    constexpr int NTPAD = GK ? 0 : round_up(nherm(LK - 1), 4);
    constexpr int NKT = ncart(LK);                            // ket terminal rows
    constexpr int RPB = NTPAD + NKT;                          // ket rows per primitive block
    constexpr int NABP = round_up(NAB, 16);
    constexpr int NCDP = round_up(NCD, 16);
    constexpr SumTab<LB, LK> sum{};


    const int npb = a.bra.nprim[I];
    const int npk = UJ ? load_const(a.ket.nprim + J) : a.ket.nprim[J];
    const PrimRec *bp = a.bra.prim + (int64_t)I * a.bra.kmax;
    const PrimRec *kp = a.ket.prim + (int64_t)J * a.ket.kmax;
    const double *Hb = a.bra.H + (int64_t)I * a.bra.pair_stride;
    const double *HkP = a.ket.H + (int64_t)J * a.ket.pair_stride;

#pragma unroll
    for (int i = 0; i < NAB; ++i)
#pragma unroll
        for (int j = 0; j < NCS; ++j) out[i][j] = 0.0;

    // The bra primitive loop runs to the side's largest count (the same for
    // every lane), each lane contributing while kb < its own count: the ket
    // loops inside stay wave-uniform, so the ket records and H rows (the same
    // ket pair in every lane of a wave) are scalar loads.
    const int nkbw = GB ? 1 : a.bra.kmax;
    const int nkk = GK ? 1 : npk;
    for (int kb = 0; kb < nkbw; ++kb) {
        if (!GB && kb >= npb) continue;
        double X[NHB][NCS];
#pragma unroll
        for (int i = 0; i < NHB; ++i)
#pragma unroll
            for (int j = 0; j < NCS; ++j) X[i][j] = 0.0;
        PrimRec B1{};
        if constexpr (!GB) B1 = bp[kb];

        // one ket primitive per iteration (wave-uniform, scalar loads): the
        // next one is fetched while this one is computed
        constexpr bool PREF = !GK && UJ;
        PrimRec Kn{};
        if constexpr (PREF) Kn = load_const(kp);
        for (int kk = 0; kk < nkk; ++kk) {
            PrimRec Kc{};
            if constexpr (PREF) {
                Kc = Kn;
                Kn = load_const(kp + (kk + 1 < nkk ? kk + 1 : kk));
            }
            double S[L + 1];
#pragma unroll
            for (int m = 0; m <= L; ++m) S[m] = 0.0;
            double PQ0 = 0.0, PQ1 = 0.0, PQ2 = 0.0;
            const int b0 = GB ? 0 : kb, b1 = GB ? npb : kb + 1;
            const int k0 = GK ? 0 : kk, k1 = GK ? npk : kk + 1;
            for (int ib = b0; ib < b1; ++ib) {
                const PrimRec B = GB ? bp[ib] : B1;
                for (int ik = k0; ik < k1; ++ik) {
                    const PrimRec K = PREF ? Kc : (UJ ? load_const(kp + ik) : kp[ik]);   // the wave's ket pair: scalar
                    const double pq = B.p + K.p;
                    const double y = rsqrt_d(pq);            // 1/sqrt(p+q)
                    const double rho = B.p * K.p * (y * y);
                    PQ0 = B.Px - K.Px;
                    PQ1 = B.Py - K.Py;
                    PQ2 = B.Pz - K.Pz;
                    const double T = rho * (PQ0 * PQ0 + PQ1 * PQ1 + PQ2 * PQ2);
                    double F[L + 1];
                    boys_eval<L>(T, F, a.boys);
                    double f = B.ws * K.ws * y;
                    const double m2r = -2.0 * rho;
#pragma unroll
                    for (int m = 0; m <= L; ++m) {
                        S[m] = fma(f, F[m], S[m]);
                        f *= m2r;
                    }
                }
            }
            double R[(L + 1) * NH];
            r_recursion<L>(S, PQ0, PQ1, PQ2, R);

            // ket transform, Eq. (32): X[h][cd] += [h|q] H_ket[q][cd]
            const double *Hk = HkP + (GK ? 0 : (int64_t)kk * RPB * NCDP);
#pragma unroll
            for (int r = 0; r < NKN + NKT; ++r) {
                const int hrow = r < NKN ? r : NTPAD + (r - NKN);
                const int qh = r < NKN ? r : nherm(LK - 1) + (r - NKN);
                double hk[NCS];
#pragma unroll
                for (int j = 0; j < NCS; ++j)
                    hk[j] = UJ ? load_const(Hk + hrow * NCDP + C0 + j) : Hk[hrow * NCDP + C0 + j];
#pragma unroll
                for (int i = 0; i < NHB; ++i) {
                    const double v = R[sum.idx[HB0 + i][qh]];
#pragma unroll
                    for (int j = 0; j < NCS; ++j) X[i][j] = fma(v, hk[j], X[i][j]);
                }
            }
        }
        // bra transform, Eq. (33): out[ab][cd] += H_bra[ab][h] X[h][cd]
        const double *Hbk = Hb + (int64_t)(GB ? 0 : kb * NHB) * NABP;
#pragma unroll
        for (int i = 0; i < NHB; ++i) {
#pragma unroll
            for (int ab = 0; ab < NAB; ++ab) {
                const double hb = Hbk[i * NABP + ab];
#pragma unroll
                for (int j = 0; j < NCS; ++j) out[ab][j] = fma(hb, X[i][j], out[ab][j]);
            }
        }
    }

}

// Ket functions per part of a shellset.  A lane holds its outputs and the
// ket-transformed block X (NAB + NHB values per ket function); where these
// exceed the registers by far, the lane takes the ket functions in parts,
// running the primitive loops once per part.  Every output element gets the
// same operations in the same order either way.
template <int LB, int NAB, int NCD, bool GB>
__host__ __device__ constexpr int valu_part_cols()
{
    constexpr int per = NAB + (GB ? ncart(LB) : nherm(LB));
    if (per * NCD <= 200) return NCD;
    return 128 / per < 1 ? 1 : (128 / per < NCD ? 128 / per : NCD);
}

template <int LB, int LK, int NAB, int NCD, bool GB, bool GK, bool UJ, int C0>
__device__ __forceinline__ void eri_valu_shellset_part(const EriArgs &a, const int I, const int J, const int nI)
{
    constexpr int NCS0 = valu_part_cols<LB, NAB, NCD, GB>();
    constexpr int NCS = C0 + NCS0 <= NCD ? NCS0 : NCD - C0;
    double out[NAB][NCS];
    eri_valu_compute<LB, LK, NAB, NCD, GB, GK, UJ, C0, NCS>(a, I, J, out);
    // store, [ij,ab,cd,kl] addressing of the caller
    const int64_t base = (a.om.count ? a.om.obase[J] : (int64_t)J * a.om.sJ) + (int64_t)I * a.om.sI;
    const int64_t mult = a.om.count ? (int64_t)nI : a.om.mult;
#pragma unroll
    for (int ab = 0; ab < NAB; ++ab)
#pragma unroll
        for (int j = 0; j < NCS; ++j)
            a.om.out[base + mult * (int64_t)(a.om.oab[ab] + a.om.ocd[C0 + j])] = out[ab][j];
    if constexpr (C0 + NCS < NCD) eri_valu_shellset_part<LB, LK, NAB, NCD, GB, GK, UJ, C0 + NCS>(a, I, J, nI);
}

// Shellset (I, J) of the calling lane, stored in the caller's layout; I < nI.
template <int LB, int LK, int NAB, int NCD, bool GB, bool GK, bool UJ = true>
__device__ __forceinline__ void eri_valu_shellset(const EriArgs &a, const int I, const int J, const int nI)
{
    eri_valu_shellset_part<LB, LK, NAB, NCD, GB, GK, UJ, 0>(a, I, J, nI);
}

// One part of the ket functions (see valu_part_cols): the Jk terms of its
// columns go out at once, the Jb rows are summed into jb over the parts, in
// the same column order as a whole shellset.
template <int LB, int LK, int NAB, int NCD, bool GB, bool GK, int C0>
__device__ __forceinline__ void eri_valu_digest_part(const EriArgs &a, const int I, const int J, const bool live,
                                                     const int lane, double (&jb)[NAB])
{
    constexpr int NCS0 = valu_part_cols<LB, NAB, NCD, GB>();
    constexpr int NCS = C0 + NCS0 <= NCD ? NCS0 : NCD - C0;
    const Digest &d = a.dig;
    double out[NAB][NCS];
    eri_valu_compute<LB, LK, NAB, NCD, GB, GK, true, C0, NCS>(a, I, J, out);
    if (d.Jb) {
#pragma unroll
        for (int ab = 0; ab < NAB; ++ab)
#pragma unroll
            for (int j = 0; j < NCS; ++j) jb[ab] = fma(out[ab][j], d.Dk[J + d.nk * (C0 + j)], jb[ab]);
    }
    if (d.Jk) {
#pragma unroll
        for (int j = 0; j < NCS; ++j) {
            double v = 0.0;
            if (live) {
#pragma unroll
                for (int ab = 0; ab < NAB; ++ab) v = fma(out[ab][j], d.Db[I + d.nb * ab], v);
            }
            v += __shfl_xor(v, 1);
            v += __shfl_xor(v, 2);
            v += __shfl_xor(v, 4);
            if ((lane & 7) == 0) atomicAdd(d.Jk + J + d.nk * (C0 + j), v);
        }
    }
    if constexpr (C0 + NCS < NCD) eri_valu_digest_part<LB, LK, NAB, NCD, GB, GK, C0 + NCS>(a, I, J, live, lane, jb);
}

// Digestion of shellsets (I0, J), one per lane, J uniform over the wave (a
// ragged tile: ket pair J and 64 bra pairs of its prefix I < nI): each lane
// adds its Jb rows with atomics, the Jk terms are summed over groups of 8
// lanes first.  Every lane of the wave must call it; lanes with I0 >= nI
// compute a copy of bra pair nI - 1 and contribute nothing.
template <int LB, int LK, int NAB, int NCD, bool GB, bool GK>
__device__ __forceinline__ void eri_valu_digest_one(const EriArgs &a, const int I0, const int J, const int nI)
{
    const int lane = (int)threadIdx.x & 63;
    const bool live = I0 < nI;
    const int I = live ? I0 : nI - 1;
    const Digest &d = a.dig;
    if constexpr (valu_part_cols<LB, NAB, NCD, GB>() < NCD) {
        double jb[NAB];
#pragma unroll
        for (int ab = 0; ab < NAB; ++ab) jb[ab] = 0.0;
        eri_valu_digest_part<LB, LK, NAB, NCD, GB, GK, 0>(a, I, J, live, lane, jb);
        if (d.Jb && live)
#pragma unroll
            for (int ab = 0; ab < NAB; ++ab) atomicAdd(d.Jb + I + d.nb * ab, jb[ab]);
        return;
    }
    double out[NAB][NCD];
    eri_valu_compute<LB, LK, NAB, NCD, GB, GK>(a, I, J, out);
    if (d.Jb && live) {
#pragma unroll
        for (int ab = 0; ab < NAB; ++ab) {
            double v = 0.0;
#pragma unroll
            for (int cd = 0; cd < NCD; ++cd) v = fma(out[ab][cd], d.Dk[J + d.nk * cd], v);
            atomicAdd(d.Jb + I + d.nb * ab, v);
        }
    }
    if (d.Jk) {
#pragma unroll
        for (int cd = 0; cd < NCD; ++cd) {
            double v = 0.0;
            if (live) {
#pragma unroll
                for (int ab = 0; ab < NAB; ++ab) v = fma(out[ab][cd], d.Db[I + d.nb * ab], v);
            }
            v += __shfl_xor(v, 1);
            v += __shfl_xor(v, 2);
            v += __shfl_xor(v, 4);
            if ((lane & 7) == 0) atomicAdd(d.Jk + J + d.nk * cd, v);
        }
    }
}

#define MDX_VALU_INSTANCES(X)                                                                       \
    /* 4-centre, spherical and Cartesian, l <= 2 per shell, bra order >= ket order */              \
    X(0, 0, 1, 1, false, false)                                                                     \
    X(1, 0, 3, 1, false, false) X(1, 1, 3, 3, false, false)                                         \
    X(2, 0, 9, 1, false, false) X(2, 1, 9, 3, false, false) X(2, 2, 9, 9, false, false)             \
    X(2, 2, 9, 5, false, false) X(2, 2, 9, 6, false, false)                                         \
    X(2, 0, 5, 1, false, false) X(2, 1, 5, 3, false, false) X(2, 2, 5, 9, false, false)             \
    X(2, 2, 5, 5, false, false)                                                                     \
    X(2, 0, 6, 1, false, false) X(2, 1, 6, 3, false, false) X(2, 2, 6, 9, false, false)             \
    X(2, 2, 6, 6, false, false)                                                                     \
    X(3, 0, 15, 1, false, false) X(3, 1, 15, 3, false, false) X(3, 2, 15, 9, false, false)          \
    X(3, 2, 15, 5, false, false)                                                                    \
    X(3, 0, 18, 1, false, false) X(3, 1, 18, 3, false, false) X(3, 2, 18, 9, false, false)          \
    X(3, 2, 18, 6, false, false)                                                                    \
    X(4, 0, 25, 1, false, false) X(4, 1, 25, 3, false, false) X(4, 2, 25, 5, false, false)          \
    X(4, 0, 36, 1, false, false) X(4, 1, 36, 3, false, false) X(4, 2, 36, 6, false, false)          \
    /* 3-centre (X|cd), solid single function (grouped) or Cartesian (unit partner) */             \
    X(0, 0, 1, 1, true, false) X(0, 1, 1, 3, true, false) X(0, 2, 1, 9, true, false)                \
    X(0, 2, 1, 5, true, false) X(0, 4, 1, 25, true, false)                                          \
    X(1, 0, 3, 1, true, false) X(1, 1, 3, 3, true, false) X(1, 2, 3, 9, true, false)                \
    X(1, 2, 3, 5, true, false) X(1, 4, 3, 25, true, false)                                          \
    X(2, 2, 5, 5, true, false) X(2, 2, 5, 9, true, false) X(2, 4, 5, 25, true, false)               \
    X(0, 2, 1, 6, false, false) X(1, 2, 3, 6, false, false) X(2, 2, 6, 6, false, false)             \
    X(0, 4, 1, 36, false, false) X(1, 4, 3, 36, false, false)                                       \
    /* 2-centre (a|c) */                                                                            \
    X(0, 0, 1, 1, true, true) X(1, 1, 3, 3, true, true) X(2, 2, 5, 5, true, true)                   \
    X(2, 0, 5, 1, true, true) X(2, 1, 5, 3, true, true) X(1, 0, 3, 1, true, true)                   \
    X(3, 3, 7, 7, true, true) X(4, 4, 9, 9, true, true) X(3, 2, 7, 5, true, true)                   \
    X(1, 1, 3, 3, false, false) X(2, 2, 6, 6, false, false)

}  // namespace mdx
