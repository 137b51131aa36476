// mfma_common.h -- pieces shared by the matrix-core integral kernels:
// the FP64 MFMA wrapper and the one-axis sweeps of the Hermite recursion
// (Eq. (31)) over an (L+1)^3 cube in LDS with bank-padded strides.
#pragma once

#include <utility>

#include "cube_layouts.h"
#include "eri_common.h"
#include "digest.h"
#include "kernels.h"

namespace mdx {

typedef double d4 __attribute__((ext_vector_type(4)));

__device__ __forceinline__ d4 mfma(double a, double b, d4 c)
{
    return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0);
}

// LDS layout of the [r]^(0) tables, D = L+1 per axis: entry (t, u, v) of a
// table at t*ST + u*SU + v, the tables of successive primitive quartets SIZE
// doubles apart.  Only entries with t + u + v <= L exist.
//  LAY < 1000: a D^3 cube padded by LAY = 100*pu + 10*pt + pc (u stride D+pu,
//              t stride D*SU+pt, size D*ST+pc); padding spreads the rows of an
//              MFMA operand gather and the lanes of a sweep over LDS banks.
//  LAY = CUBE_LAY_COMPACT: the generated compact layout, whose tables fill each
//              other's unused corners (at most QMAX tables per block).
// The best choice depends on D and on the access mix, so kernel instances
// carry it as a parameter and the autotuner chooses among them.
constexpr int CUBE_LAY_COMPACT = 1000;

template <int D_, int LAY>
struct Cube {
    static constexpr int D = D_;
    static constexpr bool COMPACT = LAY == CUBE_LAY_COMPACT;
    static_assert(COMPACT ? (D >= 1 && D <= CUBE_COMPACT_DMAX) : (LAY >= 0 && LAY < 1000), "table layout");
    static constexpr int SU = COMPACT ? CUBE_COMPACT[D - 1][1] : D + LAY / 100;
    static constexpr int ST = COMPACT ? CUBE_COMPACT[D - 1][2] : D * SU + (LAY / 10) % 10;
    static constexpr int SIZE = COMPACT ? CUBE_COMPACT[D - 1][3] : D * ST + LAY % 10;
    static constexpr int QMAX = COMPACT ? CUBE_COMPACT_QMAX : 1 << 20;
    static_assert(ST >= SU && SU >= 1, "largest entry of a table is (D-1, 0, 0)");
    static constexpr int SPAN = (D - 1) * ST + 1;   // extent of one table
    // doubles spanned by n consecutive tables
    __host__ __device__ static constexpr int words(int n) { return n > 0 ? (n - 1) * SIZE + SPAN : 0; }
    __host__ __device__ static constexpr int off(int t, int u, int v) { return t * ST + u * SU + v; }
    // offset of Hermite k
    __host__ __device__ static constexpr int off(int k)
    {
        const Tuv r = herm_tuv(k);
        return off(r.t, r.u, r.v);
    }
};

// table offsets of the ket rows as the pair data stores them: non-terminal
// Hermites, padding to a multiple of 4, terminal Hermites, padding (0)
template <class CB, int LK, int N>
struct KetRowOffsets {
    int o[N];
    constexpr KetRowOffsets() : o{}
    {
        constexpr int NKN = nherm(LK - 1), NTPAD = round_up(NKN, 4), RPB = NTPAD + ncart(LK);
        for (int k = 0; k < N; ++k) o[k] = k < NKN ? CB::off(k) : (k >= NTPAD && k < RPB ? CB::off(NKN + k - NTPAD) : 0);
    }
};

// a[g] for a lane group g in 0..3 (compile-time a)
__device__ __forceinline__ int sel4(int a0, int a1, int a2, int a3, int g)
{
    return (g & 2) ? ((g & 1) ? a3 : a2) : ((g & 1) ? a1 : a0);
}

// Shellset (I, J) of this workgroup in a plain matrix-core launch, and nI, the
// bra pairs of ket J; false: the workgroup has no shellset.
__device__ __forceinline__ bool mfma_block_shellset(const EriArgs &a, int &I, int &J, int &nI)
{
    if (a.diag) {   // diagonal shellsets (I = J) only
        J = blockIdx.x;
        I = J;
    } else if (a.tile_off) {   // ragged batch: one shellset per tile
        ragged_tile(a.tile_off, a.nket, blockIdx.x, J, I);
    } else {
        // blocks of 16 bra x 8 ket pairs, dealt to the XCDs in contiguous
        // ranges: the workgroups resident on an XCD share 16 bra and 8 ket H
        // blocks in its L2, and 16 consecutive bra pairs fill whole 128-byte
        // output lines.  Successive blocks step through the ket pairs with the
        // same 16 bra pairs, so each bra H is read once per XCD range and each
        // ket H once per 16 bra pairs.
        const int t = xcd_tile(blockIdx.x, gridDim.x);
        const int blk = t >> 7, e = t & 127;
        const int nkr = gridDim.x / (128 * a.tiles_per_J);   // blocks of ket pairs
        I = (blk / nkr) * MFMA_BRA_RUN + (e % MFMA_BRA_RUN);
        J = (blk % nkr) * MFMA_KET_RUN + (e / MFMA_BRA_RUN);
    }
    if (J >= a.nket) return false;
    nI = a.diag ? J + 1 : (a.om.count ? a.om.count[J] : a.nbra);
    return I < nI;
}

// Bra unit U (NBI consecutive bra pairs or functions from I0 = U*NBI) and ket
// pair J of this workgroup: dense batches in the XCD-aware block order of the other
// matrix-core launches, ragged batches one unit per tile.
template <int NBI>
__device__ __forceinline__ bool multi_block_unit(const EriArgs &a, int &I0, int &J, int &nI)
{
    int U;
    if (a.tile_off) {
        ragged_tile(a.tile_off, a.nket, blockIdx.x, J, U);
    } else {
        const int t = xcd_tile(blockIdx.x, gridDim.x);
        const int blk = t >> 7, e = t & 127;
        const int nkr = gridDim.x / (128 * a.tiles_per_J);   // blocks of ket pairs
        U = (blk / nkr) * MFMA_BRA_RUN + (e % MFMA_BRA_RUN);
        J = (blk % nkr) * MFMA_KET_RUN + (e / MFMA_BRA_RUN);
    }
    if (J >= a.nket) return false;
    nI = a.om.count ? a.om.count[J] : a.nbra;
    I0 = U * NBI;
    return I0 < nI;
}

// Sweep slots: the tables of a sweep round are KP consecutive blocks of nqmax
// slots, one block per ket primitive; slot Q holds a quartet when its index
// within the block is below NQ (the chunk's bra primitives).
__device__ __forceinline__ bool slot_live(int Q, int NQT, int NQ, int nqmax)
{
    if (Q >= NQT) return false;
    while (Q >= nqmax) Q -= nqmax;
    return Q < NQ;
}

// [r]^(0) of one primitive quartet, Eq. (31), as three one-axis sweeps over
// the table CB (a Cube, D = L+1).  Each sweep handles columns of a
// compile-time length, so it is fully unrolled: no predication, no wasted
// work on short columns, recursion state in registers.
//   z, y sweep: per v, raise z to v in registers, then y:
//               [0 u v]^(m), m <= M-u (M = L-v) -> cube position (m, u, v)
//   x sweep:  per (u, v), [t u v]^(0), t <= M (M = L-u-v) -> (t, u, v)
// Intermediate columns are stored at (m, u, v) and overwritten in place by
// the lane that owns them.
template <class CB, int M>
__device__ __forceinline__ void ysweep(double *__restrict__ cv /* table + (0, 0, v) */, const double *__restrict__ S, double Y,
                                       double Z)
{
    // z first: [0 0 v]^(m), m <= M, for v = L - M, from [0]^(m) (registers only)
    constexpr int D = CB::D, L = D - 1, V = L - M, SU = CB::SU, ST = CB::ST;
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
        cv[m * ST] = c[m];
        p[m] = 0.0;
    }
#pragma unroll
    for (int u = 1; u <= M; ++u) {
        double n[M + 1];
#pragma unroll
        for (int m = 0; m <= M - u; ++m) n[m] = u > 1 ? fma((double)(u - 1), p[m + 1], Y * c[m + 1]) : Y * c[m + 1];
#pragma unroll
        for (int m = 0; m <= M - u; ++m) cv[m * ST + u * SU] = n[m];
#pragma unroll
        for (int m = 0; m <= M - u; ++m) {
            p[m] = c[m];
            c[m] = n[m];
        }
        p[M - u + 1] = c[M - u + 1];
    }
}

template <class CB, int M>
__device__ __forceinline__ void xsweep(double *__restrict__ cuv /* table + (0, u, v) */, double X)
{
    constexpr int ST = CB::ST;
    double c[M + 1], p[M + 1];
#pragma unroll
    for (int m = 0; m <= M; ++m) {
        c[m] = cuv[m * ST];
        p[m] = 0.0;
    }
#pragma unroll
    for (int t = 1; t <= M; ++t) {
        double n[M + 1];
#pragma unroll
        for (int m = 0; m <= M - t; ++m) n[m] = t > 1 ? fma((double)(t - 1), p[m + 1], X * c[m + 1]) : X * c[m + 1];
        cuv[t * ST] = n[0];
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
template <class CB, int NW, int W, int M>
__device__ __forceinline__ void ycol(double *cq, const double *Sq, double Y, double Z)
{
    constexpr int v = CB::D - 1 - M;
    if constexpr (v % NW == W) ysweep<CB, M>(cq + v, Sq, Y, Z);
}

template <class CB, int NW, int W, int... Ms>
__device__ __forceinline__ void ywave(double *cube, const double *S, const double *PQ, int NQ, int NQT, int nqmax,
                                      int lane, std::integer_sequence<int, Ms...>)
{
    if (!slot_live(lane, NQT, NQ, nqmax)) return;
    double *cq = cube + lane * CB::SIZE;
    const double *Sq = S + lane * CB::D;
    const double Y = PQ[lane * 4 + 1], Z = PQ[lane * 4 + 2];
    (ycol<CB, NW, W, Ms>(cq, Sq, Y, Z), ...);
}

template <class CB, int NW, int W, int NQCT, int M>
__device__ __forceinline__ void xcols(double *cube, const double *PQ, int NQ, int NQT, int nqmax, int lane)
{
    constexpr int L = CB::D - 1, s = L - M;
    if constexpr (M > 0 && s % NW == W) {   // order 0 columns are complete after the y sweep
        constexpr int R = (NQCT * (s + 1) + 63) / 64;
        const int n = NQT * (s + 1);
#pragma unroll
        for (int r = 0; r < R; ++r) {
            const int e = lane + 64 * r;
            const int q = e / (s + 1), v = e - q * (s + 1), u = s - v;
            if (e < n && slot_live(q, NQT, NQ, nqmax)) xsweep<CB, M>(cube + q * CB::SIZE + CB::off(0, u, v), PQ[q * 4]);
        }
    }
}

template <class CB, int NW, int W, int NQCT, int... Ms>
__device__ __forceinline__ void xwave(double *cube, const double *PQ, int NQ, int NQT, int nqmax, int lane,
                                      std::integer_sequence<int, Ms...>)
{
    (xcols<CB, NW, W, NQCT, Ms>(cube, PQ, NQ, NQT, nqmax, lane), ...);
}

// One z/y column per branch region: the chains of a wave run one after the
// other, which keeps fewer registers live next to a large accumulator set.
template <class CB, int NW, int M>
__device__ __forceinline__ void ycol_branch(double *cube, const double *S, const double *PQ, int NQ, int NQT,
                                            int nqmax, int w, int lane)
{
    constexpr int v = CB::D - 1 - M;
    if (w == v % NW && slot_live(lane, NQT, NQ, nqmax))
        ysweep<CB, M>(cube + lane * CB::SIZE + v, S + lane * CB::D, PQ[lane * 4 + 1], PQ[lane * 4 + 2]);
}

template <class CB, int NW, int... Ms>
__device__ __forceinline__ void ysweeps_serial(double *cube, const double *S, const double *PQ, int NQ, int NQT,
                                               int nqmax, int w, int lane, std::integer_sequence<int, Ms...>)
{
    (ycol_branch<CB, NW, Ms>(cube, S, PQ, NQ, NQT, nqmax, w, lane), ...);
}

// z/y sweeps of the live slots Q < NQT (every wave calls this; wave w does its
// share); S and PQ are indexed by slot.  Requires NQT <= 64.  SER selects the
// column-per-branch form for register-heavy kernels.
template <class CB, int NW, bool SER, int... Ws>
__device__ __forceinline__ void ysweeps(double *cube, const double *S, const double *PQ, int NQ, int NQT, int nqmax,
                                        int w, int lane, std::integer_sequence<int, Ws...>)
{
    if constexpr (SER)
        ysweeps_serial<CB, NW>(cube, S, PQ, NQ, NQT, nqmax, w, lane, std::make_integer_sequence<int, CB::D>{});
    else
        ((w == Ws ? ywave<CB, NW, Ws>(cube, S, PQ, NQ, NQT, nqmax, lane, std::make_integer_sequence<int, CB::D>{})
                  : void()),
         ...);
}

// x sweep of all columns of order M in a branch region of its own
template <class CB, int NW, int M>
__device__ __forceinline__ void xorder_branch(double *cube, const double *PQ, int NQ, int NQT, int nqmax, int w,
                                              int lane)
{
    constexpr int L = CB::D - 1, s = L - M;
    if (M > 0 && w == s % NW)
        for (int e = lane; e < NQT * (s + 1); e += 64) {
            const int q = e / (s + 1), v = e - q * (s + 1), u = s - v;
            if (slot_live(q, NQT, NQ, nqmax)) xsweep<CB, M>(cube + q * CB::SIZE + CB::off(0, u, v), PQ[q * 4]);
        }
}

template <class CB, int NW, int... Ms>
__device__ __forceinline__ void xsweeps_serial(double *cube, const double *PQ, int NQ, int NQT, int nqmax, int w,
                                               int lane, std::integer_sequence<int, Ms...>)
{
    (xorder_branch<CB, NW, Ms>(cube, PQ, NQ, NQT, nqmax, w, lane), ...);
}

// x sweeps (after the z/y sweeps of all waves are visible); NQCT bounds NQT;
// SER as for ysweeps
template <class CB, int NW, int NQCT, bool SER, int... Ws>
__device__ __forceinline__ void xsweeps(double *cube, const double *PQ, int NQ, int NQT, int nqmax, int w, int lane,
                                        std::integer_sequence<int, Ws...>)
{
    if constexpr (SER)
        xsweeps_serial<CB, NW>(cube, PQ, NQ, NQT, nqmax, w, lane, std::make_integer_sequence<int, CB::D>{});
    else
        ((w == Ws ? xwave<CB, NW, Ws, NQCT>(cube, PQ, NQ, NQT, nqmax, lane, std::make_integer_sequence<int, CB::D>{})
                  : void()),
         ...);
}

}  // namespace mdx
