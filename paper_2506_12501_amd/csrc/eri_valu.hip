// eri_valu.hip -- plain launches of the register integral kernel: one lane
// per shellset, 64 consecutive bra pairs of one ket pair per wave.
#include "eri_valu.h"

namespace mdx {

template <int LB, int LK, int NAB, int NCD, bool GB, bool GK>
__global__ void __launch_bounds__(64) eri_valu_kernel(EriArgs a)
{
    int J, I;
    if (a.diag == 2) {   // paired batch: quartet q = (bra q, ket q), one per lane
        I = J = blockIdx.x * 64 + (int)threadIdx.x;
        if (J >= a.nket) return;
        eri_valu_shellset<LB, LK, NAB, NCD, GB, GK, false>(a, I, J, a.nbra);
        return;
    }
    if (a.diag) {   // diagonal shellsets (I = J) only: lane 0 of block J
        J = blockIdx.x;
        I = J + (int)threadIdx.x;
    } else if (a.tile_off) {   // ragged batch: tiles of 64 bra pairs
        int t0;
        ragged_tile(a.tile_off, a.nket, blockIdx.x, J, t0);
        I = t0 * 64 + (int)threadIdx.x;
    } else {
        const int t = xcd_tile(blockIdx.x, gridDim.x);
        J = t / a.tiles_per_J;
        I = (t % a.tiles_per_J) * 64 + (int)threadIdx.x;
    }
    J = __builtin_amdgcn_readfirstlane(J);   // one ket pair per wave: its data become scalar loads
    const int nI = a.diag ? J + 1 : (a.om.count ? load_const(a.om.count + J) : a.nbra);
    if (I >= nI) return;
    eri_valu_shellset<LB, LK, NAB, NCD, GB, GK>(a, I, J, nI);
}

// Digestion (dense batches): a workgroup takes 64 bra pairs, one per lane,
// and valu_dig_nj consecutive ket pairs; each lane keeps its Jb rows in
// registers over those ket pairs and adds them once, while the Jk terms of
// one ket pair are summed over groups of 8 lanes before their atomic adds.  Lanes past
// the last bra pair compute a copy of it and contribute nothing.  Over its
// 16 ket pairs a lane also keeps reusing its bra pair's data; shellsets of
// more than 81 integrals take one ket pair per workgroup (their registers are
// spent on the shellset itself).  Ragged batches (plans: ket pair J takes the
// first count[J] bra pairs) go tile by tile as the storing kernel does: one
// ket pair and 64 bra pairs of its prefix per workgroup.
template <int NAB, int NCD>
constexpr int valu_dig_nj() { return NAB * NCD > 81 ? 1 : 16; }

template <int LB, int LK, int NAB, int NCD, bool GB, bool GK>
__global__ void __launch_bounds__(64) eri_valu_digest_kernel(EriArgs a)
{
    constexpr int NJ = valu_dig_nj<NAB, NCD>();
    const int lane = (int)threadIdx.x;
    int I0, J0, J1, nI;
    if (a.tile_off) {
        int J, t0;
        ragged_tile(a.tile_off, a.nket, blockIdx.x, J, t0);
        J = __builtin_amdgcn_readfirstlane(J);
        I0 = t0 * 64 + lane;
        J0 = J;
        J1 = J + 1;
        nI = load_const(a.om.count + J);   // >= 1: the tile exists
    } else {
        const int tiles = (a.nbra + 63) / 64;
        const int jc = blockIdx.x / tiles;
        I0 = (blockIdx.x % tiles) * 64 + lane;
        J0 = jc * NJ;
        J1 = min(a.nket, (jc + 1) * NJ);
        nI = a.nbra;
    }
    const bool live = I0 < nI;
    const int I = live ? I0 : nI - 1;
    const Digest &d = a.dig;
    double jb[NAB];
#pragma unroll
    for (int ab = 0; ab < NAB; ++ab) jb[ab] = 0.0;
    for (int J = J0; J < J1; ++J) {
        int zo = 0;   // large bra sides: an opaque zero keeps the Db loads inside the loop
        if constexpr (NAB > 9) asm volatile("" : "+v"(zo));   // (no NAB registers live across it)
        double out[NAB][NCD];
        eri_valu_compute<LB, LK, NAB, NCD, GB, GK>(a, I, J, out);
        if (d.Jb) {
#pragma unroll
            for (int ab = 0; ab < NAB; ++ab)
#pragma unroll
                for (int cd = 0; cd < NCD; ++cd) jb[ab] = fma(out[ab][cd], d.Dk[J + d.nk * cd], jb[ab]);
        }
        if (d.Jk) {
#pragma unroll
            for (int cd = 0; cd < NCD; ++cd) {
                double v = 0.0;
                if (live) {
#pragma unroll
                    for (int ab = 0; ab < NAB; ++ab) v = fma(out[ab][cd], d.Db[I + zo + d.nb * ab], v);
                }
                // sums over groups of 8 lanes; one atomic per group
                v += __shfl_xor(v, 1);
                v += __shfl_xor(v, 2);
                v += __shfl_xor(v, 4);
                if ((lane & 7) == 0) atomicAdd(d.Jk + J + d.nk * cd, v);
            }
        }
    }
    if (d.Jb && live) {
#pragma unroll
        for (int ab = 0; ab < NAB; ++ab) atomicAdd(d.Jb + I + d.nb * ab, jb[ab]);
    }
}

// Large dense batches with bra sides of 9 or more functions: a workgroup
// takes 64 bra pairs (one per lane) and valu_dig_nj consecutive ket pairs,
// one after the other, so that a lane re-reads its bra pair's data from L1
// instead of L2; every ket pair's row of stores stays coalesced over the lanes.
template <int LB, int LK, int NAB, int NCD, bool GB, bool GK>
__global__ void __launch_bounds__(64) eri_valu_multi_kernel(EriArgs a)
{
    constexpr int NJ = valu_dig_nj<NAB, NCD>();
    const int tiles = (a.nbra + 63) / 64;
    const int jc = blockIdx.x / tiles;
    const int I = (blockIdx.x % tiles) * 64 + (int)threadIdx.x;
    if (I >= a.nbra) return;
    const int J1 = min(a.nket, (jc + 1) * NJ);
    for (int J = jc * NJ; J < J1; ++J) eri_valu_shellset<LB, LK, NAB, NCD, GB, GK>(a, I, J, a.nbra);
}

template <int LB, int LK, int NAB, int NCD, bool GB, bool GK>
static void launch_valu(const EriArgs &a, int nblocks, hipStream_t s)
{
    constexpr int NJ = valu_dig_nj<NAB, NCD>();
    // (measured: 1.2-1.6x for bra sides of 9 and more functions; the smallest
    // classes are faster with one ket pair per workgroup)
    if (!a.dig.on && !a.diag && !a.tile_off && NJ > 1 && NAB >= 9 && (int64_t)nblocks >= 65536) {
        const int64_t nb = (int64_t)((a.nbra + 63) / 64) * ((a.nket + NJ - 1) / NJ);
        hipLaunchKernelGGL((eri_valu_multi_kernel<LB, LK, NAB, NCD, GB, GK>), dim3((unsigned)nb), dim3(64), 0, s, a);
        return;
    }
    if (a.dig.on && a.tile_off) {   // ragged: the tiles of the storing kernel
        hipLaunchKernelGGL((eri_valu_digest_kernel<LB, LK, NAB, NCD, GB, GK>), dim3(nblocks), dim3(64), 0, s, a);
        return;
    }
    if (a.dig.on) {
        constexpr int NJ = valu_dig_nj<NAB, NCD>();
        const int64_t nb = (int64_t)((a.nbra + 63) / 64) * ((a.nket + NJ - 1) / NJ);
        if (nb > INT32_MAX) return;   // the host splits batches long before this
        hipLaunchKernelGGL((eri_valu_digest_kernel<LB, LK, NAB, NCD, GB, GK>), dim3((unsigned)nb), dim3(64), 0, s, a);
        return;
    }
    hipLaunchKernelGGL((eri_valu_kernel<LB, LK, NAB, NCD, GB, GK>), dim3(nblocks), dim3(64), 0, s, a);
}

bool eri_valu_launch(const EriKey &k, const EriArgs &a, int nblocks, hipStream_t s)
{
#define MDX_TRY(lb, lk, nab, ncd, gb, gk)                                                    \
    if (k.LB == lb && k.LK == lk && k.NAB == nab && k.NCD == ncd && k.GB == gb && k.GK == gk) { \
        launch_valu<lb, lk, nab, ncd, gb, gk>(a, nblocks, s);                                 \
        return true;                                                                          \
    }
    MDX_VALU_INSTANCES(MDX_TRY)
#undef MDX_TRY
    return false;
}

bool eri_valu_has(const EriKey &k)
{
#define MDX_HAS(lb, lk, nab, ncd, gb, gk) \
    if (k.LB == lb && k.LK == lk && k.NAB == nab && k.NCD == ncd && k.GB == gb && k.GK == gk) return true;
    MDX_VALU_INSTANCES(MDX_HAS)
#undef MDX_HAS
    return false;
}

}  // namespace mdx
