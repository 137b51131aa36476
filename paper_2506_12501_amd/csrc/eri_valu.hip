// eri_valu.hip -- plain launches of the register integral kernel: one lane
// per shellset, 64 consecutive bra pairs of one ket pair per wave.
#include "eri_valu.h"

namespace mdx {

template <int LB, int LK, int NAB, int NCD, bool GB, bool GK>
__global__ void __launch_bounds__(64) eri_valu_kernel(EriArgs a)
{
    int J, I;
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
    const int nI = a.diag ? J + 1 : (a.om.count ? a.om.count[J] : a.nbra);
    if (I >= nI) return;
    eri_valu_shellset<LB, LK, NAB, NCD, GB, GK>(a, I, J, nI);
}

template <int LB, int LK, int NAB, int NCD, bool GB, bool GK>
static void launch_valu(const EriArgs &a, int nblocks, hipStream_t s)
{
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
