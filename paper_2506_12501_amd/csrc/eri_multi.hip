// eri_multi.hip -- plain launches of the several-shellsets-per-workgroup
// 3-centre kernel: a unit of NBI bra functions against one ket pair per
// workgroup.
#include "eri_multi.h"

namespace mdx {

template <int LB, int LK, int NTAB, int NTCD, int NW, int SPW, int LAY>
__global__ void __launch_bounds__(64 * NW) eri_multi_kernel(EriArgs a)
{
    int I0, J, nI;
    if (!multi_block_unit<NW * SPW>(a, I0, J, nI)) return;   // whole workgroup
    eri_multi_unit<LB, LK, NTAB, NTCD, NW, SPW, LAY>(a, I0, J, nI);
}

template <int LB, int LK, int NTAB, int NTCD, int NW, int SPW, int LAY>
static bool launch_multi(const EriArgs &a, int nblocks, hipStream_t s)
{
    // ket pairs of one primitive pair, bra units of NBI (checked when the class is planned)
    if (a.ket.kmax != 1 || a.diag) return false;
    const size_t lds = multi_lds_bytes<LB, LK, NTAB, NTCD, NW, SPW, LAY>();
    if (lds > 160 * 1024) return false;
    auto kern = eri_multi_kernel<LB, LK, NTAB, NTCD, NW, SPW, LAY>;
    static bool lds_set = false;
    if (lds > 64 * 1024 && !lds_set) {
        if (hipFuncSetAttribute((const void *)kern, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds) != hipSuccess)
            return false;
        lds_set = true;
    }
    hipLaunchKernelGGL(kern, dim3(nblocks), dim3(64 * NW), lds, s, a);
    return true;
}

static bool mkey_is3(const EriKey &k, int lb, int lk, int nab, int ncd)
{
    return k.GB && !k.GK && k.LB == lb && k.LK == lk && k.NAB == nab && k.NCD == ncd;
}

int eri_multi_variants(const EriKey &k)
{
    int n = 0;
#define MDX_MCOUNT(lb, lk, nab, ncd, ntab, ntcd, nw, spw, lay) \
    if (mkey_is3(k, lb, lk, nab, ncd)) ++n;
    MDX_MULTI_INSTANCES(MDX_MCOUNT)
#undef MDX_MCOUNT
    return n;
}

int eri_multi_bra_per_tile(const EriKey &k, int variant)
{
    int n = 0;
#define MDX_MBPT(lb, lk, nab, ncd, ntab, ntcd, nw, spw, lay) \
    if (mkey_is3(k, lb, lk, nab, ncd) && ++n == variant) return nw * spw;
    MDX_MULTI_INSTANCES(MDX_MBPT)
#undef MDX_MBPT
    return 1;
}

bool eri_multi_launch(const EriKey &k, const EriArgs &a, int nblocks, int variant, hipStream_t s)
{
    int n = 0;
#define MDX_MTRY(lb, lk, nab, ncd, ntab, ntcd, nw, spw, lay)   \
    if (mkey_is3(k, lb, lk, nab, ncd) && ++n == variant)        \
        return launch_multi<lb, lk, ntab, ntcd, nw, spw, lay>(a, nblocks, s);
    MDX_MULTI_INSTANCES(MDX_MTRY)
#undef MDX_MTRY
    return false;
}

}  // namespace mdx
