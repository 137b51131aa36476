// eri_prim.hip -- plain launches of the single-primitive matrix-core kernel:
// one shellset per workgroup, (I, J) from the block index.
#include "eri_prim.h"

namespace mdx {

template <int LB, int LK, int NTAB, int NTCD, int NW, int WPE, int NB, bool TAIL, int LAY>
__global__ void __launch_bounds__(64 * NW) __attribute__((amdgpu_waves_per_eu(WPE))) eri_prim_kernel(EriArgs a)
{
    int I0, J, nI;
    if constexpr (NB == 1) {
        if (!mfma_block_shellset(a, I0, J, nI)) return;   // whole workgroup
    } else {
        if (!multi_block_unit<NB>(a, I0, J, nI)) return;
    }
    eri_prim_unit<LB, LK, NTAB, NTCD, NW, NB, TAIL, LAY>(a, I0, J, nI);
}

template <int LB, int LK, int NTAB, int NTCD, int NW, int WPE, int NB, bool TAIL, int LAY>
static bool launch_prim(const EriArgs &a, int nblocks, hipStream_t s)
{
    // one primitive pair per bra and per ket pair, or one primitive combination
    // of contracted pairs at a time (checked when the class is planned)
    if ((!a.prim_expand && (a.bra.kmax != 1 || a.ket.kmax != 1)) || (NB > 1 && a.diag)) return false;
    // the VALU tail assumes 16k+1 functions on both sides
    if (TAIL && (a.nab != 16 * (NTAB - 1) + 1 || a.ncd != 16 * (NTCD - 1) + 1)) return false;
    const size_t lds = prim_lds_bytes<LB, LK, NTAB, NTCD, NW, NB, TAIL, LAY>();
    if (lds > 160 * 1024) return false;
    auto kern = eri_prim_kernel<LB, LK, NTAB, NTCD, NW, WPE, NB, TAIL, LAY>;
    static bool lds_set = false;
    if (lds > 64 * 1024 && !lds_set) {
        if (hipFuncSetAttribute((const void *)kern, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds) != hipSuccess)
            return false;
        lds_set = true;
    }
    hipLaunchKernelGGL(kern, dim3(nblocks), dim3(64 * NW), lds, s, a);
    return true;
}

static bool pkey_is(const EriKey &k, int lb, int lk, int nab, int ncd)
{
    return !k.GK && !k.GB && k.LB == lb && k.LK == lk && k.NAB == nab && k.NCD == ncd;
}

int eri_prim_variants(const EriKey &k)
{
    int n = 0;
#define MDX_PCOUNT(lb, lk, nab, ncd, ntab, ntcd, nw, wpe, nb, tail, lay) \
    if (pkey_is(k, lb, lk, nab, ncd)) ++n;
    MDX_PRIM_INSTANCES(MDX_PCOUNT)
#undef MDX_PCOUNT
    return n;
}

int eri_prim_bra_per_tile(const EriKey &k, int variant)
{
    int n = 0;
#define MDX_PBPT(lb, lk, nab, ncd, ntab, ntcd, nw, wpe, nb, tail, lay) \
    if (pkey_is(k, lb, lk, nab, ncd) && ++n == variant) return nb;
    MDX_PRIM_INSTANCES(MDX_PBPT)
#undef MDX_PBPT
    return 1;
}

bool eri_prim_launch(const EriKey &k, const EriArgs &a, int nblocks, int variant, hipStream_t s)
{
    int n = 0;
#define MDX_PTRY(lb, lk, nab, ncd, ntab, ntcd, nw, wpe, nb, tail, lay) \
    if (pkey_is(k, lb, lk, nab, ncd) && ++n == variant)           \
        return launch_prim<lb, lk, ntab, ntcd, nw, wpe, nb, tail, lay>(a, nblocks, s);
    MDX_PRIM_INSTANCES(MDX_PTRY)
#undef MDX_PTRY
    return false;
}

}  // namespace mdx
