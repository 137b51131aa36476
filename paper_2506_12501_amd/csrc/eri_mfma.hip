// eri_mfma.hip -- plain launches of the matrix-core integral kernel: one
// shellset per workgroup, (I, J) from the block index.
#include "eri_mfma.h"

namespace mdx {

// DIG: contract with the densities of a.dig at the store (digestion)
template <int LB, int LK, int NTAB, int NTCD, int NTG, int MTW, int NW, bool GB, int WPE, int LAY, int KP, bool DIG>
__global__ void __launch_bounds__(64 * NW) __attribute__((amdgpu_waves_per_eu(WPE)))
eri_mfma_kernel(EriArgs a)
{
    int I, J, nI;
    if (!mfma_block_shellset(a, I, J, nI)) return;   // whole workgroup
    eri_mfma_shellset<LB, LK, NTAB, NTCD, NTG, MTW, NW, GB, LAY, KP, DIG>(a, I, J, nI);
}

template <int LB, int LK, int NTAB, int NTCD, int NTG, int MTW, int NW, bool GB, int WPE, int LAY, int KP,
          bool DIG = false>
static bool launch_mfma(const EriArgs &a0, int nblocks, hipStream_t s)
{
    EriArgs a = a0;
    constexpr int NHB = GB ? ncart(LB) : nherm(LB);
    a.nqmax = GB ? 1 : std::min(a.bra.kmax, (NW * MTW * 16) / NHB + 2);
    const size_t lds = mfma_lds_bytes<LB, LK, NTAB, NTCD, NTG, MTW, NW, GB, LAY, KP, DIG>(a.nqmax, a.ket.kmax);
    if (lds > 160 * 1024) return false;
    auto kern = eri_mfma_kernel<LB, LK, NTAB, NTCD, NTG, MTW, NW, GB, WPE, LAY, KP, DIG>;
    static size_t lds_set = 0;   // largest dynamic LDS granted to this instance so far
    if (lds > 64 * 1024 && lds > lds_set) {
        if (hipFuncSetAttribute((const void *)kern, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds) != hipSuccess)
            return false;
        lds_set = lds;
    }
    hipLaunchKernelGGL(kern, dim3(nblocks), dim3(64 * NW), lds, s, a);
    return true;
}

static bool key_is(const EriKey &k, int lb, int lk, int nab, int ncd, bool gb)
{
    return !k.GK && k.LB == lb && k.LK == lk && k.NAB == nab && k.NCD == ncd && k.GB == gb;
}

// Digestion kernels exist for the first shape (variant 1) of each class only
// (first_of_class, eri_mfma.h).
template <bool FIRST, int LB, int LK, int NTAB, int NTCD, int NTG, int MTW, int NW, bool GB, int WPE, int LAY, int KP>
struct DigestLaunch {
    static bool go(const EriArgs &, int, hipStream_t) { return false; }
};
template <int LB, int LK, int NTAB, int NTCD, int NTG, int MTW, int NW, bool GB, int WPE, int LAY, int KP>
struct DigestLaunch<true, LB, LK, NTAB, NTCD, NTG, MTW, NW, GB, WPE, LAY, KP> {
    static bool go(const EriArgs &a, int nblocks, hipStream_t s)
    {
        return launch_mfma<LB, LK, NTAB, NTCD, NTG, MTW, NW, GB, WPE, LAY, KP, true>(a, nblocks, s);
    }
};

static int eri_mfma_only_variants(const EriKey &k)
{
    int n = 0;
#define MDX_COUNT(lb, lk, nab, ncd, gb, ntab, ntcd, ntg, mtw, nw, wpe, lay, kp) \
    if (key_is(k, lb, lk, nab, ncd, gb)) ++n;
    MDX_MFMA_INSTANCES(MDX_COUNT)
#undef MDX_COUNT
    return n;
}

int eri_mfma_variants(const EriKey &k)
{
    return eri_mfma_only_variants(k) + eri_prim_variants(k) + eri_multi_variants(k);
}

bool eri_mfma_has(const EriKey &k) { return eri_mfma_variants(k) > 0; }

int eri_mfma_variant_kind(const EriKey &k, int variant)
{
    variant -= eri_mfma_only_variants(k);
    if (variant <= 0) return MFMA_GENERAL;
    return variant <= eri_prim_variants(k) ? MFMA_PRIM : MFMA_MULTI;
}

int eri_mfma_bra_per_tile(const EriKey &k, int variant)
{
    const int v = variant - eri_mfma_only_variants(k);
    switch (eri_mfma_variant_kind(k, variant)) {
    case MFMA_PRIM: return eri_prim_bra_per_tile(k, v);
    case MFMA_MULTI: return eri_multi_bra_per_tile(k, v - eri_prim_variants(k));
    default: return 1;
    }
}

bool eri_mfma_launch(const EriKey &k, const EriArgs &a, int nblocks, int variant, hipStream_t s)
{
    if (a.dig.on) {   // the class's first shape (the caller asks for variant 1)
        if (variant != 1) return false;
#define MDX_DIG(lb, lk, nab, ncd, gb, ntab, ntcd, ntg, mtw, nw, wpe, lay, kp)                                  \
    if (key_is(k, lb, lk, nab, ncd, gb))                                                                   \
        return DigestLaunch<first_of_class(MfmaRow{lb, lk, nab, ncd, gb, ntab, ntcd, ntg, mtw, nw, wpe, lay, kp}), \
                            lb, lk, ntab, ntcd, ntg, mtw, nw, gb, wpe, lay, kp>::go(a, nblocks, s);
        MDX_MFMA_INSTANCES(MDX_DIG)
#undef MDX_DIG
        return false;
    }
    int n = 0;
#define MDX_TRY(lb, lk, nab, ncd, gb, ntab, ntcd, ntg, mtw, nw, wpe, lay, kp)                     \
    if (key_is(k, lb, lk, nab, ncd, gb) && ++n == variant)                             \
        return launch_mfma<lb, lk, ntab, ntcd, ntg, mtw, nw, gb, wpe, lay, kp>(a, nblocks, s);
    MDX_MFMA_INSTANCES(MDX_TRY)
#undef MDX_TRY
    variant -= n;
    const int np = eri_prim_variants(k);
    return variant <= np ? eri_prim_launch(k, a, nblocks, variant, s) : eri_multi_launch(k, a, nblocks, variant - np, s);
}

}  // namespace mdx
