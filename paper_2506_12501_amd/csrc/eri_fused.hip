// eri_fused.hip -- persistent work-queue launches of the integral kernels.
//
// One launch serves every batch of a plan that uses the same kernel instance.
// Its workgroups stay resident and take work items (a ragged tile of one
// batch) from a device counter until the items run out; the batch's kernel
// arguments are read from a device table.  The counter is reset by a fill
// kernel in the same graph before the launch.  Every workgroup leaves the loop
// as soon as the counter passes the item count, so the grid always drains.
#include "eri_mfma.h"
#include "eri_valu.h"

namespace mdx {

__device__ __forceinline__ int queue_batch(const QueueArgs &q, int w)
{
    int lo = 0, hi = q.nb;   // base[lo] <= w < base[hi]
    while (hi - lo > 1) {
        const int mid = (lo + hi) >> 1;
        if (q.base[mid] <= w) lo = mid;
        else hi = mid;
    }
    return lo;
}

// DIG: the batches' shellsets are contracted with their densities (a.dig)
// instead of stored
template <int LB, int LK, int NTAB, int NTCD, int NTG, int MTW, int NW, bool GB, int WPE, int LAY, int KP,
          bool DIG = false>
__global__ void __launch_bounds__(64 * NW) __attribute__((amdgpu_waves_per_eu(WPE)))
eri_mfma_queue(QueueArgs q)
{
    __shared__ int item;
    for (;;) {
        __syncthreads();   // the previous item is done with LDS and with `item`
        if (threadIdx.x == 0) item = atomicAdd(q.counter, 1);
        __syncthreads();
        const int w = __builtin_amdgcn_readfirstlane(item);
        if (w >= q.total) break;
        const int b = __builtin_amdgcn_readfirstlane(queue_batch(q, w));
        const EriArgs &a = q.desc[b];   // (a local copy would go to scratch: the body indexes its offset tables)
        int J, I;
        ragged_tile(a.tile_off, a.nket, w - q.base[b], J, I);
        const int nI = a.om.count[J];
        if (I < nI) eri_mfma_shellset<LB, LK, NTAB, NTCD, NTG, MTW, NW, GB, LAY, KP, DIG>(a, I, J, nI);
    }
}

// The smallest shellsets (up to 3 integrals) keep 5 or more waves per SIMD: their
// lanes wait on Boys-table reads, which only more resident waves hide.
template <int NAB, int NCD>
constexpr int valu_queue_waves() { return NAB * NCD <= 1 ? 8 : (NAB * NCD <= 3 ? 5 : 1); }

template <int LB, int LK, int NAB, int NCD, bool GB, bool GK, bool DIG = false>
__global__ void __launch_bounds__(64) __attribute__((amdgpu_waves_per_eu(valu_queue_waves<NAB, NCD>())))
eri_valu_queue(QueueArgs q)
{
    __shared__ int item;
    for (;;) {
        __syncthreads();
        if (threadIdx.x == 0) item = atomicAdd(q.counter, 1);
        __syncthreads();
        const int w = __builtin_amdgcn_readfirstlane(item);
        if (w >= q.total) break;
        const int b = __builtin_amdgcn_readfirstlane(queue_batch(q, w));
        const EriArgs a = load_const(q.desc + b);   // batch arguments: scalar loads
        int J, t0;
        ragged_tile(a.tile_off, a.nket, w - q.base[b], J, t0);
        J = __builtin_amdgcn_readfirstlane(J);   // uniform (derived from w); its ket data become scalar loads
        t0 = __builtin_amdgcn_readfirstlane(t0);
        const int I = t0 * 64 + (int)threadIdx.x;
        const int nI = load_const(a.om.count + J);
        if constexpr (DIG) eri_valu_digest_one<LB, LK, NAB, NCD, GB, GK>(a, I, J, nI);   // whole wave
        else if (I < nI) eri_valu_shellset<LB, LK, NAB, NCD, GB, GK>(a, I, J, nI);
    }
}

template <typename K>
static int resident_blocks(K kern, int nthreads, size_t lds)
{
    int n = 0;
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&n, kern, nthreads, lds) != hipSuccess) return 0;
    return n;
}

template <typename K>
static bool prepare(K kern, size_t lds)
{
    if (lds <= 64 * 1024) return true;
    return hipFuncSetAttribute((const void *)kern, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds) == hipSuccess;
}

static bool mkey_is(const EriKey &k, int lb, int lk, int nab, int ncd, bool gb)
{
    return !k.GK && k.LB == lb && k.LK == lk && k.NAB == nab && k.NCD == ncd && k.GB == gb;
}

// the persistent digesting form of a first-of-class instance (others: none)
template <bool FIRST, int LB, int LK, int NTAB, int NTCD, int NTG, int MTW, int NW, bool GB, int WPE, int LAY, int KP>
struct QueueDig {
    static int ready(size_t) { return 0; }
    static bool go(const QueueArgs &, int, size_t, hipStream_t) { return false; }
};
template <int LB, int LK, int NTAB, int NTCD, int NTG, int MTW, int NW, bool GB, int WPE, int LAY, int KP>
struct QueueDig<true, LB, LK, NTAB, NTCD, NTG, MTW, NW, GB, WPE, LAY, KP> {
    static int ready(size_t lds);
    static bool go(const QueueArgs &q, int nblocks, size_t lds, hipStream_t s)
    {
        hipLaunchKernelGGL((eri_mfma_queue<LB, LK, NTAB, NTCD, NTG, MTW, NW, GB, WPE, LAY, KP, true>), dim3(nblocks),
                           dim3(64 * NW), lds, s, q);
        return true;
    }
};

bool eri_mfma_config(const EriKey &k, int variant, int bra_kmax, int ket_kmax, int &nqmax, size_t &lds, int &nthreads,
                     bool dig)
{
    int n = 0;
#define MDX_CFG(lb, lk, nab, ncd, gb, ntab, ntcd, ntg, mtw, nw, wpe, lay, kp)                                  \
    if (mkey_is(k, lb, lk, nab, ncd, gb) && ++n == variant) {                                      \
        constexpr int NHB = gb ? ncart(lb) : nherm(lb);                                             \
        nqmax = gb ? 1 : std::min(bra_kmax, (nw * mtw * 16) / NHB + 2);                            \
        lds = dig ? mfma_lds_bytes<lb, lk, ntab, ntcd, ntg, mtw, nw, gb, lay, kp, true>(nqmax, ket_kmax)        \
                  : mfma_lds_bytes<lb, lk, ntab, ntcd, ntg, mtw, nw, gb, lay, kp>(nqmax, ket_kmax);             \
        nthreads = 64 * nw;                                                                         \
        return true;                                                                                \
    }
    MDX_MFMA_INSTANCES(MDX_CFG)
#undef MDX_CFG
    return false;
}

template <int LB, int LK, int NTAB, int NTCD, int NTG, int MTW, int NW, bool GB, int WPE, int LAY, int KP>
int QueueDig<true, LB, LK, NTAB, NTCD, NTG, MTW, NW, GB, WPE, LAY, KP>::ready(size_t lds)
{
    auto kern = eri_mfma_queue<LB, LK, NTAB, NTCD, NTG, MTW, NW, GB, WPE, LAY, KP, true>;
    return prepare(kern, lds) ? resident_blocks(kern, 64 * NW, lds) : 0;
}

int eri_queue_prepare(const EriKey &k, bool mfma, int variant, size_t lds, bool dig)
{
    int n = 0;
    if (mfma) {
#define MDX_QP(lb, lk, nab, ncd, gb, ntab, ntcd, ntg, mtw, nw, wpe, lay, kp)                            \
    if (mkey_is(k, lb, lk, nab, ncd, gb) && ++n == variant) {                                \
        if (dig)                                                                             \
            return QueueDig<first_of_class(MfmaRow{lb, lk, nab, ncd, gb, ntab, ntcd, ntg, mtw, nw, wpe, lay, kp}), \
                            lb, lk, ntab, ntcd, ntg, mtw, nw, gb, wpe, lay, kp>::ready(lds);                   \
        auto kern = eri_mfma_queue<lb, lk, ntab, ntcd, ntg, mtw, nw, gb, wpe, lay, kp>;               \
        return prepare(kern, lds) ? resident_blocks(kern, 64 * nw, lds) : 0;                 \
    }
        MDX_MFMA_INSTANCES(MDX_QP)
#undef MDX_QP
    } else {
#define MDX_QV(lb, lk, nab, ncd, gb, gk)                                                             \
    if (k.LB == lb && k.LK == lk && k.NAB == nab && k.NCD == ncd && k.GB == gb && k.GK == gk) {     \
        if (dig) return resident_blocks(eri_valu_queue<lb, lk, nab, ncd, gb, gk, true>, 64, 0);    \
        auto kern = eri_valu_queue<lb, lk, nab, ncd, gb, gk>;                                      \
        return resident_blocks(kern, 64, 0);                                                       \
    }
        MDX_VALU_INSTANCES(MDX_QV)
#undef MDX_QV
    }
    return 0;
}

bool eri_queue_launch(const EriKey &k, bool mfma, int variant, const QueueArgs &q, int nblocks, size_t lds,
                      hipStream_t s, bool dig)
{
    int n = 0;
    if (mfma) {
#define MDX_QL(lb, lk, nab, ncd, gb, ntab, ntcd, ntg, mtw, nw, wpe, lay, kp)                                        \
    if (mkey_is(k, lb, lk, nab, ncd, gb) && ++n == variant) {                                            \
        if (dig)                                                                                         \
            return QueueDig<first_of_class(MfmaRow{lb, lk, nab, ncd, gb, ntab, ntcd, ntg, mtw, nw, wpe, lay, kp}), \
                            lb, lk, ntab, ntcd, ntg, mtw, nw, gb, wpe, lay, kp>::go(q, nblocks, lds, s);     \
        hipLaunchKernelGGL((eri_mfma_queue<lb, lk, ntab, ntcd, ntg, mtw, nw, gb, wpe, lay, kp>), dim3(nblocks),    \
                           dim3(64 * nw), lds, s, q);                                                    \
        return true;                                                                                     \
    }
        MDX_MFMA_INSTANCES(MDX_QL)
#undef MDX_QL
    } else {
#define MDX_QW(lb, lk, nab, ncd, gb, gk)                                                                   \
    if (k.LB == lb && k.LK == lk && k.NAB == nab && k.NCD == ncd && k.GB == gb && k.GK == gk) {           \
        if (dig)                                                                                         \
            hipLaunchKernelGGL((eri_valu_queue<lb, lk, nab, ncd, gb, gk, true>), dim3(nblocks), dim3(64), 0, s, q); \
        else                                                                                             \
            hipLaunchKernelGGL((eri_valu_queue<lb, lk, nab, ncd, gb, gk>), dim3(nblocks), dim3(64), 0, s, q); \
        return true;                                                                                     \
    }
        MDX_VALU_INSTANCES(MDX_QW)
#undef MDX_QW
    }
    return false;
}

}  // namespace mdx
