// nuclear_mfma.hip -- 1-particle Coulomb integrals of shells with l >= 4 on the
// matrix-core integral kernel.
//
// The field of a point charge q at C is the limit of an s Gaussian charge
// distribution of exponent zeta -> infinity, so Eqs. (24), (26), (30) are the
// 4-centre chain of Eq. (36) with a ket "pair" whose primitives are the
// charges: for ket exponent Z with Z >> p, rho = pZ/(p+Z) -> p and the [0]^(m)
// prefactor 2 pi^{5/2} / (p Z sqrt(p+Z)) times the normalisation (Z/pi)^{3/2}
// tends to 2 pi / p, Eq. (26).  With Z = 2^100 these limits hold exactly in
// double (p + Z = Z, p Z / Z = p, 1/sqrt(Z) = 2^-50), so each charge is a ket
// primitive record {p = 2^100, P = C, ws = 2^50, wt = -q/pi^{3/2}} (the bra
// pair data carry 2 pi^{5/2} K_AB c_a c_b / p).  An s ket has only its terminal
// Hermite, so the kernel's early contraction over ket primitives is exactly
// the sum over charges ahead of the Hermite-to-AO transform, Eq. (37):
//   Y[(kb, p)] = sum_I w_I [p]_I^(0),  then  V_ab = sum_p H_ab^p Y_p  (MFMA).
// Charges go through the kernel in slices of NUC_SLICE (their Boys arguments
// and [0]^(m) rows live in LDS); with several slices each writes a partial
// result and a final pass adds them.
#include "eri_mfma.h"
#include "runtime.h"

namespace mdx {

constexpr int NUC_SLICE = 64;

// Instances: bra Hermite order LB (= l_a + l_b), functions per pair NAB, then the
// tile shape (NTAB output tiles; MTW row tiles per wave; NW waves; WPE waves per
// SIMD), table layout LAY and charges per sweep round KP.  Spherical classes
// with max(l_a, l_b) >= 4 and l <= 6, and Cartesian ones up to 225 functions.
#define MDX_NUC_INSTANCES(X)                                                                  \
    X(4, 9, 1, 2, 4, 2, CUBE_LAY_COMPACT, 8)                                                  \
    X(5, 27, 2, 4, 4, 2, CUBE_LAY_COMPACT, 8) X(5, 11, 1, 4, 4, 2, CUBE_LAY_COMPACT, 8)       \
    X(6, 45, 3, 4, 4, 2, CUBE_LAY_COMPACT, 8) X(6, 33, 3, 4, 4, 2, CUBE_LAY_COMPACT, 8)       \
    X(6, 13, 1, 4, 4, 2, CUBE_LAY_COMPACT, 8)                                                 \
    X(7, 63, 4, 4, 4, 2, CUBE_LAY_COMPACT, 4) X(7, 55, 4, 4, 4, 2, CUBE_LAY_COMPACT, 4)       \
    X(7, 39, 3, 4, 4, 2, CUBE_LAY_COMPACT, 4)                                                 \
    X(8, 81, 6, 6, 4, 2, CUBE_LAY_COMPACT, 4) X(8, 77, 5, 6, 4, 2, CUBE_LAY_COMPACT, 4)       \
    X(8, 65, 5, 6, 4, 2, CUBE_LAY_COMPACT, 4)                                                 \
    X(9, 99, 7, 8, 4, 1, CUBE_LAY_COMPACT, 4) X(9, 91, 6, 8, 4, 1, CUBE_LAY_COMPACT, 4)       \
    X(10, 121, 8, 8, 4, 1, CUBE_LAY_COMPACT, 4) X(10, 117, 8, 8, 4, 1, CUBE_LAY_COMPACT, 4)   \
    X(11, 143, 9, 8, 4, 1, CUBE_LAY_COMPACT, 4)                                               \
    X(12, 169, 11, 8, 4, 1, CUBE_LAY_COMPACT, 2)                                              \
    /* Cartesian */                                                                           \
    X(4, 15, 1, 2, 4, 2, CUBE_LAY_COMPACT, 8)                                                 \
    X(5, 45, 3, 4, 4, 2, CUBE_LAY_COMPACT, 8) X(5, 21, 2, 4, 4, 2, CUBE_LAY_COMPACT, 8)       \
    X(6, 90, 6, 4, 4, 2, CUBE_LAY_COMPACT, 8) X(6, 63, 4, 4, 4, 2, CUBE_LAY_COMPACT, 8)       \
    X(6, 28, 2, 4, 4, 2, CUBE_LAY_COMPACT, 8)                                                 \
    X(7, 150, 10, 4, 4, 1, CUBE_LAY_COMPACT, 4) X(7, 126, 8, 4, 4, 1, CUBE_LAY_COMPACT, 4)    \
    X(7, 84, 6, 4, 4, 2, CUBE_LAY_COMPACT, 4)                                                 \
    X(8, 225, 15, 6, 4, 1, CUBE_LAY_COMPACT, 4) X(8, 210, 14, 6, 4, 1, CUBE_LAY_COMPACT, 4)   \
    X(8, 168, 11, 6, 4, 1, CUBE_LAY_COMPACT, 4)

template <int LB, int NTAB, int MTW, int NW, int WPE, int LAY, int KP>
__global__ void __launch_bounds__(64 * NW) __attribute__((amdgpu_waves_per_eu(WPE)))
nuclear_mfma_kernel(EriArgs a)
{
    int I, J, nI;
    if (!mfma_block_shellset(a, I, J, nI)) return;   // whole workgroup
    eri_mfma_shellset<LB, 0, NTAB, 1, 1, MTW, NW, false, LAY, KP>(a, I, J, nI);
}

template <int LB, int NTAB, int MTW, int NW, int WPE, int LAY, int KP>
static bool launch_nuc(EriArgs a, int nblocks, hipStream_t s)
{
    constexpr int NHB = nherm(LB);
    a.nqmax = std::min(a.bra.kmax, (NW * MTW * 16) / NHB + 2);
    const size_t lds = mfma_lds_bytes<LB, 0, NTAB, 1, 1, MTW, NW, false, LAY, KP>(a.nqmax, a.ket.kmax);
    if (lds > 160 * 1024) return false;
    auto kern = nuclear_mfma_kernel<LB, NTAB, MTW, NW, WPE, LAY, KP>;
    static size_t lds_set = 0;   // largest dynamic LDS granted to this instance so far
    if (lds > 64 * 1024 && lds > lds_set) {
        if (hipFuncSetAttribute((const void *)kern, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds) != hipSuccess)
            return false;
        lds_set = lds;
    }
    hipLaunchKernelGGL(kern, dim3(nblocks), dim3(64 * NW), lds, s, a);
    return true;
}

static bool nuc_has(int lb, int nab)
{
#define MDX_NH(LB, NAB, ntab, mtw, nw, wpe, lay, kp) \
    if (lb == LB && nab == NAB) return true;
    MDX_NUC_INSTANCES(MDX_NH)
#undef MDX_NH
    return false;
}

static bool nuc_launch(int lb, int nab, const EriArgs &a, int nblocks, hipStream_t s)
{
#define MDX_NL(LB, NAB, ntab, mtw, nw, wpe, lay, kp) \
    if (lb == LB && nab == NAB) return launch_nuc<LB, ntab, mtw, nw, wpe, lay, kp>(a, nblocks, s);
    MDX_NUC_INSTANCES(MDX_NL)
#undef MDX_NL
    return false;
}

// charge records of the ket "pair" (see the file comment) and the charge count
// of every slice
__global__ void __launch_bounds__(256) nuclear_charge_ket(const double *charges, int ncharge, PrimRec *prim, double *H,
                                                         int32_t *np)
{
    const int i = blockIdx.x * 256 + (int)threadIdx.x;
    if (i < ncharge) {
        const double w = -charges[4 * i + 3] * 0.17958712212516656;   // -q / pi^{3/2}
        PrimRec r{};
        r.p = 0x1p100;
        r.Px = charges[4 * i];
        r.Py = charges[4 * i + 1];
        r.Pz = charges[4 * i + 2];
        r.ws = 0x1p50;
        r.wt = w;
        prim[i] = r;
        H[16 * (int64_t)i] = w;
        for (int c = 1; c < 16; ++c) H[16 * (int64_t)i + c] = 0.0;
    }
    if (i * NUC_SLICE < ncharge) np[i] = min(NUC_SLICE, ncharge - i * NUC_SLICE);
}

// out[i] = sum_s part[s * n + i]
__global__ void __launch_bounds__(256) nuclear_sum_slices(const double *part, int nslice, int64_t n, double *out)
{
    const int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (i >= n) return;
    double v = 0.0;
    for (int s = 0; s < nslice; ++s) v += part[(int64_t)s * n + i];
    out[i] = v;
}

__global__ void __launch_bounds__(256) nuclear_zero(int64_t n, double *out)
{
    const int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (i < n) out[i] = 0.0;
}

static size_t al256n(size_t x) { return (x + 255) & ~size_t(255); }

// plan of the batch as the ERI class (ab|ss) with one ket pair of charge primitives
mdx_status nuc_plan(mdx_ctx *c, const mdx_shells *sh, int32_t npair, const int32_t *pairs, int la, int lb,
                    int32_t ncharge, bool cart, NucPlan &np)
{
    ClassPlan &cp = np.cp;
    cp = ClassPlan{};
    cp.ncentre = 4;
    cp.cart = cart;
    cp.la = la; cp.lb = lb; cp.lc = 0; cp.ld = 0;
    cp.bra = make_side(sh, pairs, npair, true, la, lb, cart, 0, true);
    np.nslice = (ncharge + NUC_SLICE - 1) / NUC_SLICE;
    cp.ket.g = make_geom(0, 0, cart, 1, 1, std::max(ncharge, 1), false);
    cp.ket.pairs.assign(1, PairRec{-1, -1, std::max(ncharge, 1), 1, 0, 0});
    cp.key = EriKey{cp.bra.g.L, 0, cp.bra.g.ncol, 1, false, false};
    if (cp.bra.g.ncol > MAXF || !nuc_has(cp.key.LB, cp.key.NAB))
        return fail(MDX_EUNSUPPORTED, "1-particle Coulomb integrals of class (%d|%d) %s: no kernel compiled", la, lb,
                    cart ? "Cartesian" : "spherical");
    cp.kind = K_MFMA;
    cp.variant = 1;
    cp.bra_per_tile = 1;
    cp.tket = c->tket + c->tket_off[cart][0][0];
    // one ket pair: a ragged batch of one bra prefix, out[ij + npair*ab]
    cp.count.assign(1, npair);
    cp.obase.assign(1, 0);
    cp.tile_off = {0, npair};
    cp.om = OutMap{};
    cp.om.sI = 1;
    for (int i = 0; i < cp.bra.g.ncol; ++i) cp.om.oab[i] = i;
    cp.om.ocd[0] = 0;
    cp.out_doubles = (int64_t)npair * cp.bra.g.ncol;
    np.L = ws_layout(cp);
    np.off_np = np.L.work;
    np.off_part = al256n(np.off_np + (size_t)std::max(np.nslice, 1) * 4);
    np.work = np.off_part + (np.nslice > 1 ? al256n((size_t)np.nslice * cp.out_doubles * 8) : 0);
    return MDX_OK;
}

// l >= 4 only: for (f|f) this path measured 10x slower than one pair per lane
// (K = 5, 100 charges: 222 vs 21 ms per 65,536 pairs) -- with no ket Hermites
// beyond the terminal one, the kernel's time is the per-charge [r]^(0) tables,
// built a few at a time in LDS
// the lane kernel (onebody.hip) takes every class with l_a + l_b <= 6
bool nuclear_on_mfma(int la, int lb) { return la + lb > 6; }

mdx_status nuclear_mfma_workspace(mdx_ctx *c, const mdx_shells *sh, int32_t npair, const int32_t *pairs, int la,
                                  int lb, int32_t ncharge, bool cart, size_t &bytes)
{
    NucPlan np;
    MDX_TRY(nuc_plan(c, sh, npair, pairs, la, lb, ncharge, cart, np));
    bytes = np.L.tables + np.work;
    return MDX_OK;
}

mdx_status nuclear_mfma_run(mdx_ctx *c, const mdx_shells *sh, const NucPlan &np, const char *tabs, char *work,
                            int32_t ncharge, const double *charges, double *V, hipStream_t s)
{
    const ClassPlan &cp = np.cp;
    const int64_t nout = cp.out_doubles;
    hipEvent_t ev1 = nullptr;
    if (c->prof_events.size() >= 2) {   // profiling hook: one window around the integral launches
        const size_t ne = c->prof_events.size() / 2, i = c->prof_count++ % ne;
        ev1 = c->prof_events[2 * i + 1];
        HIP_TRY2(hipEventRecord(c->prof_events[2 * i], s));
    }
    if (ncharge == 0) {
        hipLaunchKernelGGL(nuclear_zero, dim3((unsigned)((nout + 255) / 256)), dim3(256), 0, s, nout, V);
    } else {
        const ClassDev d = class_dev(np.L, tabs, work);
        enqueue_pairdata(c, sh, cp, d, 0, s);
        int32_t *nps = (int32_t *)(work + np.off_np);
        const int nthr = std::max(ncharge, np.nslice);
        hipLaunchKernelGGL(nuclear_charge_ket, dim3((nthr + 255) / 256), dim3(256), 0, s, charges, ncharge,
                           d.prim_ket, d.H_ket, nps);
        for (int sl = 0; sl < np.nslice; ++sl) {
            double *out = np.nslice > 1 ? (double *)(work + np.off_part) + (int64_t)sl * nout : V;
            EriArgs a;
            int nblocks = 0;
            MDX_TRY(class_args(c, cp, d, out, a, nblocks));
            a.ket.prim = d.prim_ket + (int64_t)sl * NUC_SLICE;
            a.ket.H = d.H_ket + (int64_t)sl * NUC_SLICE * 16;
            a.ket.nprim = nps + sl;
            a.ket.kmax = std::min(ncharge, NUC_SLICE);
            if (!nuc_launch(cp.key.LB, cp.key.NAB, a, nblocks, s))
                return fail(MDX_EUNSUPPORTED, "1-particle Coulomb kernel of class (%d|%d): LDS need beyond the device limit",
                            cp.la, cp.lb);
        }
        if (np.nslice > 1)
            hipLaunchKernelGGL(nuclear_sum_slices, dim3((unsigned)((nout + 255) / 256)), dim3(256), 0, s,
                               (const double *)(work + np.off_part), np.nslice, nout, V);
    }
    HIP_TRY2(hipGetLastError());
    if (ev1) HIP_TRY2(hipEventRecord(ev1, s));
    return MDX_OK;
}

mdx_status nuclear_mfma_enqueue(mdx_ctx *c, const mdx_shells *sh, int32_t npair, const int32_t *pairs, int la, int lb,
                                int32_t ncharge, const double *charges, bool cart, double *V, void *ws,
                                size_t ws_bytes, hipStream_t s)
{
    NucPlan np;
    MDX_TRY(nuc_plan(c, sh, npair, pairs, la, lb, ncharge, cart, np));
    if (!V) return fail(MDX_EINVAL, "mdx_nuclear_batch: null output");
    if (!ws) return fail(MDX_EINVAL, "mdx_nuclear_batch: null workspace");
    if ((uintptr_t)ws & 255) return fail(MDX_EINVAL, "mdx_nuclear_batch: workspace not 256-byte aligned");
    const size_t need = np.L.tables + np.work;
    if (ws_bytes < need) return fail(MDX_EWORKSPACE, "workspace %zu bytes < %zu required", ws_bytes, need);
    HIP_TRY2(hipSetDevice(c->device));
    char *w = (char *)ws;
    if (ncharge > 0) MDX_TRY(upload_tables(np.cp, class_dev(np.L, w), s));
    return nuclear_mfma_run(c, sh, np, w, w + np.L.tables, ncharge, charges, V, s);
}

}  // namespace mdx
