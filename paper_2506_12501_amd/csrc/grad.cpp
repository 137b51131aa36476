// grad.cpp -- backward pass of a class batch (mdx_eri_grad_batch).
//
// Each launch takes one side as the derivative side (pair data in the
// derivative-bra role: Hermite expansions of d/dA and d/dB) and the other
// side in the ket role; the kernel contracts with the adjoint.  Passes:
//   4-centre: bra derivative side -> slots A, B; ket derivative side -> C, D.
//   3-centre: ket pair derivative side -> C, D; A = -(C + D) by translational
//             invariance (the integral depends only on relative positions).
//   2-centre: the lower-l function is the derivative side; the other centre
//             is minus it.
// A single function enters the backward kernel as a pair with a unit s
// partner (zeta = 0, c = 1) at its own centre, whose derivative vanishes.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstring>

#include "runtime.h"

namespace mdx {

// instance files: derivative-side orders 0..4 one file each, 5 and 6 split
// by the derivative side's function tiles (every key lives in one file)
#define MDX_GRAD_FILES(F) F(l0) F(l1) F(l2) F(l3) F(l4) F(l5a) F(l5b) F(l6a) F(l6b) F(l6c)
#define MDX_GRAD_DECL(suf)                                   \
    int eri_grad_variants_##suf(const GradKey &);            \
    bool eri_grad_launch_##suf(const GradKey &, const GradArgs &, int, int, hipStream_t);
MDX_GRAD_FILES(MDX_GRAD_DECL)

int eri_grad_variants(const GradKey &k)
{
    int n = 0;
#define MDX_GRAD_SUM(suf) n += eri_grad_variants_##suf(k);
    MDX_GRAD_FILES(MDX_GRAD_SUM)
#undef MDX_GRAD_SUM
    return n;
}

bool eri_grad_launch(const GradKey &k, const GradArgs &a, int nblocks, int variant, hipStream_t s)
{
#define MDX_GRAD_GO(suf) \
    if (eri_grad_variants_##suf(k) > 0) return eri_grad_launch_##suf(k, a, nblocks, variant, s);
    MDX_GRAD_FILES(MDX_GRAD_GO)
#undef MDX_GRAD_GO
    return false;
}

namespace {

constexpr int GRAD_LMAX_PAIR = 6;   // derivative side: total order of a pair (or l of a single function)
constexpr int GRAD_LMAX_OTHER = 6;  // other side: total order

struct GradPass {
    SidePlan d, w;   // derivative side (role 2), other side (ket role)
    GradKey key{};
    int variant = 1;
    const double *tw = nullptr;
    int64_t wsI = 0, wsJ = 0, wsd = 0, wsw = 0;
    int64_t gsI = 0, gsJ = 0, gss = 0;
    int wmask = 0;
    signed char M[12][6] = {};
};

struct GradPlan {
    int npass = 0;
    GradPass pass[2];
};

struct GradWs {
    size_t pairs_d, pairs_w, items_d, items_w, np_d, np_w, prim_d, prim_w, H_d, H_w, total;
};

size_t align256(size_t x) { return (x + 255) & ~size_t(255); }

GradWs grad_ws(const GradPass &p)
{
    GradWs L{};
    size_t o = 0;
    auto take = [&](size_t bytes) { size_t r = o; o = align256(o + bytes); return r; };
    const size_t nd = p.d.pairs.size(), nw = p.w.pairs.size();
    L.pairs_d = take(nd * sizeof(PairRec));
    L.pairs_w = take(nw * sizeof(PairRec));
    L.items_d = take(p.d.items.size() * sizeof(int2));
    L.items_w = take(p.w.items.size() * sizeof(int2));
    L.np_d = take(nd * sizeof(int32_t));
    L.np_w = take(nw * sizeof(int32_t));
    L.prim_d = take(nd * p.d.g.kmax * sizeof(PrimRec));
    L.prim_w = take(nw * p.w.g.kmax * sizeof(PrimRec));
    L.H_d = take(nd * (size_t)p.d.g.pair_stride * sizeof(double));
    L.H_w = take(nw * (size_t)p.w.g.pair_stride * sizeof(double));
    L.total = o;
    return L;
}

// One pass.  dside_is_bra: the caller's bra supplies the derivative side.
// Caller layout: W[ij + nbra*(ab + nab*(cd + ncd*kl))], G[ij + nbra*(slot + 12*kl)].
mdx_status make_pass(mdx_ctx *c, const mdx_shells *sh, int ncentre, int32_t nbra, const int32_t *bra,
                     int32_t nket, const int32_t *ket, bool cart, const int l[4], bool dside_is_bra, GradPass &p)
{
    const bool bra2 = ncentre == 4, ket2 = ncentre >= 3;
    const int nab = nfunc(l[0], cart) * (bra2 ? nfunc(l[1], cart) : 1);
    const int ncd = nfunc(l[2], cart) * (ket2 ? nfunc(l[3], cart) : 1);
    const int dl0 = dside_is_bra ? l[0] : l[2], dl1 = dside_is_bra ? l[1] : l[3];
    const int wl0 = dside_is_bra ? l[2] : l[0], wl1 = dside_is_bra ? l[3] : l[1];
    const bool dtwo = dside_is_bra ? bra2 : ket2, wtwo = dside_is_bra ? ket2 : bra2;
    p.d = make_side(sh, dside_is_bra ? bra : ket, dside_is_bra ? nbra : nket, dtwo, dl0, dl1, cart, 2, false);
    p.w = make_side(sh, dside_is_bra ? ket : bra, dside_is_bra ? nket : nbra, wtwo, wl0, wl1, cart, 1, false);
    if (p.d.g.L > GRAD_LMAX_PAIR || p.w.g.L > GRAD_LMAX_OTHER)
        return fail(MDX_EUNSUPPORTED,
                    "gradient: derivative side of total order %d (limit %d) / other side %d (limit %d)", p.d.g.L,
                    GRAD_LMAX_PAIR, p.w.g.L, GRAD_LMAX_OTHER);
    p.key.LD = p.d.g.L;
    p.key.LW = p.w.g.L;
    p.key.NTN = p.d.g.ncolp / 16;
    p.key.NTW = p.w.g.ncolp / 16;
    const int nv = eri_grad_variants(p.key);
    if (nv == 0)
        return fail(MDX_EUNSUPPORTED, "gradient: no kernel for orders (%d, %d) with %d and %d functions", p.key.LD,
                    p.key.LW, p.d.g.ncol, p.w.g.ncol);
    auto it = c->grad_variant.find(std::make_tuple(ncentre, l[0], bra2 ? l[1] : -1, l[2], ket2 ? l[3] : -1, cart ? 1 : 0));
    p.variant = (it != c->grad_variant.end() && it->second >= 1 && it->second <= nv) ? it->second : 1;
    p.tw = c->tket + (p.w.g.lb >= 0 ? c->tket_off[cart][p.w.g.la][p.w.g.lb] : c->tket1_off[cart][p.w.g.la]);
    const int64_t blk = (int64_t)nbra * nab * ncd;
    if (dside_is_bra) {
        p.wsI = 1; p.wsJ = blk; p.wsd = nbra; p.wsw = (int64_t)nbra * nab;
        p.gsI = 1; p.gsJ = 12 * (int64_t)nbra; p.gss = nbra;
    } else {
        p.wsI = blk; p.wsJ = 1; p.wsd = (int64_t)nbra * nab; p.wsw = nbra;
        p.gsI = 12 * (int64_t)nbra; p.gsJ = 1; p.gss = nbra;
    }
    return MDX_OK;
}

mdx_status plan_grad(mdx_ctx *c, const mdx_shells *sh, int ncentre, int32_t nbra, const int32_t *bra, int32_t nket,
                     const int32_t *ket, int flags, GradPlan &gp, bool &empty)
{
    int l[4];
    if (flags & MDX_FUSED) return fail(MDX_EINVAL, "mdx_eri_grad_batch: MDX_FUSED applies to plans only");
    if (flags & MDX_PAIRED) return fail(MDX_EINVAL, "mdx_eri_grad_batch: MDX_PAIRED applies to mdx_eri_batch only");
    mdx_status st = check_class(c, sh, ncentre, nbra, bra, nket, ket, flags, l);
    if (st != MDX_OK) return st;
    empty = nbra == 0 || nket == 0;
    if (empty) return MDX_OK;
    const bool cart = (flags & MDX_CARTESIAN) != 0;
    gp = GradPlan{};
    if (ncentre == 4) {
        gp.npass = 2;
        for (int ps = 0; ps < 2; ++ps) {
            GradPass &p = gp.pass[ps];
            if ((st = make_pass(c, sh, ncentre, nbra, bra, nket, ket, cart, l, ps == 0, p)) != MDX_OK) return st;
            for (int k = 0; k < 6; ++k) p.M[6 * ps + k][k] = 1;
            p.wmask = ps == 0 ? 0x03F : 0xFC0;
        }
    } else if (ncentre == 3) {
        gp.npass = 1;
        GradPass &p = gp.pass[0];
        if ((st = make_pass(c, sh, ncentre, nbra, bra, nket, ket, cart, l, false, p)) != MDX_OK) return st;
        for (int k = 0; k < 6; ++k) p.M[6 + k][k] = 1;          // C, D
        for (int i = 0; i < 3; ++i) p.M[i][i] = p.M[i][3 + i] = -1;   // A = -(C + D); B slots stay 0
        p.wmask = 0xFFF;
    } else {
        gp.npass = 1;
        GradPass &p = gp.pass[0];
        const bool dbra = l[0] <= l[2];
        if ((st = make_pass(c, sh, ncentre, nbra, bra, nket, ket, cart, l, dbra, p)) != MDX_OK) return st;
        const int own = dbra ? 0 : 6, other = dbra ? 6 : 0;
        for (int i = 0; i < 3; ++i) {
            p.M[own + i][i] = 1;
            p.M[other + i][i] = -1;
        }
        p.wmask = 0xFFF;
    }
    return MDX_OK;
}

}  // namespace

int grad_class_variants(int ncentre, int la, int lb, int lc, int ld, bool cart)
{
    const bool bra2 = ncentre == 4, ket2 = ncentre >= 3;
    const int Lb = la + (bra2 ? lb : 0), Lk = lc + (ket2 ? ld : 0);
    const int nab = nfunc(la, cart) * (bra2 ? nfunc(lb, cart) : 1);
    const int ncd = nfunc(lc, cart) * (ket2 ? nfunc(ld, cart) : 1);
    auto nv = [](int LD, int LW, int nd, int nw) {
        return eri_grad_variants(GradKey{LD, LW, round_up(nd, 16) / 16, round_up(nw, 16) / 16});
    };
    if (ncentre == 4) return std::max(nv(Lb, Lk, nab, ncd), nv(Lk, Lb, ncd, nab));
    if (ncentre == 3) return nv(Lk, Lb, ncd, nab);
    return Lb <= Lk ? nv(Lb, Lk, nab, ncd) : nv(Lk, Lb, ncd, nab);
}

}  // namespace mdx

using namespace mdx;

extern "C" size_t mdx_eri_grad_workspace_size(mdx_ctx *c, const mdx_shells *sh, int ncentre, int32_t nbra,
                                              const int32_t *bra, int32_t nket, const int32_t *ket, int flags)
{
    GradPlan gp;
    bool empty = false;
    if (plan_grad(c, sh, ncentre, nbra, bra, nket, ket, flags, gp, empty) != MDX_OK) return 0;
    size_t mx = 0;
    for (int i = 0; i < gp.npass; ++i) mx = std::max(mx, grad_ws(gp.pass[i]).total);
    return mx + 256;
}

extern "C" mdx_status mdx_eri_grad_batch(mdx_ctx *c, const mdx_shells *sh, int ncentre, int32_t nbra,
                                         const int32_t *bra, int32_t nket, const int32_t *ket, int flags,
                                         const double *adjoint, double *grad, void *ws, size_t ws_bytes,
                                         mdx_stream_t stream)
{
    GradPlan gp;
    bool empty = false;
    mdx_status st = plan_grad(c, sh, ncentre, nbra, bra, nket, ket, flags, gp, empty);
    if (st != MDX_OK) return st;
    if (empty) return MDX_OK;
    if (!adjoint || !grad) return fail(MDX_EINVAL, "mdx_eri_grad_batch: null adjoint or gradient");
    if (!ws) return fail(MDX_EINVAL, "mdx_eri_grad_batch: null workspace");
    if ((uintptr_t)ws & 255) return fail(MDX_EINVAL, "mdx_eri_grad_batch: workspace not 256-byte aligned");
    size_t need = 0;
    for (int i = 0; i < gp.npass; ++i) need = std::max(need, grad_ws(gp.pass[i]).total);
    if (ws_bytes < need) return fail(MDX_EWORKSPACE, "workspace %zu bytes < %zu required", ws_bytes, need);
    HIP_TRY2(hipSetDevice(c->device));
    hipStream_t s = (hipStream_t)stream;
    MDX_TRY(refuse_capture(s, "the call copies its index tables from host memory"));
    char *w = (char *)ws;
    for (int ip = 0; ip < gp.npass; ++ip) {
        const GradPass &p = gp.pass[ip];
        const GradWs L = grad_ws(p);
        const size_t nd = p.d.pairs.size(), nw = p.w.pairs.size();
        HIP_TRY2(hipMemcpyAsync(w + L.pairs_d, p.d.pairs.data(), nd * sizeof(PairRec), hipMemcpyHostToDevice, s));
        HIP_TRY2(hipMemcpyAsync(w + L.pairs_w, p.w.pairs.data(), nw * sizeof(PairRec), hipMemcpyHostToDevice, s));
        HIP_TRY2(hipMemcpyAsync(w + L.items_d, p.d.items.data(), p.d.items.size() * sizeof(int2),
                                hipMemcpyHostToDevice, s));
        HIP_TRY2(hipMemcpyAsync(w + L.items_w, p.w.items.data(), p.w.items.size() * sizeof(int2),
                                hipMemcpyHostToDevice, s));
        for (int side = 0; side < 2; ++side) {
            const SidePlan &sp = side == 0 ? p.d : p.w;
            PairDataArgs pa{};
            pa.g = sp.g;
            pa.pairs = (const PairRec *)(w + (side == 0 ? L.pairs_d : L.pairs_w));
            pa.items = (const int2 *)(w + (side == 0 ? L.items_d : L.items_w));
            pa.nitems = (int)sp.items.size();
            pa.center = sh->center;
            pa.expo = sh->exponent;
            pa.coef = sh->coef;
            pa.Ca = c->solid + c->solid_off[sp.g.la];
            pa.Cb = sp.g.lb >= 0 ? c->solid + c->solid_off[sp.g.lb] : nullptr;
            pa.prim = (PrimRec *)(w + (side == 0 ? L.prim_d : L.prim_w));
            pa.H = (double *)(w + (side == 0 ? L.H_d : L.H_w));
            pa.nprim = (int32_t *)(w + (side == 0 ? L.np_d : L.np_w));
            launch_pairdata(pa, s);
        }
        GradArgs a{};
        a.dside = SideDev{(const PrimRec *)(w + L.prim_d), (const double *)(w + L.H_d), (const int32_t *)(w + L.np_d),
                          p.d.g.kmax, p.d.g.pair_stride};
        a.wside = SideDev{(const PrimRec *)(w + L.prim_w), (const double *)(w + L.H_w), (const int32_t *)(w + L.np_w),
                          p.w.g.kmax, p.w.g.pair_stride};
        a.nI = (int)nd;
        a.nJ = (int)nw;
        a.boys = c->boys;
        a.Tw = p.tw;
        a.nd = p.d.g.ncol;
        a.nw = p.w.g.ncol;
        a.nwp = p.w.g.ncolp;
        a.W = adjoint;
        a.wsI = p.wsI; a.wsJ = p.wsJ; a.wsd = p.wsd; a.wsw = p.wsw;
        a.G = grad;
        a.gsI = p.gsI; a.gsJ = p.gsJ; a.gss = p.gss;
        a.wmask = p.wmask;
        std::memcpy(a.M, p.M, sizeof(a.M));
        const int64_t nblocks = (int64_t)nd * nw;
        if (nblocks > INT32_MAX) return fail(MDX_EUNSUPPORTED, "gradient: %lld shellsets in one launch", (long long)nblocks);
        hipEvent_t ev1 = nullptr;
        if (c->prof_events.size() >= 2) {
            const size_t np = c->prof_events.size() / 2, i = c->prof_count++ % np;
            ev1 = c->prof_events[2 * i + 1];
            HIP_TRY2(hipEventRecord(c->prof_events[2 * i], s));
        }
        const bool ok = eri_grad_launch(p.key, a, (int)nblocks, p.variant, s);
        if (ev1) HIP_TRY2(hipEventRecord(ev1, s));
        if (!ok) return fail(MDX_EUNSUPPORTED, "gradient kernel (%d, %d, %d) could not be launched (LDS)", p.key.LD,
                             p.key.LW, p.key.NTN);
        HIP_TRY2(hipGetLastError());
    }
    return MDX_OK;
}
