// eri.cpp -- planning and launching one class of shellsets (mdx_eri_batch).
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstring>

#include "runtime.h"

namespace mdx {

static size_t align256(size_t x) { return (x + 255) & ~size_t(255); }

SideGeom make_geom(int la, int lb, bool cart, int role, int npair, int kmax, bool allow_grouped)
{
    SideGeom g{};
    g.la = la;
    g.lb = lb;
    g.L = la + std::max(lb, 0);
    g.cart = cart ? 1 : 0;
    g.grouped = (lb < 0 && !cart && allow_grouped && role != 2) ? 1 : 0;
    g.role = role;
    g.npair = npair;
    g.kmax = kmax;
    g.ncol = nfunc(la, cart) * (lb >= 0 ? nfunc(lb, cart) : 1);
    g.ncolp = round_up(g.ncol, 16);
    if (g.grouped) {
        g.nh = ncart(la);
        g.nterm = ncart(la);
        g.ntpad = 0;
        g.rows_per_block = role == 0 ? round_up(g.nterm, 16) : g.nterm;
        g.nblocks = 1;
    } else if (role == 2) {
        // derivative bra: six blocks of rows up to order L + 1
        g.nh = nherm(g.L + 1);
        g.nterm = 0;
        g.ntpad = 0;
        g.rows_per_block = round_up(kmax * g.nh, 16);
        g.nblocks = 6;
    } else if (role == 0) {
        g.nh = nherm(g.L);
        g.nterm = 0;
        g.ntpad = 0;
        g.rows_per_block = round_up(kmax * g.nh, 16);
        g.nblocks = 1;
    } else {
        g.nh = nherm(g.L);
        g.ntpad = round_up(nherm(g.L - 1), 4);
        g.nterm = ncart(g.L);
        g.rows_per_block = g.ntpad + g.nterm;
        g.nblocks = kmax;
    }
    g.pair_stride = (int64_t)g.nblocks * g.rows_per_block * g.ncolp;
    return g;
}

mdx_status check_class(mdx_ctx *c, const mdx_shells *sh, int ncentre, int32_t nbra, const int32_t *bra,
                       int32_t nket, const int32_t *ket, int flags, int l[4])
{
    l[0] = l[1] = l[2] = l[3] = -1;
    if (!c) return fail(MDX_EINVAL, "null context");
    if (!sh) return fail(MDX_EINVAL, "null shell table");
    if (ncentre < 2 || ncentre > 4) return fail(MDX_EINVAL, "ncentre = %d (must be 2, 3 or 4)", ncentre);
    if (nbra < 0 || nket < 0) return fail(MDX_EINVAL, "negative pair count");
    if ((nbra > 0 && !bra) || (nket > 0 && !ket)) return fail(MDX_EINVAL, "null pair list");
    if (flags & ~(MDX_CARTESIAN | MDX_FUSED | MDX_PAIRED)) return fail(MDX_EINVAL, "unknown flags 0x%x", flags);
    if (sh->nshell < 0 || (sh->nshell > 0 && (!sh->l || !sh->nprim || !sh->prim_offset || !sh->center ||
                                               !sh->exponent || !sh->coef)))
        return fail(MDX_EINVAL, "incomplete shell table");
    if (nbra == 0 || nket == 0) return MDX_OK;
    const bool bra2 = ncentre == 4, ket2 = ncentre >= 3;
    auto check_shell = [&](int32_t s) -> bool { return s >= 0 && s < sh->nshell && sh->nprim[s] >= 1; };
    // class of the first entries, then every entry must match
    for (int side = 0; side < 2; ++side) {
        const int32_t n = side == 0 ? nbra : nket;
        const int32_t *lst = side == 0 ? bra : ket;
        const bool two = side == 0 ? bra2 : ket2;
        if (!check_shell(lst[0]) || (two && !check_shell(lst[1])))
            return fail(MDX_EINVAL, "%s pair 0: bad shell index or nprim < 1", side ? "ket" : "bra");
        const int l0 = sh->l[lst[0]], l1 = two ? sh->l[lst[1]] : -1;
        for (int32_t i = 0; i < n; ++i) {
            const int32_t s0 = lst[2 * i], s1 = lst[2 * i + 1];
            if (!check_shell(s0) || (two && !check_shell(s1)))
                return fail(MDX_EINVAL, "%s pair %d: bad shell index or nprim < 1", side ? "ket" : "bra", i);
            if (sh->l[s0] != l0 || (two && sh->l[s1] != l1))
                return fail(MDX_EINVAL, "%s pair %d: mixed classes in one batch", side ? "ket" : "bra", i);
        }
        l[2 * side] = l0;
        l[2 * side + 1] = l1;
    }
    const int lmax_pair = MDX_LMAX_4C, lmax_single = MDX_LMAX_3C;
    auto lok = [&](int lv, bool single) { return lv >= 0 && lv <= (single ? lmax_single : lmax_pair); };
    if (l[0] < 0 || l[2] < 0) return fail(MDX_EINVAL, "negative angular momentum");
    if (!lok(l[0], !bra2) || (bra2 && !lok(l[1], false)) || !lok(l[2], !ket2) || (ket2 && !lok(l[3], false)))
        return fail(MDX_EUNSUPPORTED, "angular momentum beyond the compiled limits (l <= %d per pair shell, %d single)",
                    lmax_pair, lmax_single);
    return MDX_OK;
}

SidePlan make_side(const mdx_shells *sh, const int32_t *lst, int32_t n, bool two, int l0, int l1, bool cart,
                   int role, bool allow_grouped)
{
    SidePlan sp;
    sp.pairs.resize(n);
    int kmax = 1;
    for (int32_t i = 0; i < n; ++i) {
        PairRec r{};
        r.sa = lst[2 * i];
        r.sb = two ? lst[2 * i + 1] : -1;
        r.ka = sh->nprim[r.sa];
        r.kb = two ? sh->nprim[r.sb] : 1;
        r.offa = sh->prim_offset[r.sa];
        r.offb = two ? sh->prim_offset[r.sb] : 0;
        sp.pairs[i] = r;
        kmax = std::max(kmax, r.ka * r.kb);
    }
    sp.g = make_geom(l0, two ? l1 : -1, cart, role, n, kmax, allow_grouped);
    if (!sp.g.grouped) {
        for (int32_t i = 0; i < n; ++i)
            for (int k = 0; k < sp.pairs[i].ka * sp.pairs[i].kb; ++k) sp.items.push_back(make_int2(i, k));
    }
    return sp;
}

mdx_status plan_class(mdx_ctx *c, const mdx_shells *sh, int ncentre, int32_t nbra, const int32_t *bra,
                      int32_t nket, const int32_t *ket, const int32_t *bra_count, int flags, ClassPlan &cp)
{
    // MDX_DIGEST (plans only): matrix-core classes take their general shape
    const bool digest = (flags & MDX_DIGEST) != 0;
    flags &= ~MDX_DIGEST;
    int lv[4];
    mdx_status st = check_class(c, sh, ncentre, nbra, bra, nket, ket, flags, lv);
    if (st != MDX_OK) return st;
    const bool cart = (flags & MDX_CARTESIAN) != 0;
    cp = ClassPlan{};
    cp.ncentre = ncentre;
    cp.cart = cart;
    if (nbra == 0 || nket == 0) return MDX_OK;
    const bool bra2 = ncentre == 4, ket2 = ncentre >= 3;
    cp.la = lv[0]; cp.lb = lv[1]; cp.lc = lv[2]; cp.ld = lv[3];
    if (ncentre == 2 && (cp.lc > MDX_LMAX_3C)) return fail(MDX_EUNSUPPORTED, "2-centre l beyond limit");

    const int Lb = cp.la + std::max(cp.lb, 0), Lk = cp.lc + std::max(cp.ld, 0);
    cp.swapped = (ncentre == 4 && Lb < Lk && !bra_count);
    // kernel sides
    for (int side = 0; side < 2; ++side) {
        const bool from_bra = (side == 0) != cp.swapped;
        const int l0 = from_bra ? cp.la : cp.lc, l1 = from_bra ? cp.lb : cp.ld;
        (side == 0 ? cp.bra : cp.ket) = make_side(sh, from_bra ? bra : ket, from_bra ? nbra : nket,
                                                  from_bra ? bra2 : ket2, l0, l1, cart, side, true);
    }
    cp.key.LB = cp.bra.g.L;
    cp.key.LK = cp.ket.g.L;
    cp.key.NAB = cp.bra.g.ncol;
    cp.key.NCD = cp.ket.g.ncol;
    cp.key.GB = cp.bra.g.grouped != 0;
    cp.key.GK = cp.ket.g.grouped != 0;

    // kernel choice: tuned override, else the register kernel when it exists
    auto it = c->variant.find(std::make_tuple(ncentre, cp.la, cp.lb, cp.lc, cp.ld, cart ? 1 : 0));
    const int var = it != c->variant.end() ? it->second : -1;
    const bool has_valu = eri_valu_has(cp.key), has_mfma = eri_mfma_has(cp.key);
    if (var == 0 && has_valu) cp.kind = K_VALU;
    else if (var >= 1 && var <= eri_mfma_variants(cp.key)) { cp.kind = K_MFMA; cp.variant = var; }
    else if (has_valu) cp.kind = K_VALU;
    else if (has_mfma) cp.kind = K_MFMA;
    else
        return fail(MDX_EUNSUPPORTED, "no kernel compiled for class (%d %d|%d %d) ncentre %d %s", cp.la, cp.lb, cp.lc,
                    cp.ld, ncentre, cart ? "Cartesian" : "spherical");
    if (cp.kind == K_MFMA && cp.variant == 0) {
        // untuned: the general kernel, or for batches of single primitive pairs
        // the first kernel written for them
        cp.variant = 1;
        const int n = eri_mfma_variants(cp.key);
        for (int v = 2; v <= n; ++v) {
            const int kind = eri_mfma_variant_kind(cp.key, v);
            if ((kind == MFMA_PRIM && cp.bra.g.kmax == 1 && cp.ket.g.kmax == 1) ||
                (kind == MFMA_MULTI && cp.ket.g.kmax == 1)) {
                cp.variant = v;
                break;
            }
        }
    }
    if (digest && cp.kind == K_MFMA) {
        // digestion is compiled for the first (general) shape of each class
        if (eri_mfma_variant_kind(cp.key, 1) != MFMA_GENERAL)
            return fail(MDX_EUNSUPPORTED, "digestion of class (%d %d|%d %d): no general matrix-core kernel", cp.la,
                        cp.lb, cp.lc, cp.ld);
        cp.variant = 1;
    }
    if (cp.kind == K_MFMA) {
        const int kind = eri_mfma_variant_kind(cp.key, cp.variant);
        if (kind == MFMA_PRIM && (cp.bra.g.kmax != 1 || cp.ket.g.kmax != 1)) {
            // contracted pairs on a single-primitive kernel: one launch per
            // primitive combination (kb, kk), each adding to the output (Eq. (5):
            // the contracted integral is the sum of its primitive integrals, whose
            // weights sit in the pair data).  Every pair of a side must have the
            // same contraction degree, so that primitive kb exists in all of them.
            auto uniform = [](const SidePlan &sp) {
                for (const PairRec &r : sp.pairs)
                    if (r.ka * r.kb != sp.g.kmax) return false;
                return true;
            };
            if (bra_count || (flags & MDX_PAIRED) || !uniform(cp.bra) || !uniform(cp.ket))
                return fail(MDX_EUNSUPPORTED,
                            "variant %d of class (%d %d|%d %d) takes contracted pairs only in dense batches with one "
                            "contraction degree per side", cp.variant, cp.la, cp.lb, cp.lc, cp.ld);
            cp.expand = true;
        }
        if (kind == MFMA_MULTI && cp.ket.g.kmax != 1)
            return fail(MDX_EUNSUPPORTED, "variant %d of class (%d %d|%d %d) serves single-primitive ket pairs only",
                        cp.variant, cp.la, cp.lb, cp.lc, cp.ld);
        cp.bra_per_tile = eri_mfma_bra_per_tile(cp.key, cp.variant);
    }

    // terminal ket matrix
    const int kl0 = cp.ket.g.la, kl1 = cp.ket.g.lb;
    cp.tket = c->tket + (kl1 >= 0 ? c->tket_off[cart][kl0][kl1] : c->tket1_off[cart][kl0]);

    // output map (caller layout [ij, ab, cd, kl])
    const int nab_c = nfunc(cp.la, cart) * (bra2 ? nfunc(cp.lb, cart) : 1);
    const int ncd_c = nfunc(cp.lc, cart) * (ket2 ? nfunc(cp.ld, cart) : 1);
    OutMap &om = cp.om;
    const int nabk = cp.bra.g.ncol, ncdk = cp.ket.g.ncol;
    if (nabk > MAXF || ncdk > MAXF) return fail(MDX_EUNSUPPORTED, "too many functions per pair");
    if (!bra_count) {
        if (!cp.swapped) {
            om.sI = 1;
            om.sJ = (int64_t)nbra * nab_c * ncd_c;
            om.mult = nbra;
            for (int i = 0; i < nabk; ++i) om.oab[i] = i;
            for (int j = 0; j < ncdk; ++j) om.ocd[j] = j * nab_c;
        } else {
            om.sJ = 1;
            om.sI = (int64_t)nbra * nab_c * ncd_c;
            om.mult = nbra;
            for (int i = 0; i < nabk; ++i) om.oab[i] = i * nab_c;
            for (int j = 0; j < ncdk; ++j) om.ocd[j] = j;
        }
        cp.out_doubles = (int64_t)nbra * nket * nab_c * ncd_c;
    } else {
        cp.count.resize(nket);
        cp.obase.resize(nket);
        cp.tile_off.resize(nket + 1);
        const int rows = cp.kind == K_VALU ? 64 : cp.bra_per_tile;   // bra pairs per tile
        int64_t off = 0, ntile = 0;
        for (int32_t k = 0; k < nket; ++k) {
            const int32_t n = bra_count[k];
            if (n < 0 || n > nbra) return fail(MDX_EINVAL, "bra_count[%d] = %d outside [0, %d]", k, n, nbra);
            cp.count[k] = n;
            cp.obase[k] = off;
            off += (int64_t)n * nab_c * ncd_c;
            cp.tile_off[k] = (int32_t)ntile;
            ntile += (n + rows - 1) / rows;
            if (ntile > INT32_MAX) return fail(MDX_EUNSUPPORTED, "more than 2^31 tiles in one batch");
        }
        cp.tile_off[nket] = (int32_t)ntile;
        om.sI = 1;
        om.sJ = 0;
        om.mult = 0;
        for (int i = 0; i < nabk; ++i) om.oab[i] = i;
        for (int j = 0; j < ncdk; ++j) om.ocd[j] = j * nab_c;
        cp.out_doubles = off;
    }
    if (flags & MDX_PAIRED) {   // quartet q = (bra q, ket q): the shellsets I = J of the outer product
        if (bra_count) return fail(MDX_EINVAL, "MDX_PAIRED with bra prefixes");
        if (nbra != nket) return fail(MDX_EINVAL, "MDX_PAIRED needs nbra == nket (%d, %d)", nbra, nket);
        cp.diag = cp.paired = true;
        if (cp.kind == K_MFMA) {   // the first shape: one shellset per workgroup
            cp.variant = 1;
            cp.bra_per_tile = eri_mfma_bra_per_tile(cp.key, 1);
            if (cp.bra_per_tile != 1)
                return fail(MDX_EUNSUPPORTED, "MDX_PAIRED for class (%d %d|%d %d)", cp.la, cp.lb, cp.lc, cp.ld);
        }
        // out[q + n*(ab + nab*cd)] in the caller's orientation; I = J = q
        om.sI = 0;
        om.sJ = 1;
        om.mult = nbra;
        cp.out_doubles = (int64_t)nbra * nab_c * ncd_c;
    }
    return MDX_OK;
}

WsLayout ws_layout(const ClassPlan &cp)
{
    WsLayout L{};
    size_t o = 0;
    auto take = [&](size_t bytes) { size_t r = o; o = align256(o + bytes); return r; };
    const size_t nb = cp.bra.pairs.size(), nk = cp.ket.pairs.size();
    // index tables (built on the host)
    L.pairs_bra = take(nb * sizeof(PairRec));
    L.pairs_ket = take(nk * sizeof(PairRec));
    L.items_bra = take(cp.bra.items.size() * sizeof(int2));
    L.items_ket = take(cp.ket.items.size() * sizeof(int2));
    L.count = take(cp.count.size() * sizeof(int32_t));
    L.obase = take(cp.obase.size() * sizeof(int64_t));
    L.tile_off = take(cp.tile_off.size() * sizeof(int32_t));
    L.tables = o;
    // pair data (written by the pair-data kernels), offsets from the work region
    o = 0;
    L.np_bra = take(nb * sizeof(int32_t));
    L.np_ket = take(nk * sizeof(int32_t));
    L.prim_bra = take(nb * cp.bra.g.kmax * sizeof(PrimRec));
    L.prim_ket = take(nk * cp.ket.g.kmax * sizeof(PrimRec));
    L.H_bra = take(nb * (size_t)cp.bra.g.pair_stride * sizeof(double));
    L.H_ket = take(nk * (size_t)cp.ket.g.pair_stride * sizeof(double));
    L.work = o;
    L.total = L.tables + L.work;
    return L;
}

ClassDev class_dev(const WsLayout &L, const char *tabs, char *work)
{
    ClassDev d{};
    d.pairs_bra = (const PairRec *)(tabs + L.pairs_bra);
    d.pairs_ket = (const PairRec *)(tabs + L.pairs_ket);
    d.items_bra = (const int2 *)(tabs + L.items_bra);
    d.items_ket = (const int2 *)(tabs + L.items_ket);
    d.count = (const int32_t *)(tabs + L.count);
    d.obase = (const int64_t *)(tabs + L.obase);
    d.tile_off = (const int32_t *)(tabs + L.tile_off);
    d.prim_bra = (PrimRec *)(work + L.prim_bra);
    d.prim_ket = (PrimRec *)(work + L.prim_ket);
    d.np_bra = (int32_t *)(work + L.np_bra);
    d.np_ket = (int32_t *)(work + L.np_ket);
    d.H_bra = (double *)(work + L.H_bra);
    d.H_ket = (double *)(work + L.H_ket);
    return d;
}

ClassDev class_dev(const WsLayout &L, char *ws) { return class_dev(L, ws, ws + L.tables); }

mdx_status upload_tables(const ClassPlan &cp, const ClassDev &d, hipStream_t s)
{
    MDX_TRY(refuse_capture(s, "the call copies its index tables from host memory"));
    const size_t nb = cp.bra.pairs.size(), nk = cp.ket.pairs.size();
    HIP_TRY2(hipMemcpyAsync((void *)d.pairs_bra, cp.bra.pairs.data(), nb * sizeof(PairRec), hipMemcpyHostToDevice, s));
    HIP_TRY2(hipMemcpyAsync((void *)d.pairs_ket, cp.ket.pairs.data(), nk * sizeof(PairRec), hipMemcpyHostToDevice, s));
    if (!cp.bra.items.empty())
        HIP_TRY2(hipMemcpyAsync((void *)d.items_bra, cp.bra.items.data(), cp.bra.items.size() * sizeof(int2),
                                hipMemcpyHostToDevice, s));
    if (!cp.ket.items.empty())
        HIP_TRY2(hipMemcpyAsync((void *)d.items_ket, cp.ket.items.data(), cp.ket.items.size() * sizeof(int2),
                                hipMemcpyHostToDevice, s));
    if (!cp.count.empty()) {
        HIP_TRY2(hipMemcpyAsync((void *)d.count, cp.count.data(), cp.count.size() * 4, hipMemcpyHostToDevice, s));
        HIP_TRY2(hipMemcpyAsync((void *)d.obase, cp.obase.data(), cp.obase.size() * 8, hipMemcpyHostToDevice, s));
    }
    if (!cp.tile_off.empty())
        HIP_TRY2(hipMemcpyAsync((void *)d.tile_off, cp.tile_off.data(), cp.tile_off.size() * sizeof(int32_t),
                                hipMemcpyHostToDevice, s));
    return MDX_OK;
}

mdx_status copy_tables(const ClassPlan &cp, const WsLayout &L, char *dst)
{
    auto put = [&](size_t off, const void *src, size_t bytes) -> hipError_t {
        return bytes ? hipMemcpy(dst + off, src, bytes, hipMemcpyHostToDevice) : hipSuccess;
    };
    HIP_TRY2(put(L.pairs_bra, cp.bra.pairs.data(), cp.bra.pairs.size() * sizeof(PairRec)));
    HIP_TRY2(put(L.pairs_ket, cp.ket.pairs.data(), cp.ket.pairs.size() * sizeof(PairRec)));
    HIP_TRY2(put(L.items_bra, cp.bra.items.data(), cp.bra.items.size() * sizeof(int2)));
    HIP_TRY2(put(L.items_ket, cp.ket.items.data(), cp.ket.items.size() * sizeof(int2)));
    HIP_TRY2(put(L.count, cp.count.data(), cp.count.size() * sizeof(int32_t)));
    HIP_TRY2(put(L.obase, cp.obase.data(), cp.obase.size() * sizeof(int64_t)));
    HIP_TRY2(put(L.tile_off, cp.tile_off.data(), cp.tile_off.size() * sizeof(int32_t)));
    return MDX_OK;
}

mdx_status refuse_capture(hipStream_t s, const char *why)
{
    hipStreamCaptureStatus cs = hipStreamCaptureStatusNone;
    HIP_TRY2(hipStreamIsCapturing(s, &cs));
    if (cs != hipStreamCaptureStatusNone)
        return fail(MDX_EINVAL, "stream is being captured and %s; capture the prepared form "
                    "(mdx_eri_prepare/mdx_eri_run, mdx_one_body_prepare/run, mdx_nuclear_prepare/run) instead", why);
    return MDX_OK;
}

void enqueue_pairdata(mdx_ctx *c, const mdx_shells *sh, const ClassPlan &cp, const ClassDev &d, int side,
                      hipStream_t s)
{
    const SidePlan &sp = side == 0 ? cp.bra : cp.ket;
    PairDataArgs pa{};
    pa.g = sp.g;
    pa.pairs = side == 0 ? d.pairs_bra : d.pairs_ket;
    pa.items = side == 0 ? d.items_bra : d.items_ket;
    pa.nitems = (int)sp.items.size();
    pa.center = sh->center;
    pa.expo = sh->exponent;
    pa.coef = sh->coef;
    pa.Ca = c->solid + c->solid_off[sp.g.la];
    pa.Cb = sp.g.lb >= 0 ? c->solid + c->solid_off[sp.g.lb] : nullptr;
    pa.prim = side == 0 ? d.prim_bra : d.prim_ket;
    pa.H = side == 0 ? d.H_bra : d.H_ket;
    pa.nprim = side == 0 ? d.np_bra : d.np_ket;
    launch_pairdata(pa, s);
}

mdx_status class_args(mdx_ctx *c, const ClassPlan &cp, const ClassDev &d, double *out, EriArgs &a, int &nblocks)
{
    const size_t nb = cp.bra.pairs.size(), nk = cp.ket.pairs.size();
    a = EriArgs{};
    a.bra = SideDev{d.prim_bra, d.H_bra, d.np_bra, cp.bra.g.kmax, cp.bra.g.pair_stride};
    a.ket = SideDev{d.prim_ket, d.H_ket, d.np_ket, cp.ket.g.kmax, cp.ket.g.pair_stride};
    a.nbra = (int)nb;
    a.nket = (int)nk;
    a.boys = c->boys;
    a.Tket = cp.tket;
    a.nab = cp.bra.g.ncol;
    a.ncd = cp.ket.g.ncol;
    a.om = cp.om;
    a.om.out = out;
    if (cp.diag) {
        // register kernel on a paired batch: one quartet per lane (diag = 2);
        // otherwise one shellset per workgroup
        a.diag = (cp.paired && cp.kind == K_VALU) ? 2 : 1;
        nblocks = a.diag == 2 ? (int)((nk + 63) / 64) : (int)nk;
    } else if (cp.count.empty()) {
        int64_t nbl;
        if (cp.kind == K_VALU) {   // 64 bra pairs (one per lane) per ket pair
            a.tiles_per_J = (int)((nb + 63) / 64);
            nbl = (int64_t)a.tiles_per_J * (int64_t)nk;
        } else {                   // blocks of MFMA_BRA_RUN bra tiles x MFMA_KET_RUN ket pairs
            const size_t units = (nb + cp.bra_per_tile - 1) / cp.bra_per_tile;
            a.tiles_per_J = (int)((units + MFMA_BRA_RUN - 1) / MFMA_BRA_RUN);
            nbl = (int64_t)a.tiles_per_J * (int64_t)((nk + MFMA_KET_RUN - 1) / MFMA_KET_RUN) * 128;
        }
        if (nbl > INT32_MAX) return fail(MDX_EUNSUPPORTED, "%lld workgroups in one launch (split the batch)", (long long)nbl);
        nblocks = (int)nbl;
    } else {
        a.om.count = d.count;
        a.om.obase = d.obase;
        a.tile_off = d.tile_off;
        nblocks = cp.tile_off.back();
    }
    a.ntile_total = nblocks;
    return MDX_OK;
}

mdx_status launch_class(mdx_ctx *c, const ClassPlan &cp, const EriArgs &a, int nblocks, hipStream_t s)
{
    if (nblocks == 0) return MDX_OK;
    hipEvent_t ev1 = nullptr;
    if (c->prof_events.size() >= 2) {
        const size_t np = c->prof_events.size() / 2, i = c->prof_count++ % np;
        ev1 = c->prof_events[2 * i + 1];
        HIP_TRY2(hipEventRecord(c->prof_events[2 * i], s));
    }
    const bool ok = cp.kind == K_VALU ? eri_valu_launch(cp.key, a, nblocks, s)
                                      : eri_mfma_launch(cp.key, a, nblocks, cp.variant, s);
    if (ev1) HIP_TRY2(hipEventRecord(ev1, s));
    if (!ok) return fail(MDX_EUNSUPPORTED, "kernel instance missing or its LDS need exceeds the device limit");
    HIP_TRY2(hipGetLastError());
    return MDX_OK;
}

mdx_status enqueue_class(mdx_ctx *c, const mdx_shells *sh, const ClassPlan &cp, const WsLayout &L, char *ws,
                         double *out, hipStream_t s, bool upload, const Digest *dig)
{
    if (cp.bra.pairs.empty() || cp.ket.pairs.empty()) return MDX_OK;
    const ClassDev d = class_dev(L, ws);
    if (upload) MDX_TRY(upload_tables(cp, d, s));
    return enqueue_class_dev(c, sh, cp, d, out, s, dig);
}

mdx_status enqueue_class_dev(mdx_ctx *c, const mdx_shells *sh, const ClassPlan &cp, const ClassDev &d, double *out,
                             hipStream_t s, const Digest *dig)
{
    if (cp.bra.pairs.empty() || cp.ket.pairs.empty()) return MDX_OK;
    mdx_status st;
    enqueue_pairdata(c, sh, cp, d, 0, s);
    enqueue_pairdata(c, sh, cp, d, 1, s);
    EriArgs a;
    int nblocks = 0;
    if ((st = class_args(c, cp, d, out, a, nblocks)) != MDX_OK) return st;
    if (dig) a.dig = *dig;
    if (!cp.expand) return launch_class(c, cp, a, nblocks, s);
    if (dig) return fail(MDX_EUNSUPPORTED, "digestion of contracted pairs on a single-primitive kernel");
    // primitive combination (kb, kk): the pair data of primitive kb of every bra
    // pair (rows kb*nh.. of the bra H, record kb) and of primitive kk of every
    // ket pair (block kk of the ket H, record kk)
    const SideGeom &gb = cp.bra.g, &gk = cp.ket.g;
    for (int kb = 0; kb < gb.kmax; ++kb)
        for (int kk = 0; kk < gk.kmax; ++kk) {
            EriArgs e = a;
            e.prim_expand = 1;
            e.accumulate = (kb | kk) != 0;
            e.bra.prim = a.bra.prim + kb;
            e.bra.H = a.bra.H + (int64_t)kb * gb.nh * gb.ncolp;
            e.ket.prim = a.ket.prim + kk;
            e.ket.H = a.ket.H + (int64_t)kk * gk.rows_per_block * gk.ncolp;
            if ((st = launch_class(c, cp, e, nblocks, s)) != MDX_OK) return st;
        }
    return MDX_OK;
}

}  // namespace mdx

using namespace mdx;

extern "C" size_t mdx_eri_workspace_size(mdx_ctx *c, const mdx_shells *sh, int ncentre, int32_t nbra,
                                         const int32_t *bra, int32_t nket, const int32_t *ket, int flags)
{
    if (flags & MDX_DIGEST) {
        fail(MDX_EINVAL, "mdx_eri_workspace_size: MDX_DIGEST applies to plans only");
        return 0;
    }
    ClassPlan cp;
    if (plan_class(c, sh, ncentre, nbra, bra, nket, ket, nullptr, flags, cp) != MDX_OK) return 0;
    return ws_layout(cp).total + 256;
}

extern "C" mdx_status mdx_eri_batch(mdx_ctx *c, const mdx_shells *sh, int ncentre, int32_t nbra, const int32_t *bra,
                                    int32_t nket, const int32_t *ket, int flags, double *out, void *ws,
                                    size_t ws_bytes, mdx_stream_t stream)
{
    if (flags & MDX_DIGEST) return fail(MDX_EINVAL, "mdx_eri_batch: MDX_DIGEST applies to plans only");
    if (flags & MDX_FUSED) return fail(MDX_EINVAL, "mdx_eri_batch: MDX_FUSED applies to plans only");
    ClassPlan cp;
    mdx_status st = plan_class(c, sh, ncentre, nbra, bra, nket, ket, nullptr, flags, cp);
    if (st != MDX_OK) return st;
    if (nbra == 0 || nket == 0) return MDX_OK;
    if (!out) return fail(MDX_EINVAL, "mdx_eri_batch: null output");
    if (!ws) return fail(MDX_EINVAL, "mdx_eri_batch: null workspace");
    if ((uintptr_t)ws & 255) return fail(MDX_EINVAL, "mdx_eri_batch: workspace not 256-byte aligned");
    const WsLayout L = ws_layout(cp);
    if (ws_bytes < L.total) return fail(MDX_EWORKSPACE, "workspace %zu bytes < %zu required", ws_bytes, L.total);
    HIP_TRY2(hipSetDevice(c->device));
    return enqueue_class(c, sh, cp, L, (char *)ws, out, (hipStream_t)stream, true);
}

extern "C" mdx_status mdx_eri_batch_noalloc(mdx_ctx *c, const mdx_shells *sh, int ncentre, int32_t nbra,
                                            const int32_t *bra, int32_t nket, const int32_t *ket, int flags,
                                            double *out, mdx_stream_t stream)
{
    if (flags & MDX_DIGEST) return fail(MDX_EINVAL, "mdx_eri_batch_noalloc: MDX_DIGEST applies to plans only");
    if (flags & MDX_FUSED) return fail(MDX_EINVAL, "mdx_eri_batch_noalloc: MDX_FUSED applies to plans only");
    ClassPlan cp;
    mdx_status st = plan_class(c, sh, ncentre, nbra, bra, nket, ket, nullptr, flags, cp);
    if (st != MDX_OK) return st;
    if (nbra == 0 || nket == 0) return MDX_OK;
    if (!out) return fail(MDX_EINVAL, "mdx_eri_batch_noalloc: null output");
    if (!c->scratch) return fail(MDX_EDEVICE, "mdx_eri_batch_noalloc: the context has no static scratch");
    const WsLayout L = ws_layout(cp);
    if (L.total > (size_t)MDX_NOALLOC_SCRATCH_BYTES)
        return fail(MDX_EWORKSPACE,
                    "mdx_eri_batch_noalloc: the batch needs %zu bytes of scratch, the static buffer holds %zu "
                    "(split the batch, or use mdx_eri_batch with a workspace)",
                    L.total, (size_t)MDX_NOALLOC_SCRATCH_BYTES);
    HIP_TRY2(hipSetDevice(c->device));
    // the same planning, tables and kernels as mdx_eri_batch; nothing in the
    // scratch needs to start at zero (the workspace contract of mdx_eri_batch)
    return enqueue_class(c, sh, cp, L, c->scratch, out, (hipStream_t)stream, true);
}

extern "C" mdx_status mdx_eri_prepare(mdx_ctx *c, const mdx_shells *sh, int ncentre, int32_t nbra, const int32_t *bra,
                                      int32_t nket, const int32_t *ket, int flags, mdx_batch **out)
{
    if (!out) return fail(MDX_EINVAL, "mdx_eri_prepare: null handle pointer");
    *out = nullptr;
    if (flags & MDX_DIGEST) return fail(MDX_EINVAL, "mdx_eri_prepare: MDX_DIGEST applies to plans only");
    if (flags & MDX_FUSED) return fail(MDX_EINVAL, "mdx_eri_prepare: MDX_FUSED applies to plans only");
    mdx_batch *b = new mdx_batch;
    mdx_status st = plan_class(c, sh, ncentre, nbra, bra, nket, ket, nullptr, flags, b->cp);
    if (st == MDX_OK) st = batch_init(b, c, sh, B_ERI, flags);
    if (st == MDX_OK && !b->cp.bra.pairs.empty() && !b->cp.ket.pairs.empty()) {
        b->L = ws_layout(b->cp);
        b->ws_need = b->L.work;
        b->out_doubles = b->cp.out_doubles;
        st = batch_tables(b, b->L.tables);
        if (st == MDX_OK) st = copy_tables(b->cp, b->L, b->dtab);
    }
    if (st != MDX_OK) {
        mdx_batch_destroy(b);
        return st;
    }
    *out = b;
    return MDX_OK;
}

extern "C" mdx_status mdx_eri_run(const mdx_batch *b, const mdx_shells *sh, double *out, void *ws, size_t ws_bytes,
                                  mdx_stream_t stream)
{
    MDX_TRY(batch_check(b, sh, B_ERI, ws, ws_bytes, "mdx_eri_run"));
    if (b->out_doubles == 0) return MDX_OK;
    if (!out) return fail(MDX_EINVAL, "mdx_eri_run: null output");
    return enqueue_class_dev(b->c, sh, b->cp, class_dev(b->L, b->dtab, (char *)ws), out, (hipStream_t)stream);
}

extern "C" mdx_status mdx_eri_digest_batch(mdx_ctx *c, const mdx_shells *sh, int ncentre, int32_t nbra,
                                           const int32_t *bra, int32_t nket, const int32_t *ket, int flags,
                                           const double *Dbra, const double *Dket, double *Jbra, double *Jket,
                                           void *ws, size_t ws_bytes, mdx_stream_t stream)
{
    if (flags & MDX_DIGEST) return fail(MDX_EINVAL, "mdx_eri_digest_batch: MDX_DIGEST applies to plans only");
    if (flags & MDX_FUSED) return fail(MDX_EINVAL, "mdx_eri_digest_batch: MDX_FUSED applies to plans only");
    if (flags & MDX_PAIRED) return fail(MDX_EINVAL, "mdx_eri_digest_batch: MDX_PAIRED applies to mdx_eri_batch only");
    ClassPlan cp;
    mdx_status st = plan_class(c, sh, ncentre, nbra, bra, nket, ket, nullptr, flags, cp);
    if (st != MDX_OK) return st;
    if (nbra == 0 || nket == 0 || (!Jbra && !Jket)) return MDX_OK;   // nothing is read or written
    if (Jbra && !Dket) return fail(MDX_EINVAL, "mdx_eri_digest_batch: Jbra needs Dket");
    if (Jket && !Dbra) return fail(MDX_EINVAL, "mdx_eri_digest_batch: Jket needs Dbra");
    if (!ws) return fail(MDX_EINVAL, "mdx_eri_digest_batch: null workspace");
    if ((uintptr_t)ws & 255) return fail(MDX_EINVAL, "mdx_eri_digest_batch: workspace not 256-byte aligned");
    // digestion is compiled for the first shape of the general matrix-core
    // kernel of each class (the single-primitive and 3-centre variants store
    // their tail rows in lane patterns of their own)
    if (cp.kind == K_MFMA) {
        cp.variant = 1;
        cp.bra_per_tile = eri_mfma_bra_per_tile(cp.key, 1);
    }
    const WsLayout L = ws_layout(cp);
    if (ws_bytes < L.total) return fail(MDX_EWORKSPACE, "workspace %zu bytes < %zu required", ws_bytes, L.total);
    Digest dg{};
    dg.on = 1;
    if (!cp.swapped) {
        dg.Db = Dbra; dg.Dk = Dket; dg.Jb = Jbra; dg.Jk = Jket;
        dg.nb = nbra; dg.nk = nket;
    } else {   // the kernel runs with the caller's ket pairs as its bra pairs
        dg.Db = Dket; dg.Dk = Dbra; dg.Jb = Jket; dg.Jk = Jbra;
        dg.nb = nket; dg.nk = nbra;
    }
    HIP_TRY2(hipSetDevice(c->device));
    return enqueue_class(c, sh, cp, L, (char *)ws, nullptr, (hipStream_t)stream, true, &dg);
}
