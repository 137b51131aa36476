// plan.cpp -- multi-class plans (plain launches or one fused graph), Schwarz
// factors, kernel-variant and profiling controls.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <numeric>
#include <cstring>
#include <map>
#include <string>

#include "runtime.h"

using namespace mdx;

namespace {

size_t al256(size_t x) { return (x + 255) & ~size_t(255); }

struct PlanBatch {
    ClassPlan cp;
    int64_t out_offset = 0;
    size_t t_pairs_bra = 0, t_pairs_ket = 0, t_items_bra = 0, t_items_ket = 0, t_count = 0, t_obase = 0,
           t_tile_off = 0;   // in the plan's tables
    size_t w_prim_bra = 0, w_prim_ket = 0, w_np_bra = 0, w_np_ket = 0, w_H_bra = 0, w_H_ket = 0;   // in ws
    int nqmax = 1;
    int rec[2] = {-1, -1};   // fused: side records of the bra and ket pair data
};

// Fused plans compute the pair data of a side once: a record is the longest
// pair list of one role and class, and every batch side whose list is a prefix
// of it reads the record's rows (the screened ket lists are prefixes of the
// sorted bucket lists).
struct SideRec {
    SidePlan sp;
    int role = 0;
    size_t t_pairs = 0, t_items = 0;
    size_t w_prim = 0, w_np = 0, w_H = 0;
};

// batches of a fused plan that share one kernel instance
struct QueueGroup {
    EriKey key{};
    bool mfma = false;
    int variant = 0;
    std::vector<int> batches;
    std::vector<int32_t> base;   // [nb+1]
    size_t t_desc = 0, t_base = 0;
    int counter = 0;             // index into the plan's counters
    size_t lds = 0;
    int nblocks = 0;
};

}  // namespace

struct mdx_plan {
    mdx_ctx *c = nullptr;
    int flags = 0;
    bool fused = false;
    std::vector<PlanBatch> b;
    std::vector<QueueGroup> q;
    std::vector<SideRec> recs;
    int64_t out_size = 0;
    size_t ws_total = 0;
    char *dtab = nullptr;        // device tables (plan-owned)
    size_t dtab_bytes = 0;
    size_t t_counters = 0;
    int ncounter = 0;
    size_t t_pd = 0, t_pdbase = 0;   // fused: the side records as one pair-data launch
    // basis metadata at creation
    int32_t nshell = 0;
    std::vector<int32_t> l, nprim, poff;
    // fused execution
    static constexpr int NS = 4;
    hipStream_t cs[NS] = {};
    hipEvent_t ev[2 * NS] = {};
    hipGraphExec_t exec = nullptr;
    const void *k_center = nullptr, *k_exp = nullptr, *k_coef = nullptr;
    double *k_out = nullptr;
    void *k_ws = nullptr;
    std::vector<mdx_digest_block> k_blk;   // digesting graph: the blocks its descriptors hold
    std::vector<EriArgs> descs;

    ~mdx_plan()
    {
        if (exec) hipGraphExecDestroy(exec);
        for (auto &e : ev)
            if (e) hipEventDestroy(e);
        for (auto &s : cs)
            if (s) hipStreamDestroy(s);
        if (dtab) hipFree(dtab);
    }
};

namespace {

ClassDev batch_dev(const mdx_plan *p, const PlanBatch &pb, char *ws)
{
    ClassDev d{};
    if (pb.rec[0] >= 0) {
        const SideRec &rb = p->recs[pb.rec[0]], &rk = p->recs[pb.rec[1]];
        d.pairs_bra = (const PairRec *)(p->dtab + rb.t_pairs);
        d.pairs_ket = (const PairRec *)(p->dtab + rk.t_pairs);
        d.items_bra = (const int2 *)(p->dtab + rb.t_items);
        d.items_ket = (const int2 *)(p->dtab + rk.t_items);
        d.count = (const int32_t *)(p->dtab + pb.t_count);
        d.obase = (const int64_t *)(p->dtab + pb.t_obase);
        d.tile_off = (const int32_t *)(p->dtab + pb.t_tile_off);
        d.prim_bra = (PrimRec *)(ws + rb.w_prim);
        d.prim_ket = (PrimRec *)(ws + rk.w_prim);
        d.np_bra = (int32_t *)(ws + rb.w_np);
        d.np_ket = (int32_t *)(ws + rk.w_np);
        d.H_bra = (double *)(ws + rb.w_H);
        d.H_ket = (double *)(ws + rk.w_H);
        return d;
    }
    d.pairs_bra = (const PairRec *)(p->dtab + pb.t_pairs_bra);
    d.pairs_ket = (const PairRec *)(p->dtab + pb.t_pairs_ket);
    d.items_bra = (const int2 *)(p->dtab + pb.t_items_bra);
    d.items_ket = (const int2 *)(p->dtab + pb.t_items_ket);
    d.count = (const int32_t *)(p->dtab + pb.t_count);
    d.obase = (const int64_t *)(p->dtab + pb.t_obase);
    d.tile_off = (const int32_t *)(p->dtab + pb.t_tile_off);
    d.prim_bra = (PrimRec *)(ws + pb.w_prim_bra);
    d.prim_ket = (PrimRec *)(ws + pb.w_prim_ket);
    d.np_bra = (int32_t *)(ws + pb.w_np_bra);
    d.np_ket = (int32_t *)(ws + pb.w_np_ket);
    d.H_bra = (double *)(ws + pb.w_H_bra);
    d.H_ket = (double *)(ws + pb.w_H_ket);
    return d;
}

mdx_status build_graph(mdx_plan *p, const mdx_shells *sh, double *out, char *ws, hipStream_t user,
                       const mdx_digest_block *blk = nullptr)
{
    const bool dig = blk != nullptr;
    mdx_ctx *c = p->c;
    if (p->exec) {
        HIP_TRY2(hipGraphExecDestroy(p->exec));
        p->exec = nullptr;
    }
    // kernel arguments of every batch, in device memory (the previous graph may
    // still be running on the caller's stream: let it finish first)
    HIP_TRY2(hipStreamSynchronize(user));
    p->descs.assign(p->b.size(), EriArgs{});
    for (size_t i = 0; i < p->b.size(); ++i) {
        PlanBatch &pb = p->b[i];
        int nbl = 0;
        mdx_status st = class_args(c, pb.cp, batch_dev(p, pb, ws), out ? out + pb.out_offset : nullptr, p->descs[i],
                                   nbl);
        if (st != MDX_OK) return st;
        p->descs[i].nqmax = pb.nqmax;
        if (dig) {
            Digest &d = p->descs[i].dig;
            d.on = 1;
            d.Db = blk[i].Dbra;
            d.Dk = blk[i].Dket;
            d.Jb = blk[i].Jbra;
            d.Jk = blk[i].Jket;
            d.nb = (int64_t)pb.cp.bra.pairs.size();
            d.nk = (int64_t)pb.cp.ket.pairs.size();
        }
    }
    for (const QueueGroup &g : p->q) {
        std::vector<EriArgs> d;
        for (int bi : g.batches) d.push_back(p->descs[bi]);
        HIP_TRY2(hipMemcpy(p->dtab + g.t_desc, d.data(), d.size() * sizeof(EriArgs), hipMemcpyHostToDevice));
    }
    // pair data of every side record, one launch
    std::vector<PairDataArgs> pds;
    std::vector<int32_t> pdbase(1, 0);
    size_t pd_lds = 0;
    for (const SideRec &r : p->recs) {
        PairDataArgs pa{};
        pa.g = r.sp.g;
        pa.pairs = (const PairRec *)(p->dtab + r.t_pairs);
        pa.items = (const int2 *)(p->dtab + r.t_items);
        pa.nitems = (int)r.sp.items.size();
        pa.center = sh->center;
        pa.expo = sh->exponent;
        pa.coef = sh->coef;
        pa.Ca = c->solid + c->solid_off[r.sp.g.la];
        pa.Cb = r.sp.g.lb >= 0 ? c->solid + c->solid_off[r.sp.g.lb] : nullptr;
        pa.prim = (PrimRec *)(ws + r.w_prim);
        pa.H = (double *)(ws + r.w_H);
        pa.nprim = (int32_t *)(ws + r.w_np);
        size_t lds = 0;
        const int nblk = std::max(pairdata_prepare(pa, lds), 0);
        if ((int64_t)pdbase.back() + nblk > INT32_MAX) return fail(MDX_EUNSUPPORTED, "pair data: too many workgroups");
        pdbase.push_back(pdbase.back() + nblk);
        if (nblk > 0) pd_lds = std::max(pd_lds, lds);
        pds.push_back(pa);
    }
    if (!pds.empty()) {
        HIP_TRY2(hipMemcpy(p->dtab + p->t_pd, pds.data(), pds.size() * sizeof(PairDataArgs), hipMemcpyHostToDevice));
        HIP_TRY2(hipMemcpy(p->dtab + p->t_pdbase, pdbase.data(), pdbase.size() * 4, hipMemcpyHostToDevice));
    }
    PairDataMulti pdm{};
    pdm.recs = (const PairDataArgs *)(p->dtab + p->t_pd);
    pdm.base = (const int32_t *)(p->dtab + p->t_pdbase);
    pdm.nrec = (int)pds.size();

    hipStream_t s0 = p->cs[0];
    HIP_TRY2(hipStreamBeginCapture(s0, hipStreamCaptureModeThreadLocal));
    mdx_status st = MDX_OK;
    auto capture = [&]() -> mdx_status {
        int *counters = (int *)(p->dtab + p->t_counters);
        launch_fill_i32(counters, p->ncounter, 0, s0);
        // pair data of all batches: one launch over every side record
        launch_pairdata_multi(pdm, pdbase.back(), pd_lds, s0);
        // fork: one persistent launch per kernel instance over the streams
        HIP_TRY2(hipEventRecord(p->ev[mdx_plan::NS], s0));
        for (int k = 1; k < mdx_plan::NS; ++k) HIP_TRY2(hipStreamWaitEvent(p->cs[k], p->ev[mdx_plan::NS], 0));
        // launch order: the matrix-core groups first, highest total angular
        // momentum first, then the register-kernel groups in plan order.  The
        // matrix-core classes have few, long work items (one shellset per
        // workgroup); launched last they run nearly alone at the end of the
        // graph.  The register-kernel groups have many short items and end
        // the graph with several of them draining together.
        std::vector<int> order(p->q.size());
        std::iota(order.begin(), order.end(), 0);
        std::stable_sort(order.begin(), order.end(), [&](int x, int y) {
            const QueueGroup &u = p->q[x], &v = p->q[y];
            if (u.mfma != v.mfma) return u.mfma;
            return u.mfma && u.key.LB + u.key.LK > v.key.LB + v.key.LK;
        });
        int rr = 0;
        for (const int gix : order) {
            const QueueGroup &g = p->q[gix];
            QueueArgs qa{};
            qa.desc = (const EriArgs *)(p->dtab + g.t_desc);
            qa.base = (const int32_t *)(p->dtab + g.t_base);
            qa.nb = (int)g.batches.size();
            qa.total = g.base.back();
            qa.counter = counters + g.counter;
            if (!eri_queue_launch(g.key, g.mfma, g.variant, qa, g.nblocks, g.lds, p->cs[rr++ % mdx_plan::NS], dig))
                return fail(MDX_EUNSUPPORTED, "persistent kernel instance missing");
        }
        for (int k = 1; k < mdx_plan::NS; ++k) {
            HIP_TRY2(hipEventRecord(p->ev[mdx_plan::NS + k], p->cs[k]));
            HIP_TRY2(hipStreamWaitEvent(s0, p->ev[mdx_plan::NS + k], 0));
        }
        return MDX_OK;
    };
    st = capture();
    hipGraph_t graph = nullptr;
    const hipError_t e = hipStreamEndCapture(s0, &graph);
    if (st != MDX_OK) {
        if (graph) hipGraphDestroy(graph);
        return st;
    }
    if (e != hipSuccess) return fail(MDX_EDEVICE, "hipStreamEndCapture: %s", hipGetErrorString(e));
    const hipError_t e2 = hipGraphInstantiate(&p->exec, graph, nullptr, nullptr, 0);
    hipGraphDestroy(graph);
    if (e2 != hipSuccess) {
        p->exec = nullptr;
        return fail(MDX_EDEVICE, "hipGraphInstantiate: %s", hipGetErrorString(e2));
    }
    p->k_center = sh->center;
    p->k_exp = sh->exponent;
    p->k_coef = sh->coef;
    p->k_out = out;
    p->k_ws = ws;
    return MDX_OK;
}

}  // namespace

extern "C" mdx_status mdx_plan_create(mdx_ctx *c, const mdx_shells *sh, int nbatch, const mdx_batch_desc *batches,
                                      int flags, mdx_plan **out)
{
    if (!out) return fail(MDX_EINVAL, "mdx_plan_create: null output handle");
    *out = nullptr;
    if (!c) return fail(MDX_EINVAL, "null context");
    if (!sh) return fail(MDX_EINVAL, "null shell table");
    if (nbatch < 0 || (nbatch > 0 && !batches)) return fail(MDX_EINVAL, "mdx_plan_create: bad batch list");
    if (flags & ~(MDX_CARTESIAN | MDX_FUSED | MDX_DIGEST)) return fail(MDX_EINVAL, "unknown flags 0x%x", flags);
    mdx_plan *p = new (std::nothrow) mdx_plan;
    if (!p) return fail(MDX_ENOMEM, "mdx_plan_create: out of host memory");
    p->c = c;
    p->flags = flags;
    p->fused = (flags & MDX_FUSED) != 0;
    p->b.resize(nbatch);
    size_t tab = 0, ws = 0;
    auto ttake = [&](size_t bytes) { size_t r = tab; tab = al256(tab + bytes); return r; };
    auto wtake = [&](size_t bytes) { size_t r = ws; ws = al256(ws + bytes); return r; };
    for (int i = 0; i < nbatch; ++i) {
        const mdx_batch_desc &bd = batches[i];
        if (bd.out_offset < 0) {
            delete p;
            return fail(MDX_EINVAL, "batch %d: negative out_offset", i);
        }
        std::vector<int32_t> full;
        const int32_t *cnt = bd.bra_count;
        if (!cnt) {
            full.assign(std::max(bd.nket, 0), bd.nbra);
            cnt = full.data();
        }
        PlanBatch &pb = p->b[i];
        mdx_status st = plan_class(c, sh, bd.ncentre, bd.nbra, bd.bra, bd.nket, bd.ket, cnt,
                                   flags & (MDX_CARTESIAN | MDX_DIGEST), pb.cp);
        if (st != MDX_OK) {
            const std::string msg = mdx_last_error();
            delete p;
            return fail(st, "batch %d: %s", i, msg.c_str());
        }
        pb.out_offset = bd.out_offset;
        p->out_size = std::max(p->out_size, bd.out_offset + pb.cp.out_doubles);
        const ClassPlan &cp = pb.cp;
        const size_t nb = cp.bra.pairs.size(), nk = cp.ket.pairs.size();
        pb.t_pairs_bra = ttake(nb * sizeof(PairRec));
        pb.t_pairs_ket = ttake(nk * sizeof(PairRec));
        pb.t_items_bra = ttake(cp.bra.items.size() * sizeof(int2));
        pb.t_items_ket = ttake(cp.ket.items.size() * sizeof(int2));
        pb.t_count = ttake(cp.count.size() * 4);
        pb.t_obase = ttake(cp.obase.size() * 8);
        pb.t_tile_off = ttake(cp.tile_off.size() * 4);
        pb.w_np_bra = wtake(nb * 4);
        pb.w_np_ket = wtake(nk * 4);
        pb.w_prim_bra = wtake(nb * cp.bra.g.kmax * sizeof(PrimRec));
        pb.w_prim_ket = wtake(nk * cp.ket.g.kmax * sizeof(PrimRec));
        pb.w_H_bra = wtake(nb * (size_t)cp.bra.g.pair_stride * 8);
        pb.w_H_ket = wtake(nk * (size_t)cp.ket.g.pair_stride * 8);
    }
    // fused: one pair-data record per distinct side (prefix sharing), then
    // group the batches by kernel instance
    if (p->fused) {
        struct Ref { int batch, side; size_t len; };
        std::vector<Ref> refs;
        for (int i = 0; i < nbatch; ++i) {
            const ClassPlan &cp = p->b[i].cp;
            if (cp.bra.pairs.empty() || cp.ket.pairs.empty()) continue;
            refs.push_back({i, 0, cp.bra.pairs.size()});
            refs.push_back({i, 1, cp.ket.pairs.size()});
        }
        std::stable_sort(refs.begin(), refs.end(), [](const Ref &x, const Ref &y) { return x.len > y.len; });
        std::multimap<std::tuple<int, int, int, int, int32_t, int32_t>, int> index;
        for (const Ref &r : refs) {
            ClassPlan &cp = p->b[r.batch].cp;
            SidePlan &sp = r.side == 0 ? cp.bra : cp.ket;
            const auto key = std::make_tuple(r.side, sp.g.la, sp.g.lb, sp.g.cart, sp.pairs[0].sa, sp.pairs[0].sb);
            int found = -1;
            for (auto it = index.lower_bound(key); it != index.end() && it->first == key; ++it) {
                const SideRec &rec = p->recs[it->second];
                if (rec.sp.g.grouped == sp.g.grouped && rec.sp.pairs.size() >= sp.pairs.size() &&
                    std::memcmp(rec.sp.pairs.data(), sp.pairs.data(), sp.pairs.size() * sizeof(PairRec)) == 0) {
                    found = it->second;
                    break;
                }
            }
            if (found < 0) {
                found = (int)p->recs.size();
                SideRec rec;
                rec.sp = sp;
                rec.role = r.side;
                p->recs.push_back(std::move(rec));
                index.emplace(key, found);
            }
            p->b[r.batch].rec[r.side] = found;
        }
        // batches address the record's rows: take its geometry (kmax, strides)
        for (PlanBatch &pb : p->b) {
            if (pb.rec[0] < 0) continue;
            const int na = (int)pb.cp.bra.pairs.size(), nk = (int)pb.cp.ket.pairs.size();
            pb.cp.bra.g = p->recs[pb.rec[0]].sp.g;
            pb.cp.ket.g = p->recs[pb.rec[1]].sp.g;
            pb.cp.bra.g.npair = na;
            pb.cp.ket.g.npair = nk;
        }
        ws = 0;
        for (SideRec &r : p->recs) {
            const size_t n = r.sp.pairs.size();
            r.t_pairs = ttake(n * sizeof(PairRec));
            r.t_items = ttake(r.sp.items.size() * sizeof(int2));
            r.w_np = wtake(n * 4);
            r.w_prim = wtake(n * r.sp.g.kmax * sizeof(PrimRec));
            r.w_H = wtake(n * (size_t)r.sp.g.pair_stride * 8);
        }
        std::map<std::tuple<int, int, int, int, int, int, int, int>, int> gi;
        for (int i = 0; i < nbatch; ++i) {
            PlanBatch &pb = p->b[i];
            const ClassPlan &cp = pb.cp;
            if (cp.bra.pairs.empty() || cp.ket.pairs.empty() || cp.tile_off.back() == 0) continue;
            const bool mfma = cp.kind == K_MFMA;
            size_t lds = 0;
            if (mfma) {
                int nt = 0;
                if (!eri_mfma_config(cp.key, cp.variant, cp.bra.g.kmax, cp.ket.g.kmax, pb.nqmax, lds, nt,
                                     (flags & MDX_DIGEST) != 0)) {
                    delete p;
                    return fail(MDX_EUNSUPPORTED,
                                "batch %d: variant %d of its class has no persistent form (fused plans take the "
                                "general matrix-core variants)", i, cp.variant);
                }
            }
            const auto k = std::make_tuple(cp.key.LB, cp.key.LK, cp.key.NAB, cp.key.NCD, (int)cp.key.GB,
                                           (int)cp.key.GK, (int)mfma, cp.variant);
            auto it = gi.find(k);
            if (it == gi.end()) {
                it = gi.emplace(k, (int)p->q.size()).first;
                QueueGroup g;
                g.key = cp.key;
                g.mfma = mfma;
                g.variant = cp.variant;
                g.base.push_back(0);
                p->q.push_back(g);
            }
            QueueGroup &g = p->q[it->second];
            g.batches.push_back(i);
            const int64_t tot = (int64_t)g.base.back() + cp.tile_off.back();
            if (tot > INT32_MAX) {
                delete p;
                return fail(MDX_EUNSUPPORTED, "more than 2^31 work items for one kernel instance");
            }
            g.base.push_back((int32_t)tot);
            g.lds = std::max(g.lds, lds);
        }
        for (size_t gix = 0; gix < p->q.size(); ++gix) {
            QueueGroup &g = p->q[gix];
            if (g.lds + 256 > 160 * 1024) {
                delete p;
                return fail(MDX_EUNSUPPORTED, "fused launch needs %zu bytes of LDS", g.lds);
            }
            const int per_cu = eri_queue_prepare(g.key, g.mfma, g.variant, g.lds, (flags & MDX_DIGEST) != 0);
            if (per_cu <= 0) {
                delete p;
                return fail(MDX_EUNSUPPORTED, "persistent kernel cannot be made resident");
            }
            g.nblocks = std::max(1, std::min(g.base.back(), per_cu * std::max(c->ncu, 1)));
            g.t_desc = ttake(g.batches.size() * sizeof(EriArgs));
            g.t_base = ttake(g.base.size() * 4);
            g.counter = (int)gix;
        }
        p->ncounter = (int)p->q.size();
        p->t_counters = ttake(std::max(p->ncounter, 1) * 4);
        p->t_pd = ttake(std::max(p->recs.size(), (size_t)1) * sizeof(PairDataArgs));
        p->t_pdbase = ttake((p->recs.size() + 1) * 4);
    }
    p->ws_total = ws;
    p->dtab_bytes = std::max(tab, (size_t)256);
    hipError_t e = hipSetDevice(c->device);
    if (e == hipSuccess) e = hipMalloc((void **)&p->dtab, p->dtab_bytes);
    if (e != hipSuccess) {
        p->dtab = nullptr;
        delete p;
        return fail(MDX_EDEVICE, "mdx_plan_create: %s", hipGetErrorString(e));
    }
    for (const PlanBatch &pb : p->b) {
        const ClassPlan &cp = pb.cp;
        auto up = [&](size_t off, const void *src, size_t bytes) {
            if (e == hipSuccess && bytes) e = hipMemcpy(p->dtab + off, src, bytes, hipMemcpyHostToDevice);
        };
        up(pb.t_pairs_bra, cp.bra.pairs.data(), cp.bra.pairs.size() * sizeof(PairRec));
        up(pb.t_pairs_ket, cp.ket.pairs.data(), cp.ket.pairs.size() * sizeof(PairRec));
        up(pb.t_items_bra, cp.bra.items.data(), cp.bra.items.size() * sizeof(int2));
        up(pb.t_items_ket, cp.ket.items.data(), cp.ket.items.size() * sizeof(int2));
        up(pb.t_count, cp.count.data(), cp.count.size() * 4);
        up(pb.t_obase, cp.obase.data(), cp.obase.size() * 8);
        up(pb.t_tile_off, cp.tile_off.data(), cp.tile_off.size() * 4);
    }
    for (const QueueGroup &g : p->q)
        if (e == hipSuccess) e = hipMemcpy(p->dtab + g.t_base, g.base.data(), g.base.size() * 4, hipMemcpyHostToDevice);
    for (const SideRec &r : p->recs) {
        if (e == hipSuccess && !r.sp.pairs.empty())
            e = hipMemcpy(p->dtab + r.t_pairs, r.sp.pairs.data(), r.sp.pairs.size() * sizeof(PairRec),
                          hipMemcpyHostToDevice);
        if (e == hipSuccess && !r.sp.items.empty())
            e = hipMemcpy(p->dtab + r.t_items, r.sp.items.data(), r.sp.items.size() * sizeof(int2),
                          hipMemcpyHostToDevice);
    }
    if (e == hipSuccess && p->fused) {
        for (auto &s : p->cs)
            if (e == hipSuccess) e = hipStreamCreateWithFlags(&s, hipStreamNonBlocking);
        for (auto &ev : p->ev)
            if (e == hipSuccess) e = hipEventCreateWithFlags(&ev, hipEventDisableTiming);
    }
    if (e != hipSuccess) {
        delete p;
        return fail(MDX_EDEVICE, "mdx_plan_create: %s", hipGetErrorString(e));
    }
    p->nshell = sh->nshell;
    p->l.assign(sh->l, sh->l + sh->nshell);
    p->nprim.assign(sh->nprim, sh->nprim + sh->nshell);
    p->poff.assign(sh->prim_offset, sh->prim_offset + sh->nshell);
    *out = p;
    return MDX_OK;
}

extern "C" size_t mdx_plan_workspace_size(const mdx_plan *p) { return p ? p->ws_total + 256 : 0; }
extern "C" int64_t mdx_plan_output_size(const mdx_plan *p) { return p ? p->out_size : 0; }

extern "C" mdx_status mdx_plan_execute(mdx_plan *p, const mdx_shells *sh, double *out, void *ws, size_t ws_bytes,
                                       mdx_stream_t stream)
{
    if (!p) return fail(MDX_EINVAL, "null plan");
    if (p->flags & MDX_DIGEST) return fail(MDX_EINVAL, "mdx_plan_execute: a MDX_DIGEST plan runs through mdx_plan_digest");
    if (!sh || sh->nshell != p->nshell ||
        (p->nshell > 0 && (!sh->l || !sh->nprim || !sh->prim_offset || !sh->center || !sh->exponent || !sh->coef)))
        return fail(MDX_EINVAL, "mdx_plan_execute: shell table does not match the plan");
    if (p->nshell > 0 && (std::memcmp(sh->l, p->l.data(), p->nshell * 4) ||
                          std::memcmp(sh->nprim, p->nprim.data(), p->nshell * 4) ||
                          std::memcmp(sh->prim_offset, p->poff.data(), p->nshell * 4)))
        return fail(MDX_EINVAL, "mdx_plan_execute: shell metadata differ from the plan's");
    if (p->out_size == 0) return MDX_OK;
    if (!out) return fail(MDX_EINVAL, "mdx_plan_execute: null output");
    if (!ws) return fail(MDX_EINVAL, "mdx_plan_execute: null workspace");
    if ((uintptr_t)ws & 255) return fail(MDX_EINVAL, "mdx_plan_execute: workspace not 256-byte aligned");
    if (ws_bytes < p->ws_total) return fail(MDX_EWORKSPACE, "workspace %zu bytes < %zu required", ws_bytes, p->ws_total);
    mdx_ctx *c = p->c;
    HIP_TRY2(hipSetDevice(c->device));
    hipStream_t s = (hipStream_t)stream;
    char *w = (char *)ws;
    if (!p->fused) {
        for (const PlanBatch &pb : p->b) {
            const ClassPlan &cp = pb.cp;
            if (cp.bra.pairs.empty() || cp.ket.pairs.empty() || cp.tile_off.back() == 0) continue;
            const ClassDev d = batch_dev(p, pb, w);
            enqueue_pairdata(c, sh, cp, d, 0, s);
            enqueue_pairdata(c, sh, cp, d, 1, s);
            EriArgs a;
            int nbl = 0;
            mdx_status st = class_args(c, cp, d, out + pb.out_offset, a, nbl);
            if (st == MDX_OK) st = launch_class(c, cp, a, nbl, s);
            if (st != MDX_OK) return st;
        }
        return MDX_OK;
    }
    if (!p->exec || p->k_center != sh->center || p->k_exp != sh->exponent || p->k_coef != sh->coef ||
        p->k_out != out || p->k_ws != ws) {
        mdx_status st = build_graph(p, sh, out, w, s);
        if (st != MDX_OK) return st;
    }
    HIP_TRY2(hipGraphLaunch(p->exec, s));
    return MDX_OK;
}

extern "C" mdx_status mdx_plan_digest(mdx_plan *p, const mdx_shells *sh, const mdx_digest_block *blk, void *ws,
                                      size_t ws_bytes, mdx_stream_t stream)
{
    if (!p) return fail(MDX_EINVAL, "null plan");
    if (!(p->flags & MDX_DIGEST)) return fail(MDX_EINVAL, "mdx_plan_digest: the plan was created without MDX_DIGEST");
    if (!sh || sh->nshell != p->nshell ||
        (p->nshell > 0 && (!sh->l || !sh->nprim || !sh->prim_offset || !sh->center || !sh->exponent || !sh->coef)))
        return fail(MDX_EINVAL, "mdx_plan_digest: shell table does not match the plan");
    if (p->nshell > 0 && (std::memcmp(sh->l, p->l.data(), p->nshell * 4) ||
                          std::memcmp(sh->nprim, p->nprim.data(), p->nshell * 4) ||
                          std::memcmp(sh->prim_offset, p->poff.data(), p->nshell * 4)))
        return fail(MDX_EINVAL, "mdx_plan_digest: shell metadata differ from the plan's");
    if (p->b.empty()) return MDX_OK;
    if (!blk) return fail(MDX_EINVAL, "mdx_plan_digest: null block array");
    for (size_t i = 0; i < p->b.size(); ++i) {
        if (blk[i].Jbra && !blk[i].Dket) return fail(MDX_EINVAL, "mdx_plan_digest: batch %zu: Jbra needs Dket", i);
        if (blk[i].Jket && !blk[i].Dbra) return fail(MDX_EINVAL, "mdx_plan_digest: batch %zu: Jket needs Dbra", i);
    }
    if (!ws) return fail(MDX_EINVAL, "mdx_plan_digest: null workspace");
    if ((uintptr_t)ws & 255) return fail(MDX_EINVAL, "mdx_plan_digest: workspace not 256-byte aligned");
    if (ws_bytes < p->ws_total) return fail(MDX_EWORKSPACE, "workspace %zu bytes < %zu required", ws_bytes, p->ws_total);
    mdx_ctx *c = p->c;
    HIP_TRY2(hipSetDevice(c->device));
    hipStream_t s = (hipStream_t)stream;
    char *w = (char *)ws;
    if (p->fused) {   // the digesting graph; its batch descriptors hold the blocks' pointers
        const bool same = p->k_blk.size() == p->b.size() &&
                          std::memcmp(p->k_blk.data(), blk, p->b.size() * sizeof(mdx_digest_block)) == 0;
        if (!p->exec || !same || p->k_center != sh->center || p->k_exp != sh->exponent || p->k_coef != sh->coef ||
            p->k_ws != ws) {
            mdx_status st = build_graph(p, sh, nullptr, w, s, blk);
            if (st != MDX_OK) return st;
            p->k_blk.assign(blk, blk + p->b.size());
        }
        HIP_TRY2(hipGraphLaunch(p->exec, s));
        return MDX_OK;
    }
    for (size_t i = 0; i < p->b.size(); ++i) {
        const PlanBatch &pb = p->b[i];
        const ClassPlan &cp = pb.cp;
        if (cp.bra.pairs.empty() || cp.ket.pairs.empty() || cp.tile_off.back() == 0) continue;
        if (!blk[i].Jbra && !blk[i].Jket) continue;
        const ClassDev d = batch_dev(p, pb, w);
        enqueue_pairdata(c, sh, cp, d, 0, s);
        enqueue_pairdata(c, sh, cp, d, 1, s);
        EriArgs a;
        int nbl = 0;
        mdx_status st = class_args(c, cp, d, nullptr, a, nbl);
        if (st != MDX_OK) return st;
        a.dig.on = 1;
        a.dig.Db = blk[i].Dbra;
        a.dig.Dk = blk[i].Dket;
        a.dig.Jb = blk[i].Jbra;
        a.dig.Jk = blk[i].Jket;
        a.dig.nb = (int64_t)cp.bra.pairs.size();
        a.dig.nk = (int64_t)cp.ket.pairs.size();
        if ((st = launch_class(c, cp, a, nbl, s)) != MDX_OK) return st;
    }
    return MDX_OK;
}

extern "C" void mdx_plan_destroy(mdx_plan *p) { delete p; }

// ---------------------------------------------------------------------------
// Schwarz factors
// ---------------------------------------------------------------------------
namespace {

mdx_status plan_schwarz(mdx_ctx *c, const mdx_shells *sh, int32_t npair, const int32_t *pairs, int flags,
                        ClassPlan &cp)
{
    if (flags & ~MDX_CARTESIAN) return fail(MDX_EINVAL, "mdx_schwarz: unknown flags 0x%x", flags);
    mdx_status st = plan_class(c, sh, 4, npair, pairs, npair, pairs, nullptr, flags, cp);
    if (st != MDX_OK) return st;
    cp.diag = true;
    // diagonal block of pair J at out[J*nab*nab + ab + nab*cd]
    const int nab = cp.bra.g.ncol;
    cp.om.sI = 0;
    cp.om.sJ = (int64_t)nab * nab;
    cp.om.mult = 1;
    for (int i = 0; i < nab; ++i) {
        cp.om.oab[i] = i;
        cp.om.ocd[i] = i * nab;
    }
    return MDX_OK;
}

}  // namespace

extern "C" size_t mdx_schwarz_workspace_size(mdx_ctx *c, const mdx_shells *sh, int32_t npair, const int32_t *pairs,
                                             int flags)
{
    ClassPlan cp;
    if (plan_schwarz(c, sh, npair, pairs, flags, cp) != MDX_OK) return 0;
    const size_t nab = cp.bra.g.ncol;
    return al256(ws_layout(cp).total) + al256((size_t)npair * nab * nab * 8) + 256;
}

extern "C" mdx_status mdx_schwarz(mdx_ctx *c, const mdx_shells *sh, int32_t npair, const int32_t *pairs, int flags,
                                  double *Q, void *ws, size_t ws_bytes, mdx_stream_t stream)
{
    ClassPlan cp;
    mdx_status st = plan_schwarz(c, sh, npair, pairs, flags, cp);
    if (st != MDX_OK) return st;
    if (npair == 0) return MDX_OK;
    if (!Q) return fail(MDX_EINVAL, "mdx_schwarz: null Q");
    if (!ws) return fail(MDX_EINVAL, "mdx_schwarz: null workspace");
    if ((uintptr_t)ws & 255) return fail(MDX_EINVAL, "mdx_schwarz: workspace not 256-byte aligned");
    const WsLayout L = ws_layout(cp);
    const size_t nab = cp.bra.g.ncol;
    const size_t need = al256(L.total) + al256((size_t)npair * nab * nab * 8);
    if (ws_bytes < need) return fail(MDX_EWORKSPACE, "workspace %zu bytes < %zu required", ws_bytes, need);
    HIP_TRY2(hipSetDevice(c->device));
    hipStream_t s = (hipStream_t)stream;
    double *diag = (double *)((char *)ws + al256(L.total));
    if ((st = enqueue_class(c, sh, cp, L, (char *)ws, diag, s, true)) != MDX_OK) return st;
    launch_schwarz(diag, npair, (int)nab, Q, s);
    HIP_TRY2(hipGetLastError());
    return MDX_OK;
}

// ---------------------------------------------------------------------------
// controls
// ---------------------------------------------------------------------------
extern "C" mdx_status mdx_set_variant(mdx_ctx *c, int ncentre, int la, int lb, int lc, int ld, int flags, int variant)
{
    if (!c) return fail(MDX_EINVAL, "null context");
    if (ncentre < 2 || ncentre > 4 || la < 0 || lc < 0 || (ncentre == 4 && lb < 0) || (ncentre >= 3 && ld < 0) ||
        la > 8 || lb > 8 || lc > 8 || ld > 8)
        return fail(MDX_EINVAL, "mdx_set_variant: bad class");
    if (flags & ~(MDX_CARTESIAN | MDX_GRADIENT)) return fail(MDX_EINVAL, "mdx_set_variant: unknown flags 0x%x", flags);
    const bool cart = (flags & MDX_CARTESIAN) != 0;
    const auto key_t = std::make_tuple(ncentre, la, ncentre == 4 ? lb : -1, lc, ncentre >= 3 ? ld : -1, cart ? 1 : 0);
    if (flags & MDX_GRADIENT) {
        if (variant < 0) {
            c->grad_variant.erase(key_t);
            return MDX_OK;
        }
        if (variant < 1 || variant > grad_class_variants(ncentre, la, lb, lc, ld, cart))
            return fail(MDX_EINVAL, "mdx_set_variant: class has no backward variant %d", variant);
        c->grad_variant[key_t] = variant;
        return MDX_OK;
    }
    if (variant < 0) {
        c->variant.erase(key_t);
        return MDX_OK;
    }
    // class key in kernel orientation, as plan_class derives it
    const bool bra2 = ncentre == 4, ket2 = ncentre >= 3;
    int Lb = la + (bra2 ? lb : 0), Lk = lc + (ket2 ? ld : 0);
    int nab = nfunc(la, cart) * (bra2 ? nfunc(lb, cart) : 1);
    int ncd = nfunc(lc, cart) * (ket2 ? nfunc(ld, cart) : 1);
    bool gb = !bra2 && !cart, gk = !ket2 && !cart;
    if (ncentre == 4 && Lb < Lk) {
        std::swap(Lb, Lk);
        std::swap(nab, ncd);
    }
    const EriKey k{Lb, Lk, nab, ncd, gb, gk};
    const bool ok = variant == 0 ? eri_valu_has(k) : variant <= eri_mfma_variants(k);
    if (!ok) return fail(MDX_EINVAL, "mdx_set_variant: class has no variant %d", variant);
    c->variant[key_t] = variant;
    return MDX_OK;
}

extern "C" mdx_status mdx_set_profile_events(mdx_ctx *c, void *const *events, int nevents)
{
    if (!c) return fail(MDX_EINVAL, "null context");
    if (nevents < 0 || (nevents & 1)) return fail(MDX_EINVAL, "nevents = %d must be even and >= 0", nevents);
    c->prof_events.clear();
    c->prof_count = 0;
    if (events)
        for (int i = 0; i < nevents; ++i) c->prof_events.push_back((hipEvent_t)events[i]);
    return MDX_OK;
}
