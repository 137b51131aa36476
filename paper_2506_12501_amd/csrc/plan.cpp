// plan.cpp -- multi-class plans (filled in below the class runtime).
#include "runtime.h"

struct mdx_plan {
    int dummy;
};

extern "C" mdx_status mdx_plan_create(mdx_ctx *, const mdx_shells *, int, const mdx_batch_desc *, int, mdx_plan **out)
{
    if (out) *out = nullptr;
    return mdx::fail(MDX_EUNSUPPORTED, "plans not built yet");
}
extern "C" size_t mdx_plan_workspace_size(const mdx_plan *) { return 0; }
extern "C" int64_t mdx_plan_output_size(const mdx_plan *) { return 0; }
extern "C" mdx_status mdx_plan_execute(mdx_plan *, const mdx_shells *, double *, void *, size_t, mdx_stream_t)
{
    return mdx::fail(MDX_EUNSUPPORTED, "plans not built yet");
}
extern "C" void mdx_plan_destroy(mdx_plan *) {}
extern "C" mdx_status mdx_set_variant(mdx_ctx *c, int ncentre, int la, int lb, int lc, int ld, int flags, int variant)
{
    if (!c) return mdx::fail(MDX_EINVAL, "null context");
    if (ncentre < 2 || ncentre > 4 || la < 0 || lc < 0 || (ncentre == 4 && lb < 0) || (ncentre >= 3 && ld < 0) ||
        la > 8 || lb > 8 || lc > 8 || ld > 8)
        return mdx::fail(MDX_EINVAL, "mdx_set_variant: bad class");
    if (flags & ~(MDX_CARTESIAN | MDX_GRADIENT)) return mdx::fail(MDX_EINVAL, "mdx_set_variant: unknown flags 0x%x", flags);
    const bool cart = (flags & MDX_CARTESIAN) != 0;
    const auto key_t = std::make_tuple(ncentre, la, ncentre == 4 ? lb : -1, lc, ncentre >= 3 ? ld : -1, cart ? 1 : 0);
    if (flags & MDX_GRADIENT) {
        if (variant < 0) {
            c->grad_variant.erase(key_t);
            return MDX_OK;
        }
        if (variant < 1 || variant > mdx::grad_class_variants(ncentre, la, lb, lc, ld, cart))
            return mdx::fail(MDX_EINVAL, "mdx_set_variant: class has no backward variant %d", variant);
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
    int nab = mdx::nfunc(la, cart) * (bra2 ? mdx::nfunc(lb, cart) : 1);
    int ncd = mdx::nfunc(lc, cart) * (ket2 ? mdx::nfunc(ld, cart) : 1);
    bool gb = !bra2 && !cart, gk = !ket2 && !cart;
    if (ncentre == 4 && Lb < Lk) {
        std::swap(Lb, Lk);
        std::swap(nab, ncd);
    }
    const mdx::EriKey k{Lb, Lk, nab, ncd, gb, gk};
    const bool ok = variant == 0 ? mdx::eri_valu_has(k) : variant <= mdx::eri_mfma_variants(k);
    if (!ok) return mdx::fail(MDX_EINVAL, "mdx_set_variant: class has no variant %d", variant);
    c->variant[key_t] = variant;
    return MDX_OK;
}

extern "C" mdx_status mdx_set_profile_events(mdx_ctx *c, void *const *events, int nevents)
{
    if (!c) return mdx::fail(MDX_EINVAL, "null context");
    if (nevents < 0 || (nevents & 1)) return mdx::fail(MDX_EINVAL, "nevents = %d must be even and >= 0", nevents);
    c->prof_events.clear();
    c->prof_count = 0;
    if (events)
        for (int i = 0; i < nevents; ++i) c->prof_events.push_back((hipEvent_t)events[i]);
    return MDX_OK;
}
