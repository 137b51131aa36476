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
    c->variant[std::make_tuple(ncentre, la, lb, lc, ld, (flags & MDX_CARTESIAN) ? 1 : 0)] = variant;
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
