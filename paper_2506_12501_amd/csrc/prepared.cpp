// prepared.cpp -- batches planned once and run many times (mdx_*_prepare,
// mdx_*_run).  A run enqueues only kernel launches on the caller's stream:
// no host tables are copied and nothing is allocated, so a run can be
// captured into a HIP graph, and its host cost does not grow with the batch.
#include <hip/hip_runtime.h>

#include <cstring>

#include "runtime.h"

namespace mdx {

mdx_status batch_init(mdx_batch *b, mdx_ctx *c, const mdx_shells *sh, int kind, int flags)
{
    b->c = c;
    b->kind = kind;
    b->flags = flags;
    b->nshell = sh->nshell;
    if (sh->nshell > 0) {
        b->l.assign(sh->l, sh->l + sh->nshell);
        b->nprim.assign(sh->nprim, sh->nprim + sh->nshell);
        b->poff.assign(sh->prim_offset, sh->prim_offset + sh->nshell);
    }
    return MDX_OK;
}

mdx_status batch_tables(mdx_batch *b, size_t bytes)
{
    if (bytes == 0) return MDX_OK;
    HIP_TRY2(hipSetDevice(b->c->device));
    if (hipMalloc((void **)&b->dtab, bytes) != hipSuccess) {
        b->dtab = nullptr;
        (void)hipGetLastError();
        return fail(MDX_ENOMEM, "prepared batch: %zu bytes of device tables", bytes);
    }
    return MDX_OK;
}

mdx_status batch_check(const mdx_batch *b, const mdx_shells *sh, int kind, const void *ws, size_t ws_bytes,
                       const char *who)
{
    if (!b) return fail(MDX_EINVAL, "%s: null batch", who);
    if (b->kind != kind)
        return fail(MDX_EINVAL, "%s: the batch was prepared for another integral kind", who);
    if (!sh || sh->nshell != b->nshell ||
        (b->nshell > 0 && (!sh->l || !sh->nprim || !sh->prim_offset || !sh->center || !sh->exponent || !sh->coef)))
        return fail(MDX_EINVAL, "%s: shell table does not match the prepared batch", who);
    if (b->nshell > 0 && (std::memcmp(sh->l, b->l.data(), b->nshell * 4) ||
                          std::memcmp(sh->nprim, b->nprim.data(), b->nshell * 4) ||
                          std::memcmp(sh->prim_offset, b->poff.data(), b->nshell * 4)))
        return fail(MDX_EINVAL, "%s: shell metadata differ from the prepared batch's", who);
    if (b->ws_need > 0) {
        if (!ws) return fail(MDX_EINVAL, "%s: null workspace", who);
        if ((uintptr_t)ws & 255) return fail(MDX_EINVAL, "%s: workspace not 256-byte aligned", who);
        if (ws_bytes < b->ws_need)
            return fail(MDX_EWORKSPACE, "%s: workspace %zu bytes < %zu required", who, ws_bytes, b->ws_need);
    }
    int dev = -1;
    HIP_TRY2(hipGetDevice(&dev));
    if (dev != b->c->device) HIP_TRY2(hipSetDevice(b->c->device));
    return MDX_OK;
}

}  // namespace mdx

using namespace mdx;

extern "C" size_t mdx_batch_workspace_size(const mdx_batch *b) { return b ? b->ws_need + 256 : 0; }

extern "C" int64_t mdx_batch_output_size(const mdx_batch *b) { return b ? b->out_doubles : 0; }

extern "C" void mdx_batch_destroy(mdx_batch *b)
{
    if (!b) return;
    if (b->dtab) (void)hipSetDevice(b->c->device);
    delete b;
}
