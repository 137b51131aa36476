// grad.cpp -- mdx_eri_grad_batch (backward pass).
#include "runtime.h"

extern "C" size_t mdx_eri_grad_workspace_size(mdx_ctx *, const mdx_shells *, int, int32_t, const int32_t *, int32_t,
                                              const int32_t *, int)
{
    return 0;
}
extern "C" mdx_status mdx_eri_grad_batch(mdx_ctx *, const mdx_shells *, int, int32_t, const int32_t *, int32_t,
                                         const int32_t *, int, const double *, double *, void *, size_t, mdx_stream_t)
{
    return mdx::fail(MDX_EUNSUPPORTED, "gradient not built yet");
}
