// grad_mfma_l4.hip -- backward kernel instances whose derivative side
// has total Hermite order 4; X(LD, LW, NTN, MTW, NW, WPE, LAY).
#include "grad_mfma.h"

namespace mdx {

#define MDX_GRAD_LIST_4(X) \
    X(4, 0, 1, 4, 4, 2, 0) \
    X(4, 1, 1, 4, 4, 2, 0) \
    X(4, 2, 1, 4, 4, 2, 0) \
    X(4, 3, 1, 4, 4, 2, 0) \
    X(4, 4, 1, 4, 4, 2, 0) \
    X(4, 5, 1, 4, 4, 2, 0) \
    X(4, 6, 1, 4, 4, 2, 0) \
    X(4, 0, 2, 4, 4, 2, 0) \
    X(4, 1, 2, 4, 4, 2, 0) \
    X(4, 2, 2, 4, 4, 2, 0) \
    X(4, 3, 2, 4, 4, 2, 0) \
    X(4, 4, 2, 4, 4, 2, 0) \
    X(4, 4, 2, 5, 4, 2, 0) \
    X(4, 4, 2, 3, 4, 2, 0) \
    X(4, 4, 2, 4, 4, 1, 0) \
    X(4, 5, 2, 4, 4, 2, 0) \
    X(4, 6, 2, 4, 4, 2, 0) \
    X(4, 0, 3, 3, 4, 2, 0) \
    X(4, 1, 3, 3, 4, 2, 0) \
    X(4, 2, 3, 3, 4, 2, 0) \
    X(4, 3, 3, 3, 4, 2, 0) \
    X(4, 4, 3, 3, 4, 2, 0) \
    X(4, 5, 3, 3, 4, 2, 0) \
    X(4, 6, 3, 3, 4, 2, 0)

MDX_GRAD_DISPATCH(l4, MDX_GRAD_LIST_4)

}  // namespace mdx
