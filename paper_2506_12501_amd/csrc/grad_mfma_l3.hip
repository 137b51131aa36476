// grad_mfma_l3.hip -- backward kernel instances whose derivative side
// has total Hermite order 3; X(LD, LW, NTN, MTW, NW, WPE, LAY).
#include "grad_mfma.h"

namespace mdx {

#define MDX_GRAD_LIST_3(X) \
    X(3, 0, 1, 4, 4, 2, 0) \
    X(3, 1, 1, 4, 4, 2, 0) \
    X(3, 2, 1, 4, 4, 2, 0) \
    X(3, 3, 1, 4, 4, 2, 0) \
    X(3, 4, 1, 4, 4, 2, 0) \
    X(3, 5, 1, 4, 4, 2, 0) \
    X(3, 6, 1, 4, 4, 2, 0) \
    X(3, 0, 2, 4, 4, 2, 0) \
    X(3, 1, 2, 4, 4, 2, 0) \
    X(3, 2, 2, 4, 4, 2, 0) \
    X(3, 3, 2, 4, 4, 2, 0) \
    X(3, 4, 2, 4, 4, 2, 0) \
    X(3, 5, 2, 4, 4, 2, 0) \
    X(3, 6, 2, 4, 4, 2, 0)

MDX_GRAD_DISPATCH(l3, MDX_GRAD_LIST_3)

}  // namespace mdx
