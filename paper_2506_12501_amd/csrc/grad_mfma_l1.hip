// grad_mfma_l1.hip -- backward kernel instances whose derivative side
// has total Hermite order 1; X(LD, LW, NTN, MTW, NW, WPE, LAY).
#include "grad_mfma.h"

namespace mdx {

#define MDX_GRAD_LIST_1(X) \
    X(1, 0, 1, 2, 4, 2, 0) \
    X(1, 1, 1, 2, 4, 2, 0) \
    X(1, 2, 1, 2, 4, 2, 0) \
    X(1, 3, 1, 2, 4, 2, 0) \
    X(1, 4, 1, 2, 4, 2, 0) \
    X(1, 5, 1, 2, 4, 2, 0) \
    X(1, 6, 1, 2, 4, 2, 0)

MDX_GRAD_DISPATCH(l1, MDX_GRAD_LIST_1)

}  // namespace mdx
