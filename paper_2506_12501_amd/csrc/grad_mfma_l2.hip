// grad_mfma_l2.hip -- backward kernel instances whose derivative side
// has total Hermite order 2; X(LD, LW, NTN, NTW, MTW, NW, WPE, LAY, KP).
#include "grad_mfma.h"

namespace mdx {

#define MDX_GRAD_LIST_L2(X) \
    X(2, 0, 1, 1, 3, 4, 2, 0, 1) \
    X(2, 1, 1, 1, 3, 4, 2, 0, 1) \
    X(2, 2, 1, 1, 3, 4, 2, 0, 1) \
    X(2, 3, 1, 1, 3, 4, 2, 0, 1) \
    X(2, 3, 1, 2, 3, 4, 2, 0, 1) \
    X(2, 4, 1, 1, 3, 4, 2, 0, 1) \
    X(2, 4, 1, 2, 3, 4, 2, 0, 1) \
    X(2, 4, 1, 3, 3, 4, 2, 0, 1) \
    X(2, 5, 1, 1, 3, 4, 2, 0, 1) \
    X(2, 5, 1, 2, 3, 4, 2, 0, 1) \
    X(2, 5, 1, 3, 3, 4, 2, 0, 1) \
    X(2, 5, 1, 4, 3, 4, 2, 0, 1) \
    X(2, 6, 1, 1, 3, 4, 2, 0, 1) \
    X(2, 6, 1, 2, 3, 4, 2, 0, 1) \
    X(2, 6, 1, 3, 3, 4, 2, 0, 1) \
    X(2, 6, 1, 4, 3, 4, 2, 0, 1)

MDX_GRAD_DISPATCH(l2, MDX_GRAD_LIST_L2)

}  // namespace mdx
