// grad_mfma_l1.hip -- backward kernel instances whose derivative side
// has total Hermite order 1; X(LD, LW, NTN, NTW, MTW, NW, WPE, LAY, KP).
#include "grad_mfma.h"

namespace mdx {

#define MDX_GRAD_LIST_L1(X) \
    X(1, 0, 1, 1, 2, 4, 2, 0, 1) \
    X(1, 1, 1, 1, 2, 4, 2, 0, 1) \
    X(1, 2, 1, 1, 2, 4, 2, 0, 1) \
    X(1, 3, 1, 1, 2, 4, 2, 0, 1) \
    X(1, 3, 1, 2, 2, 4, 2, 0, 1) \
    X(1, 4, 1, 1, 2, 4, 2, 0, 1) \
    X(1, 4, 1, 2, 2, 4, 2, 0, 1) \
    X(1, 4, 1, 3, 2, 4, 2, 0, 1) \
    X(1, 5, 1, 1, 2, 4, 2, 0, 1) \
    X(1, 5, 1, 2, 2, 4, 2, 0, 1) \
    X(1, 5, 1, 3, 2, 4, 2, 0, 1) \
    X(1, 5, 1, 4, 2, 4, 2, 0, 1) \
    X(1, 6, 1, 1, 2, 4, 2, 0, 1) \
    X(1, 6, 1, 2, 2, 4, 2, 0, 1) \
    X(1, 6, 1, 3, 2, 4, 2, 0, 1) \
    X(1, 6, 1, 4, 2, 4, 2, 0, 1)

MDX_GRAD_DISPATCH(l1, MDX_GRAD_LIST_L1)

}  // namespace mdx
