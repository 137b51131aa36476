// grad_mfma_l0.hip -- backward kernel instances whose derivative side
// has total Hermite order 0; X(LD, LW, NTN, NTW, MTW, NW, WPE, LAY, KP).
#include "grad_mfma.h"

namespace mdx {

#define MDX_GRAD_LIST_L0(X) \
    X(0, 0, 1, 1, 2, 4, 2, 0, 1) \
    X(0, 1, 1, 1, 2, 4, 2, 0, 1) \
    X(0, 2, 1, 1, 2, 4, 2, 0, 1) \
    X(0, 3, 1, 1, 2, 4, 2, 0, 1) \
    X(0, 3, 1, 2, 2, 4, 2, 0, 1) \
    X(0, 4, 1, 1, 2, 4, 2, 0, 1) \
    X(0, 4, 1, 2, 2, 4, 2, 0, 1) \
    X(0, 4, 1, 3, 2, 4, 2, 0, 1) \
    X(0, 5, 1, 1, 2, 4, 2, 0, 1) \
    X(0, 5, 1, 2, 2, 4, 2, 0, 1) \
    X(0, 5, 1, 3, 2, 4, 2, 0, 1) \
    X(0, 5, 1, 4, 2, 4, 2, 0, 1) \
    X(0, 6, 1, 1, 2, 4, 2, 0, 1) \
    X(0, 6, 1, 2, 2, 4, 2, 0, 1) \
    X(0, 6, 1, 3, 2, 4, 2, 0, 1) \
    X(0, 6, 1, 4, 2, 4, 2, 0, 1)

MDX_GRAD_DISPATCH(l0, MDX_GRAD_LIST_L0)

}  // namespace mdx
