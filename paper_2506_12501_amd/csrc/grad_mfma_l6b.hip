// grad_mfma_l6b.hip -- backward kernel instances whose derivative side
// has total Hermite order 6, 3 function tiles; X(LD, LW, NTN, NTW, MTW, NW, WPE, LAY, KP).
#include "grad_mfma.h"

namespace mdx {

#define MDX_GRAD_LIST_L6B(X) \
    X(6, 0, 3, 1, 2, 4, 1, CUBE_LAY_COMPACT, 1) \
    X(6, 1, 3, 1, 2, 4, 1, CUBE_LAY_COMPACT, 1) \
    X(6, 2, 3, 1, 2, 4, 1, CUBE_LAY_COMPACT, 1) \
    X(6, 3, 3, 1, 2, 4, 1, CUBE_LAY_COMPACT, 1) \
    X(6, 3, 3, 2, 2, 4, 1, CUBE_LAY_COMPACT, 1) \
    X(6, 4, 3, 1, 2, 4, 1, CUBE_LAY_COMPACT, 1) \
    X(6, 4, 3, 2, 2, 4, 1, CUBE_LAY_COMPACT, 1) \
    X(6, 4, 3, 3, 2, 4, 1, CUBE_LAY_COMPACT, 1) \
    X(6, 5, 3, 1, 2, 4, 1, CUBE_LAY_COMPACT, 1) \
    X(6, 5, 3, 2, 2, 4, 1, CUBE_LAY_COMPACT, 1) \
    X(6, 5, 3, 3, 2, 4, 1, CUBE_LAY_COMPACT, 1) \
    X(6, 5, 3, 4, 2, 4, 1, CUBE_LAY_COMPACT, 1) \
    X(6, 6, 3, 1, 2, 4, 1, CUBE_LAY_COMPACT, 1) \
    X(6, 6, 3, 2, 2, 4, 1, CUBE_LAY_COMPACT, 1) \
    X(6, 6, 3, 3, 2, 4, 1, CUBE_LAY_COMPACT, 1) \
    X(6, 6, 3, 4, 2, 4, 1, CUBE_LAY_COMPACT, 1)

MDX_GRAD_DISPATCH(l6b, MDX_GRAD_LIST_L6B)

}  // namespace mdx
