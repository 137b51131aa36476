// grad_mfma_l6c.hip -- backward kernel instances whose derivative side
// has total Hermite order 6, 4 function tiles; X(LD, LW, NTN, NTW, MTW, NW, WPE, LAY, KP).
#include "grad_mfma.h"

namespace mdx {

#define MDX_GRAD_LIST_L6C(X) \
    X(6, 0, 4, 1, 2, 4, 1, CUBE_LAY_COMPACT, 1) \
    X(6, 1, 4, 1, 2, 4, 1, CUBE_LAY_COMPACT, 1) \
    X(6, 2, 4, 1, 2, 4, 1, CUBE_LAY_COMPACT, 1) \
    X(6, 3, 4, 1, 2, 4, 1, CUBE_LAY_COMPACT, 1) \
    X(6, 3, 4, 2, 2, 4, 1, CUBE_LAY_COMPACT, 1) \
    X(6, 4, 4, 1, 2, 4, 1, CUBE_LAY_COMPACT, 1) \
    X(6, 4, 4, 2, 2, 4, 1, CUBE_LAY_COMPACT, 1) \
    X(6, 4, 4, 3, 2, 4, 1, CUBE_LAY_COMPACT, 1) \
    X(6, 5, 4, 1, 2, 4, 1, CUBE_LAY_COMPACT, 1) \
    X(6, 5, 4, 2, 2, 4, 1, CUBE_LAY_COMPACT, 1) \
    X(6, 5, 4, 3, 2, 4, 1, CUBE_LAY_COMPACT, 1) \
    X(6, 5, 4, 4, 2, 4, 1, CUBE_LAY_COMPACT, 1) \
    X(6, 6, 4, 1, 2, 4, 1, CUBE_LAY_COMPACT, 1) \
    X(6, 6, 4, 2, 2, 4, 1, CUBE_LAY_COMPACT, 1) \
    X(6, 6, 4, 3, 2, 4, 1, CUBE_LAY_COMPACT, 1) \
    X(6, 6, 4, 4, 2, 4, 1, CUBE_LAY_COMPACT, 1)

MDX_GRAD_DISPATCH(l6c, MDX_GRAD_LIST_L6C)

}  // namespace mdx
