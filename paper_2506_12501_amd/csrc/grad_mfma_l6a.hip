// grad_mfma_l6a.hip -- backward kernel instances whose derivative side
// has total Hermite order 6, 1-2 function tiles; X(LD, LW, NTN, NTW, MTW, NW, WPE, LAY, KP).
#include "grad_mfma.h"

namespace mdx {

#define MDX_GRAD_LIST_L6A(X) \
    X(6, 0, 1, 1, 2, 4, 1, CUBE_LAY_COMPACT, 1) \
    X(6, 1, 1, 1, 2, 4, 1, CUBE_LAY_COMPACT, 1) \
    X(6, 2, 1, 1, 2, 4, 1, CUBE_LAY_COMPACT, 1) \
    X(6, 3, 1, 1, 2, 4, 1, CUBE_LAY_COMPACT, 1) \
    X(6, 3, 1, 2, 2, 4, 1, CUBE_LAY_COMPACT, 1) \
    X(6, 4, 1, 1, 2, 4, 1, CUBE_LAY_COMPACT, 1) \
    X(6, 4, 1, 2, 2, 4, 1, CUBE_LAY_COMPACT, 1) \
    X(6, 4, 1, 3, 2, 4, 1, CUBE_LAY_COMPACT, 1) \
    X(6, 5, 1, 1, 2, 4, 1, CUBE_LAY_COMPACT, 1) \
    X(6, 5, 1, 2, 2, 4, 1, CUBE_LAY_COMPACT, 1) \
    X(6, 5, 1, 3, 2, 4, 1, CUBE_LAY_COMPACT, 1) \
    X(6, 5, 1, 4, 2, 4, 1, CUBE_LAY_COMPACT, 1) \
    X(6, 6, 1, 1, 2, 4, 1, CUBE_LAY_COMPACT, 1) \
    X(6, 6, 1, 2, 2, 4, 1, CUBE_LAY_COMPACT, 1) \
    X(6, 6, 1, 3, 2, 4, 1, CUBE_LAY_COMPACT, 1) \
    X(6, 6, 1, 4, 2, 4, 1, CUBE_LAY_COMPACT, 1) \
    X(6, 0, 2, 1, 2, 4, 1, CUBE_LAY_COMPACT, 1) \
    X(6, 1, 2, 1, 2, 4, 1, CUBE_LAY_COMPACT, 1) \
    X(6, 2, 2, 1, 2, 4, 1, CUBE_LAY_COMPACT, 1) \
    X(6, 3, 2, 1, 2, 4, 1, CUBE_LAY_COMPACT, 1) \
    X(6, 3, 2, 2, 2, 4, 1, CUBE_LAY_COMPACT, 1) \
    X(6, 4, 2, 1, 2, 4, 1, CUBE_LAY_COMPACT, 1) \
    X(6, 4, 2, 2, 2, 4, 1, CUBE_LAY_COMPACT, 1) \
    X(6, 4, 2, 3, 2, 4, 1, CUBE_LAY_COMPACT, 1) \
    X(6, 5, 2, 1, 2, 4, 1, CUBE_LAY_COMPACT, 1) \
    X(6, 5, 2, 2, 2, 4, 1, CUBE_LAY_COMPACT, 1) \
    X(6, 5, 2, 3, 2, 4, 1, CUBE_LAY_COMPACT, 1) \
    X(6, 5, 2, 4, 2, 4, 1, CUBE_LAY_COMPACT, 1) \
    X(6, 6, 2, 1, 2, 4, 1, CUBE_LAY_COMPACT, 1) \
    X(6, 6, 2, 2, 2, 4, 1, CUBE_LAY_COMPACT, 1) \
    X(6, 6, 2, 3, 2, 4, 1, CUBE_LAY_COMPACT, 1) \
    X(6, 6, 2, 4, 2, 4, 1, CUBE_LAY_COMPACT, 1)

MDX_GRAD_DISPATCH(l6a, MDX_GRAD_LIST_L6A)

}  // namespace mdx
