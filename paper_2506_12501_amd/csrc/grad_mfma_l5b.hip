// grad_mfma_l5b.hip -- backward kernel instances whose derivative side
// has total Hermite order 5, 3-4 function tiles; X(LD, LW, NTN, NTW, MTW, NW, WPE, LAY, KP).
#include "grad_mfma.h"

namespace mdx {

#define MDX_GRAD_LIST_L5B(X) \
    X(5, 0, 3, 1, 2, 4, 1, CUBE_LAY_COMPACT, 1) \
    X(5, 1, 3, 1, 2, 4, 1, CUBE_LAY_COMPACT, 1) \
    X(5, 2, 3, 1, 2, 4, 1, CUBE_LAY_COMPACT, 1) \
    X(5, 3, 3, 1, 2, 4, 1, CUBE_LAY_COMPACT, 1) \
    X(5, 3, 3, 2, 2, 4, 1, CUBE_LAY_COMPACT, 1) \
    X(5, 4, 3, 1, 2, 4, 1, CUBE_LAY_COMPACT, 1) \
    X(5, 4, 3, 2, 2, 4, 1, CUBE_LAY_COMPACT, 1) \
    X(5, 4, 3, 3, 2, 4, 1, CUBE_LAY_COMPACT, 1) \
    X(5, 5, 3, 1, 2, 4, 1, CUBE_LAY_COMPACT, 1) \
    X(5, 5, 3, 2, 2, 4, 1, CUBE_LAY_COMPACT, 1) \
    X(5, 5, 3, 3, 2, 4, 1, CUBE_LAY_COMPACT, 1) \
    X(5, 5, 3, 4, 2, 4, 1, CUBE_LAY_COMPACT, 1) \
    X(5, 6, 3, 1, 2, 4, 1, CUBE_LAY_COMPACT, 1) \
    X(5, 6, 3, 2, 2, 4, 1, CUBE_LAY_COMPACT, 1) \
    X(5, 6, 3, 3, 2, 4, 1, CUBE_LAY_COMPACT, 1) \
    X(5, 6, 3, 4, 2, 4, 1, CUBE_LAY_COMPACT, 1) \
    X(5, 0, 4, 1, 2, 4, 1, CUBE_LAY_COMPACT, 1) \
    X(5, 1, 4, 1, 2, 4, 1, CUBE_LAY_COMPACT, 1) \
    X(5, 2, 4, 1, 2, 4, 1, CUBE_LAY_COMPACT, 1) \
    X(5, 3, 4, 1, 2, 4, 1, CUBE_LAY_COMPACT, 1) \
    X(5, 3, 4, 2, 2, 4, 1, CUBE_LAY_COMPACT, 1) \
    X(5, 4, 4, 1, 2, 4, 1, CUBE_LAY_COMPACT, 1) \
    X(5, 4, 4, 2, 2, 4, 1, CUBE_LAY_COMPACT, 1) \
    X(5, 4, 4, 3, 2, 4, 1, CUBE_LAY_COMPACT, 1) \
    X(5, 5, 4, 1, 2, 4, 1, CUBE_LAY_COMPACT, 1) \
    X(5, 5, 4, 2, 2, 4, 1, CUBE_LAY_COMPACT, 1) \
    X(5, 5, 4, 3, 2, 4, 1, CUBE_LAY_COMPACT, 1) \
    X(5, 5, 4, 4, 2, 4, 1, CUBE_LAY_COMPACT, 1) \
    X(5, 6, 4, 1, 2, 4, 1, CUBE_LAY_COMPACT, 1) \
    X(5, 6, 4, 2, 2, 4, 1, CUBE_LAY_COMPACT, 1) \
    X(5, 6, 4, 3, 2, 4, 1, CUBE_LAY_COMPACT, 1) \
    X(5, 6, 4, 4, 2, 4, 1, CUBE_LAY_COMPACT, 1)

MDX_GRAD_DISPATCH(l5b, MDX_GRAD_LIST_L5B)

}  // namespace mdx
