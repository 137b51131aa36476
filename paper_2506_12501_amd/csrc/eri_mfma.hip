// eri_mfma.hip -- placeholder until the matrix-core kernel lands.
#include "kernels.h"

namespace mdx {
bool eri_mfma_has(const EriKey &) { return false; }
bool eri_mfma_launch(const EriKey &, const EriArgs &, int, int, hipStream_t) { return false; }
}  // namespace mdx
