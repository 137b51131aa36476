// digest.h -- contraction of integral blocks with pair-blocked densities
// at the output store of the integral kernels (the "consume" use of a batch:
// a Coulomb-matrix build never writes the integrals to memory).
#pragma once

#include "kernels.h"

namespace mdx {

// Digestion of one 16 x 4 block of a shellset (I, J) held one element per
// lane: lane (g, c) holds element (ab, cd) = v, valid where ab_ok and cd_ok;
// dk = Dk[J + nk*cd] and db = Db[I + nb*ab] (the caller stages them).
// Every lane of the wave must call it.  The Jb terms are summed over the 16
// lanes of a row group (xor 1..8), the Jk terms over the 4 lanes of a column
// (xor 16, 32); one lane per row / column then adds to J with a vector
// atomic.
__device__ __forceinline__ void digest_block(const Digest &d, int I, int J, int ab, int cd, bool ab_ok, bool cd_ok,
                                             double v, int g, int c, double dk, double db)
{
    const bool ok = ab_ok && cd_ok;
    if (d.Jb) {
        double sb = ok ? v * dk : 0.0;
        sb += __shfl_xor(sb, 1);
        sb += __shfl_xor(sb, 2);
        sb += __shfl_xor(sb, 4);
        sb += __shfl_xor(sb, 8);
        if (c == 0 && ab_ok) atomicAdd(d.Jb + I + d.nb * ab, sb);
    }
    if (d.Jk) {
        double sk = ok ? v * db : 0.0;
        sk += __shfl_xor(sk, 16);
        sk += __shfl_xor(sk, 32);
        if (g == 0 && cd_ok) atomicAdd(d.Jk + J + d.nk * cd, sk);
    }
}

}  // namespace mdx
