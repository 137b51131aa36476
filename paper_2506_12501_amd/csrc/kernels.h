// kernels.h -- launch interfaces of the gfx950 kernels (host side).
#pragma once

#include "mdx_internal.h"

namespace mdx {

// 1/sqrt(x) and 1/x for positive, normal, finite x: the hardware estimates
// refined by two Newton steps each (to about an ulp; no IEEE rounding
// fix-ups, which cost two to three times as many instructions)
__device__ __forceinline__ double rsqrt_d(double x)
{
    double y = __builtin_amdgcn_rsq(x);
    const double h = 0.5 * x;
    y = fma(y, fma(-h * y, y, 0.5), y);
    y = fma(y, fma(-h * y, y, 0.5), y);
    return y;
}
// Read of data that no kernel writes while the reading kernel runs (pair data,
// tables), through the constant address space: with a wave-uniform address the
// compiler issues a scalar load instead of one vector load per lane.
template <typename T>
__device__ __forceinline__ T load_const(const T *p)
{
    static_assert(sizeof(T) % 4 == 0, "whole words");
    typedef const __attribute__((address_space(4))) int cint;
    cint *q = (cint *)(const void *)p;
    T r;
    int *d = (int *)&r;
#pragma unroll
    for (int i = 0; i < (int)(sizeof(T) / 4); ++i) d[i] = q[i];
    return r;
}

__device__ __forceinline__ double rcp_d(double x)
{
    double r = __builtin_amdgcn_rcp(x);
    r = fma(r, fma(-x, r, 1.0), r);
    r = fma(r, fma(-x, r, 1.0), r);
    return r;
}

// Blocks are dealt to the 8 XCDs round-robin.  Renumber them so that each XCD
// receives a contiguous range of work items (consecutive bra pairs of a ket
// pair share that XCD's L2 and its output cache lines).
__device__ __forceinline__ int xcd_tile(int b, int n)
{
    const int q = n >> 3, r = n & 7, x = b & 7, k = b >> 3;
    return x * q + min(x, r) + k;
}

// ket pair J and first bra pair of tile t of a ragged batch: tile_off[J] is
// the number of tiles before ket J (binary search; kets without tiles are skipped)
__device__ __forceinline__ void ragged_tile(const int32_t *tile_off, int nket, int t, int &J, int &t0)
{
    int lo = 0, hi = nket;
    while (hi - lo > 1) {
        const int mid = (lo + hi) >> 1;
        if (tile_off[mid] <= t) lo = mid;
        else hi = mid;
    }
    J = lo;
    t0 = t - tile_off[lo];
}

// class key of an integral kernel (kernel orientation)
struct EriKey {
    int LB, LK;     // total Hermite order of bra and ket
    int NAB, NCD;   // functions per bra / ket pair
    bool GB, GK;    // single-function solid sides (primitives summed in [0]^(m))
};

// Contraction of a batch with pair-blocked densities in place of the output
// store (kernel orientation; all zero when the integrals are stored):
//   Jb[I + nb*ab] += sum_{J,cd} (ab|cd)_{I,J} Dk[J + nk*cd]
//   Jk[J + nk*cd] += sum_{I,ab} (ab|cd)_{I,J} Db[I + nb*ab]
struct Digest {
    const double *Db, *Dk;
    double *Jb, *Jk;   // either may be null
    int64_t nb, nk;
    int on;
};

// Dense matrix-core launches walk blocks of MFMA_BRA_RUN consecutive bra
// units x MFMA_KET_RUN ket pairs (128 workgroups): 16 consecutive bra pairs
// fill whole 128-byte lines of the [ij, ab, cd, kl] output.
constexpr int MFMA_BRA_RUN = 16, MFMA_KET_RUN = 8;

struct EriArgs {
    SideDev bra, ket;
    int nbra, nket;
    int tiles_per_J;          // dense tiling: bra tiles (VALU) / 8-pair bra blocks (MFMA)
    const int32_t *tile_off;  // ragged: [nket+1] tiles before each ket pair (VALU tile: 64 bra
                              // pairs, MFMA tile: one), or null
    int diag;                 // 1: only the diagonal shellsets I = J (one per block);
                              // 2 (register kernel): I = J, one per lane
    const double *boys;       // Boys table
    const double *Tket;       // terminal ket matrix [ncart(LK) pad 4][ncolp] (MFMA kernel)
    int ntile_total;          // number of tiles (persistent kernels)
    int nqmax;                // MFMA kernel: primitive quartets held in LDS at once
    int nab, ncd;             // functions per bra / ket pair (kernel orientation)
    int *counter;             // work counter (persistent kernels)
    OutMap om;
    Digest dig;               // dig.on: contract instead of storing (plain launches only)
    int prim_expand;          // single-primitive kernel on one primitive pair of contracted pairs
                              // (the caller offsets the pair-data pointers; see enqueue_class)
    int accumulate;           // single-primitive kernel: add to the output instead of storing
};

struct PairDataArgs {
    SideGeom g;
    const PairRec *pairs;
    const int2 *items;   // (pair, primitive pair) of every block; unused for a grouped side
    int nitems;
    const double *center, *expo, *coef;
    const double *Ca, *Cb;   // solid coefficients [nsph(l)][ncart(l)], null for Cartesian
    PrimRec *prim;
    double *H;
    int32_t *nprim;
    int per_block;       // items per workgroup (set by launch_pairdata)
};
void launch_pairdata(const PairDataArgs &a, hipStream_t s);
// per_block of a record set, its workgroup count returned and LDS bytes in lds
int pairdata_prepare(PairDataArgs &a, size_t &lds);
// records recs[0 .. nrec-1] (prepared, in device memory), record r owning
// workgroups base[r] .. base[r+1]-1 of one launch of nblk = base[nrec]
struct PairDataMulti {
    const PairDataArgs *recs;
    const int32_t *base;
    int nrec;
};
void launch_pairdata_multi(const PairDataMulti &m, int nblk, size_t lds, hipStream_t s);

bool eri_valu_has(const EriKey &k);
bool eri_valu_launch(const EriKey &k, const EriArgs &a, int nblocks, hipStream_t s);
bool eri_mfma_has(const EriKey &k);
int eri_mfma_variants(const EriKey &k);
// Variant kinds of a matrix-core class, numbered in this order: the general
// kernel's instances, then single-primitive kernels (bra and ket pairs of one
// primitive pair each), then 3-centre kernels taking several bra functions per
// workgroup (ket pairs of one primitive pair).
enum { MFMA_GENERAL = 0, MFMA_PRIM = 1, MFMA_MULTI = 2 };
int eri_mfma_variant_kind(const EriKey &k, int variant);
// bra pairs / functions per tile of a variant (one workgroup)
int eri_mfma_bra_per_tile(const EriKey &k, int variant);
int eri_prim_variants(const EriKey &k);
int eri_prim_bra_per_tile(const EriKey &k, int variant);
bool eri_prim_launch(const EriKey &k, const EriArgs &a, int nblocks, int variant, hipStream_t s);
int eri_multi_variants(const EriKey &k);
int eri_multi_bra_per_tile(const EriKey &k, int variant);
bool eri_multi_launch(const EriKey &k, const EriArgs &a, int nblocks, int variant, hipStream_t s);
bool eri_mfma_launch(const EriKey &k, const EriArgs &a, int nblocks, int variant, hipStream_t s);

// Backward kernel arguments.  The derivative side (pair data in the
// derivative-bra role) supplies the rows; the other side (ket role) is
// contracted with the adjoint W inside the kernel.
//   W[I*wsI + J*wsJ + i*wsd + j*wsw]   i: derivative-side function, j: other side
//   G[I*gsI + J*gsJ + slot*gss] = sum_k M[slot][k] g_k   for slots in wmask,
//   g_k (k = 0..5) = sum_ij W d(ij)/d{A_x, A_y, A_z, B_x, B_y, B_z} of the
//   derivative side's two centres.
struct GradArgs {
    SideDev dside, wside;
    int nI, nJ;               // pairs on the derivative / other side
    const double *boys;
    const double *Tw;         // terminal matrix of the other side [ncart(LW) pad 4][nwp]
    int nqmax;
    int nd, nw, nwp;          // functions per pair (derivative side, other side), other side's column stride
    const double *W;
    int64_t wsI, wsJ, wsd, wsw;
    double *G;
    int64_t gsI, gsJ, gss;
    int wmask;
    signed char M[12][6];
};

// class key of a backward kernel: Hermite orders of the two sides and
// 16-column tiles of the derivative side's and the other side's functions
struct GradKey {
    int LD, LW, NTN, NTW;
};
int eri_grad_variants(const GradKey &k);
bool eri_grad_launch(const GradKey &k, const GradArgs &a, int nblocks, int variant, hipStream_t s);

// persistent work-queue launch over several ragged batches of one kernel instance
struct QueueArgs {
    const EriArgs *desc;   // [nb] kernel arguments of each batch (device memory)
    const int32_t *base;   // [nb+1] work items (tiles) before each batch
    int nb;
    int total;             // base[nb]
    int *counter;          // zero before the launch
};
// dig: the digesting form (first shape of a class only)
bool eri_mfma_config(const EriKey &k, int variant, int bra_kmax, int ket_kmax, int &nqmax, size_t &lds, int &nthreads,
                     bool dig = false);
// sets the dynamic-LDS limit of the queue kernel; returns resident workgroups per CU (0: unusable)
int eri_queue_prepare(const EriKey &k, bool mfma, int variant, size_t lds, bool dig = false);
bool eri_queue_launch(const EriKey &k, bool mfma, int variant, const QueueArgs &q, int nblocks, size_t lds,
                      hipStream_t s, bool dig = false);
void launch_schwarz(const double *diag, int npair, int nab, double *Q, hipStream_t s);
void launch_fill_i32(int32_t *p, int n, int32_t v, hipStream_t s);

void launch_boys(const double *x, int n, int mmax, double *F, const double *tab, hipStream_t s);

}  // namespace mdx
