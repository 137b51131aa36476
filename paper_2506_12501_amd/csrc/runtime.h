// runtime.h -- host-side state and planning helpers.
#pragma once

#include <hip/hip_runtime.h>

#include <array>
#include <cstdarg>
#include <map>
#include <string>
#include <tuple>
#include <vector>

#include "../../include/mdx.h"
#include "kernels.h"
#include "mdx_internal.h"

struct mdx_ctx {
    int device = 0;
    int ncu = 0;
    double *boys = nullptr;      // Boys table
    double *solid = nullptr;     // Cartesian->solid coefficients, l <= 8
    size_t solid_off[9] = {};
    std::vector<std::vector<double>> solid_host;
    double *tket = nullptr;      // terminal ket matrices
    size_t tket_off[2][MDX_LMAX_4C + 1][MDX_LMAX_4C + 1] = {};
    size_t tket1_off[2][7] = {};
    std::map<std::tuple<int, int, int, int, int, int>, int> variant;        // autotuner overrides
    std::map<std::tuple<int, int, int, int, int, int>, int> grad_variant;   // same, backward kernel
    char *scratch = nullptr;     // device address of the static scratch buffer (mdx_eri_batch_noalloc)
    std::vector<hipEvent_t> prof_events;   // profiling hook (pairs)
    size_t prof_count = 0;
};

#define HIP_TRY2(expr)                                                                        \
    do {                                                                                      \
        hipError_t e_ = (expr);                                                               \
        if (e_ != hipSuccess) return mdx::fail(MDX_EDEVICE, "%s: %s", #expr, hipGetErrorString(e_)); \
    } while (0)

#define MDX_TRY(expr)                          \
    do {                                       \
        const mdx_status st_ = (expr);         \
        if (st_ != MDX_OK) return st_;         \
    } while (0)

namespace mdx {

mdx_status fail(mdx_status s, const char *fmt, ...);
void build_tket(mdx_ctx *c, int lc, int ld, bool cart, std::vector<double> &T);

// One side of a class in kernel orientation, with its pair list.
struct SidePlan {
    SideGeom g{};
    std::vector<PairRec> pairs;
    std::vector<int2> items;   // (pair, primitive pair) for the pair-data kernel; empty if grouped
};

// kernel families
enum KernelKind { K_VALU = 0, K_MFMA = 1 };

// A planned class batch (kernel orientation).
struct ClassPlan {
    int ncentre = 4;
    int cart = 0;
    int la = 0, lb = 0, lc = 0, ld = 0;   // caller's
    bool swapped = false;                 // kernel bra = caller ket
    bool diag = false;                    // only the shellsets I = J (Schwarz factors, paired batches)
    bool paired = false;                  // MDX_PAIRED: quartet q = (bra q, ket q), out[q + n*(ab + nab*cd)]
    bool expand = false;                  // single-primitive kernel over each primitive combination of
                                          // contracted pairs, accumulated (one contraction degree per side)
    SidePlan bra, ket;
    EriKey key{};
    KernelKind kind = K_VALU;
    int variant = 0;
    int bra_per_tile = 1;                 // matrix-core tile: bra pairs / functions per workgroup
    OutMap om{};
    // ragged output (plans): per kernel-ket bra counts and bases
    std::vector<int32_t> count;
    std::vector<int64_t> obase;
    int64_t out_doubles = 0;
    // ragged launches: tiles before each kernel ket pair ([nket+1])
    std::vector<int32_t> tile_off;
    const double *tket = nullptr;
};

// device layout of one class: the index tables built on the host (offsets
// from the table region), then the pair data the pair-data kernels write
// (offsets from the work region).  A plain call puts both in its workspace,
// tables first; a prepared batch keeps the tables in memory of its own.
struct WsLayout {
    size_t pairs_bra, pairs_ket, items_bra, items_ket, count, obase, tile_off;   // table region
    size_t np_bra, np_ket, prim_bra, prim_ket, H_bra, H_ket;                     // work region
    size_t tables, work, total;                                                  // total = tables + work
};

SideGeom make_geom(int la, int lb, bool cart, int role, int npair, int kmax, bool allow_grouped);
SidePlan make_side(const mdx_shells *sh, const int32_t *lst, int32_t n, bool two, int l0, int l1, bool cart,
                   int role, bool allow_grouped);
// validates a class batch; l = (l_a, l_b, l_c, l_d), -1 for absent functions
// (all -1 when the batch is empty)
mdx_status check_class(mdx_ctx *c, const mdx_shells *sh, int ncentre, int32_t nbra, const int32_t *bra,
                       int32_t nket, const int32_t *ket, int flags, int l[4]);
// largest backward-kernel variant count over the passes of a class (0: none)
int grad_class_variants(int ncentre, int la, int lb, int lc, int ld, bool cart);
mdx_status plan_class(mdx_ctx *c, const mdx_shells *sh, int ncentre, int32_t nbra, const int32_t *bra,
                      int32_t nket, const int32_t *ket, const int32_t *bra_count, int flags, ClassPlan &cp);
WsLayout ws_layout(const ClassPlan &cp);
// device addresses of one class's tables and pair data
struct ClassDev {
    const PairRec *pairs_bra, *pairs_ket;
    const int2 *items_bra, *items_ket;
    const int32_t *count;
    const int64_t *obase;
    const int32_t *tile_off;
    PrimRec *prim_bra, *prim_ket;
    int32_t *np_bra, *np_ket;
    double *H_bra, *H_ket;
};
ClassDev class_dev(const WsLayout &L, const char *tabs, char *work);
ClassDev class_dev(const WsLayout &L, char *ws);   // tables at ws, work region after them
// copies the index tables from host memory (refused while the stream is captured)
mdx_status upload_tables(const ClassPlan &cp, const ClassDev &d, hipStream_t s);
// device copy of the index tables into dst (L.tables bytes), synchronous
mdx_status copy_tables(const ClassPlan &cp, const WsLayout &L, char *dst);
// MDX_EINVAL if s is being captured into a graph: calls that copy host tables
// per call cannot be replayed (their prepared forms can)
mdx_status refuse_capture(hipStream_t s, const char *why);
void enqueue_pairdata(mdx_ctx *c, const mdx_shells *sh, const ClassPlan &cp, const ClassDev &d, int side,
                      hipStream_t s);
mdx_status class_args(mdx_ctx *c, const ClassPlan &cp, const ClassDev &d, double *out, EriArgs &a, int &nblocks);
mdx_status launch_class(mdx_ctx *c, const ClassPlan &cp, const EriArgs &a, int nblocks, hipStream_t s);
mdx_status enqueue_class(mdx_ctx *c, const mdx_shells *sh, const ClassPlan &cp, const WsLayout &L, char *ws,
                         double *out, hipStream_t s, bool upload,
                         const Digest *dig = nullptr);
// the same with the tables already on the device at d (no upload)
mdx_status enqueue_class_dev(mdx_ctx *c, const mdx_shells *sh, const ClassPlan &cp, const ClassDev &d, double *out,
                             hipStream_t s, const Digest *dig = nullptr);

// the lane records of a 1-particle batch (pairs validated)
void onebody_records(const mdx_shells *sh, int32_t npair, const int32_t *pairs, std::vector<PairRec> &pr);
// one launch of the overlap/kinetic or nuclear kernels of class (la, lb) over
// resident lane records
mdx_status onebody_launch(mdx_ctx *c, const mdx_shells *sh, const PairRec *pairs, int32_t npair, int la, int lb,
                          bool cart, double *S, double *T, hipStream_t s);
mdx_status nuclear_lane_launch(mdx_ctx *c, const mdx_shells *sh, const PairRec *pairs, int32_t npair, int la,
                               int lb, bool cart, int32_t ncharge, const double *charges, double *V, hipStream_t s);

}  // namespace mdx

// A prepared batch (mdx_eri_prepare, mdx_one_body_prepare, mdx_nuclear_prepare):
// the host planning of one call done once, its index tables resident in
// device memory of its own, so that a run enqueues kernels only.
enum BatchKind { B_ERI = 1, B_ONEBODY = 2, B_NUC = 3 };

struct mdx_batch {
    mdx_ctx *c = nullptr;
    int kind = 0;
    int flags = 0;
    int32_t nshell = 0;                      // basis metadata at preparation
    std::vector<int32_t> l, nprim, poff;
    char *dtab = nullptr;                    // device index tables
    size_t ws_need = 0;                      // workspace bytes of a run
    int64_t out_doubles = 0;                 // doubles per output array
    mdx::ClassPlan cp;                       // B_ERI
    mdx::WsLayout L{};
    int la = -1, lb = -1;                    // 1-particle classes
    int32_t npair = 0, ncharge = 0;
    ~mdx_batch()
    {
        if (dtab) hipFree(dtab);
    }
};

namespace mdx {
// records the context, kind and basis metadata of a new batch
mdx_status batch_init(mdx_batch *b, mdx_ctx *c, const mdx_shells *sh, int kind, int flags);
// allocates `bytes` of device memory for the batch's index tables (MDX_ENOMEM
// on failure; nothing for 0 bytes)
mdx_status batch_tables(mdx_batch *b, size_t bytes);
// run-time checks shared by the run calls: kind, shell table against the
// metadata at preparation, workspace; makes the context's device current
mdx_status batch_check(const mdx_batch *b, const mdx_shells *sh, int kind, const void *ws, size_t ws_bytes,
                       const char *who);
}  // namespace mdx

