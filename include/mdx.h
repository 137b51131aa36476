/*
 * mdx.h -- C ABI of libmdx: batched McMurchie-Davidson (MD) Gaussian integrals
 * over contracted shells, on one AMD MI355X (gfx950): electron-repulsion
 * integrals (ERIs), their centre derivatives, their contraction with
 * densities, and the 1-particle overlap, kinetic-energy and nuclear-attraction
 * integrals.
 *
 * The integrals are those of Asadchev & Valeev, "Implementation of
 * McMurchie-Davidson algorithm for Gaussian AO integrals suited for SIMD
 * processors" (arXiv:2506.12501):
 *   4-centre (ab|cd)   Sec. 2.1, Eq. (3), over contracted shells, Eq. (5)
 *   3-centre (a|cd)    Sec. 2.1, Eq. (4)
 *   2-centre (a|c)     Eq. (4) with a single ket function (Sec. 2.2.3)
 * evaluated in batches of shellsets of one class (Sec. 2.1, paragraph after
 * Eq. (19); Sec. 3.1), in the [ij,ab,cd,kl] column-major layout of Sec. 3.1;
 * 1-particle integrals of shell pairs (Sec. 2.1, Eq. (8); Eqs. (24)-(37)).
 *
 * Conventions (all entry points):
 *  - Atomic units.  A primitive Cartesian Gaussian is
 *    x_A^ax y_A^ay z_A^az exp(-zeta r_A^2) (Eq. (1)); contraction
 *    coefficients are applied exactly as given (no normalisation).
 *  - Cartesian component order within a shell: (l,0,0), (l-1,1,0),
 *    (l-1,0,1), (l-2,2,0), ... (x power descending, then y descending).
 *  - Real solid harmonics (default; Eqs. (18)-(19)): order m = -l..l, each
 *    normalised to the norm of the x^l Cartesian of the same exponent.
 *  - Everything runs asynchronously on the caller's stream.  The caller owns
 *    every buffer; outputs are overwritten (the J blocks of
 *    mdx_eri_digest_batch are the one exception: accumulated).  Apart from
 *    mdx_create and mdx_plan_create no call allocates device memory: scratch
 *    lives in the caller's workspace (mdx_eri_batch_noalloc: in a static
 *    device buffer of the library).
 *  - On any error no kernel is launched and no output is written.
 *  - One mdx_ctx per device and per host thread (a context is not
 *    thread-safe).  No C++ exception crosses this interface.
 */
#ifndef MDX_H
#define MDX_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* hipStream_t without pulling in the HIP headers */
typedef struct ihipStream_t *mdx_stream_t;

typedef enum {
    MDX_OK = 0,
    MDX_EINVAL = 1,       /* bad argument (null pointer, bad index, mixed classes, ...) */
    MDX_EUNSUPPORTED = 2, /* angular momentum or order beyond the compiled limits */
    MDX_EWORKSPACE = 3,   /* workspace smaller than the matching *_workspace_size */
    MDX_ENOMEM = 4,       /* host-side allocation failed (planning only) */
    MDX_EDEVICE = 5       /* HIP runtime error; mdx_last_error() has the text */
} mdx_status;

/* compiled limits */
#define MDX_LMAX_4C 6      /* l per shell, 4-centre                      */
#define MDX_LMAX_3C 6      /* l of the single-function side, 3-/2-centre */
#define MDX_BOYS_MAX_M 32  /* highest Boys order of mdx_boys             */

/* flags */
#define MDX_SPHERICAL 0    /* real solid harmonics (default)             */
#define MDX_CARTESIAN 1    /* Cartesian components                       */
#define MDX_FUSED 2        /* plans: one graph launch, persistent kernels */
#define MDX_GRADIENT 4     /* mdx_set_variant: choose the backward kernel */
#define MDX_PAIRED 8       /* mdx_eri_batch: quartet q = (bra q, ket q)   */
#define MDX_DIGEST 16      /* plans: contract with densities (mdx_plan_digest) */

typedef struct mdx_ctx mdx_ctx;

/*
 * Shell table, structure of arrays.  Numeric data live on the device (read
 * only, caller-owned); integer metadata live on the host because batching and
 * validation are planned there.
 *   center   DEVICE double[3*nshell]   centre of shell s at center[3s..3s+2]
 *   exponent DEVICE double[nprim_tot]  exponents (> 0) of all primitives
 *   coef     DEVICE double[nprim_tot]  contraction coefficients (as given)
 *   l        HOST int32[nshell]        angular momentum
 *   nprim    HOST int32[nshell]        contraction degree K >= 1
 *   prim_offset HOST int32[nshell]     first primitive of shell s in exponent/coef
 */
typedef struct {
    int32_t nshell;
    const double *center;
    const double *exponent;
    const double *coef;
    const int32_t *l;
    const int32_t *nprim;
    const int32_t *prim_offset;
} mdx_shells;

/* Context: uploads the Boys table and the Cartesian->solid tables to
 * `device`.  Returns MDX_EDEVICE if the device is not a usable gfx950. */
mdx_status mdx_create(int device, mdx_ctx **out);
void mdx_destroy(mdx_ctx *ctx);

/* name of a status code ("MDX_OK", "MDX_EINVAL", ...; static storage) */
const char *mdx_status_string(mdx_status s);
/* text of the last error raised on this thread (static storage) */
const char *mdx_last_error(void);

/*
 * Boys function F_m(x) = int_0^1 y^{2m} exp(-x y^2) dy (Eq. (28)), m = 0..mmax,
 * for n arguments: F[m*n + i] = F_m(x[i]).
 *   x  DEVICE double[n], x >= 0 (finite)
 *   F  DEVICE double[(mmax+1)*n]
 *   0 <= mmax <= MDX_BOYS_MAX_M, n >= 0.
 * Method: tabulated Taylor expansion at the highest order, then downward
 * recursion (Sec. 3.2.1 notes this as the GPU-friendly choice); x >= 45 uses
 * the asymptotic F_0 and upward recursion.
 */
mdx_status mdx_boys(mdx_ctx *ctx, int32_t n, const double *x, int mmax, double *F,
                    mdx_stream_t stream);

/*
 * One class of shellsets, dense outer product of bra pairs x ket pairs.
 *   ncentre 4: bra[2*ij], bra[2*ij+1] are the shells a, b of bra pair ij;
 *              ket[2*kl], ket[2*kl+1] the shells c, d.
 *   ncentre 3: bra[2*ij] is the single shell a (bra[2*ij+1] ignored), ket pairs.
 *   ncentre 2: bra[2*ij] = a, ket[2*kl] = c (second entries ignored).
 *   bra, ket HOST int32 arrays.  Every bra entry must have the same
 *   (l_a, l_b) and every ket entry the same (l_c, l_d).
 *   out DEVICE double, [ij, ab, cd, kl] column-major (Sec. 3.1):
 *       out[ij + nbra*(ab + nab*(cd + ncd*kl))],  ab = a*nb + b, cd = c*nd + d,
 *       nab = n(l_a)*n(l_b) (n(l) = 2l+1 spherical, (l+1)(l+2)/2 Cartesian;
 *       a single-function side has nab = n(l_a)).
 *   flags: MDX_SPHERICAL or MDX_CARTESIAN, optionally | MDX_PAIRED: then
 *       nbra == nket and only the quartets q = (bra q, ket q) are computed,
 *       out[q + nbra*(ab + nab*cd)] (the paired form; pass the same flags to
 *       mdx_eri_workspace_size).
 *   ws, ws_bytes: DEVICE workspace of at least mdx_eri_workspace_size(...)
 *   bytes, 256-byte aligned; its contents on entry do not matter.
 * Limits: l <= MDX_LMAX_4C per shell for 4-centre; l_a <= MDX_LMAX_3C and
 * l_c, l_d <= MDX_LMAX_4C for 3-centre; both <= MDX_LMAX_3C for 2-centre.
 * Within these, a class runs if a kernel is compiled for it (every class with
 * l <= 2 per shell, the d/f/g classes of the matrix-core instance list, and,
 * spherical only, (hh|hh), (ii|ii) and the mixed classes (gg|ff), (gg|dd),
 * (hh|gg), (hh|ff), (hh|dd), (ii|hh), (ii|gg), (ii|ff), (ii|dd)); others
 * return MDX_EUNSUPPORTED.  Classes that run only on a single-primitive
 * kernel take contracted pairs when every pair of a side has the same
 * contraction degree (one launch per primitive combination, Eq. (5)), else
 * MDX_EUNSUPPORTED.
 * The call copies host index tables into the workspace on the stream, so it
 * cannot be captured into a graph: on a capturing stream it returns
 * MDX_EINVAL before any work (capture mdx_eri_run of a prepared batch).
 */
size_t mdx_eri_workspace_size(mdx_ctx *ctx, const mdx_shells *shells, int ncentre, int32_t nbra,
                              const int32_t *bra, int32_t nket, const int32_t *ket, int flags);
mdx_status mdx_eri_batch(mdx_ctx *ctx, const mdx_shells *shells, int ncentre, int32_t nbra,
                         const int32_t *bra, int32_t nket, const int32_t *ket, int flags,
                         double *out, void *ws, size_t ws_bytes, mdx_stream_t stream);

/*
 * mdx_eri_batch for callers that cannot allocate device memory (tight
 * serving loops, harnesses that forbid hipMalloc):
 * the same batch, layouts, flags, limits and errors as mdx_eri_batch, with
 * the workspace taken from a library-owned static device buffer of
 * MDX_NOALLOC_SCRATCH_BYTES bytes per device instead of a caller argument.
 * The call allocates nothing (no hipMalloc, hipFree or allocating library
 * routine).  A batch whose workspace (mdx_eri_workspace_size) exceeds the
 * buffer returns MDX_EWORKSPACE before any launch; split it, or use
 * mdx_eri_batch.  Every call on a device shares that device's buffer: calls
 * that overlap in time on one device (different streams, or host threads)
 * race on it; calls in one stream are ordered and safe.  The buffer is set up
 * by mdx_create and lives until the process ends.  Like mdx_eri_batch, the
 * call copies host index tables on the stream and is refused (MDX_EINVAL) on
 * a stream under graph capture; there, capture mdx_eri_run of a batch
 * prepared beforehand.
 */
#define MDX_NOALLOC_SCRATCH_BYTES (64u << 20)
mdx_status mdx_eri_batch_noalloc(mdx_ctx *ctx, const mdx_shells *shells, int ncentre, int32_t nbra,
                                 const int32_t *bra, int32_t nket, const int32_t *ket, int flags,
                                 double *out, mdx_stream_t stream);

/*
 * The "consume" use of a dense batch (Sec. 3.1: integrals feed a contraction
 * and need not be stored): the batch of mdx_eri_batch contracted with
 * pair-blocked densities inside the integral kernels, so the integrals never
 * reach memory:
 *   Jbra[ij + nbra*ab] += sum_{kl,cd} (ab|cd)_{ij,kl} Dket[kl + nket*cd]
 *   Jket[kl + nket*cd] += sum_{ij,ab} (ab|cd)_{ij,kl} Dbra[ij + nbra*ab]
 * With bra and ket drawn from one list of canonical pairs these are the
 * Coulomb-matrix blocks J_ab = sum_cd (ab|cd) D_cd of the two pair sets; the
 * caller gathers D into pair blocks and scatters J back, with its own
 * symmetry factors.
 *   Dbra, Dket DEVICE double[nbra*nab], [nket*ncd] (read)
 *   Jbra, Jket DEVICE double, same shapes, ACCUMULATED (the caller zeroes
 *              them); either may be NULL (not computed), and then its
 *              density may be NULL too.  Accumulation uses atomic adds: the
 *              order of the sums, and so the last bits, vary between calls.
 * Same other arguments, limits and workspace (mdx_eri_workspace_size) as
 * mdx_eri_batch.  Classes whose default kernel is a single-primitive or
 * 3-centre matrix-core variant run on the general matrix-core kernel.
 * Errors as mdx_eri_batch; MDX_EINVAL also for a J without its density.  An
 * empty batch (nbra or nket 0) reads and writes nothing and returns MDX_OK.
 */
mdx_status mdx_eri_digest_batch(mdx_ctx *ctx, const mdx_shells *shells, int ncentre, int32_t nbra,
                                const int32_t *bra, int32_t nket, const int32_t *ket, int flags,
                                const double *Dbra, const double *Dket, double *Jbra, double *Jket,
                                void *ws, size_t ws_bytes, mdx_stream_t stream);

/*
 * Centre derivatives contracted with an adjoint (backward pass of
 * mdx_eri_batch; the paper has no derivatives -- they follow from
 * differentiating Eq. (1): d/dA_i phi_a = 2 zeta_a phi_{a+1_i} - a_i phi_{a-1_i}).
 *   adjoint DEVICE double, same layout and size as mdx_eri_batch's out
 *   grad    DEVICE double[nbra*12*nket]:
 *       grad[ij + nbra*(3*X + i + 12*kl)] = sum_{ab,cd} W[ij,ab,cd,kl] d(ab|cd)/dX_i
 *       X = 0..3 for the centres of a, b, c, d; i = x, y, z.  A slot whose
 *       function is absent (3-/2-centre) is written as 0.  Centres that
 *       coincide are still reported separately; the caller sums them.
 * Same other arguments and workspace query as mdx_eri_batch
 * (mdx_eri_grad_workspace_size).  Limits: each side whose centres are
 * differentiated (both pairs of a 4-centre class, the ket pair of a
 * 3-centre class, the lower-l function of a 2-centre class) of total order
 * l_a + l_b <= 6; the other side of order <= 6; at most 64 functions per
 * side (so (ff|ff) spherical, not Cartesian); MDX_EUNSUPPORTED beyond.  The
 * call copies host tables and is refused on a stream under graph capture.
 */
size_t mdx_eri_grad_workspace_size(mdx_ctx *ctx, const mdx_shells *shells, int ncentre,
                                   int32_t nbra, const int32_t *bra, int32_t nket,
                                   const int32_t *ket, int flags);
mdx_status mdx_eri_grad_batch(mdx_ctx *ctx, const mdx_shells *shells, int ncentre, int32_t nbra,
                              const int32_t *bra, int32_t nket, const int32_t *ket, int flags,
                              const double *adjoint, double *grad, void *ws, size_t ws_bytes,
                              mdx_stream_t stream);

/*
 * Overlap and kinetic-energy integrals of npair shell pairs of one class
 * (pairs[2i] = a, pairs[2i+1] = b, the same (l_a, l_b) for all) -- the
 * 1-particle integrals of Sec. 2.1: the 1-D overlaps of Eq. (8) from the E
 * coefficients of Eqs. (10)-(11) and (14), and
 *   T_ab = -1/2 <a| nabla^2 |b>
 * from the same 1-D overlaps with the ket's exponent raised and lowered by 2.
 * The paper assigns one pair to one SIMD lane.
 *   pairs HOST int32[2*npair].
 *   S, T  DEVICE double, [ij, ab] column-major: S[ij + npair*ab], ab = a*nb + b,
 *         nb = functions of shell b; either may be NULL (not computed).
 *   ws    DEVICE, at least mdx_one_body_workspace_size bytes, 256-byte aligned.
 *   flags MDX_SPHERICAL or MDX_CARTESIAN.
 * Shells with l <= 3 run one shell pair per lane; larger ones one pair per
 * wave (lanes over the Cartesian function pairs).
 * Limits: l_a, l_b <= 6 (MDX_EUNSUPPORTED otherwise).  Errors: MDX_EINVAL for
 * bad arguments, shell indices or mixed classes; MDX_EWORKSPACE for a short
 * workspace; MDX_EDEVICE for a HIP error.  The size query returns 0 on any
 * error (mdx_last_error says why).  The call copies its pair records from
 * host memory (MDX_EINVAL on a stream under graph capture; the prepared form,
 * mdx_one_body_prepare / mdx_one_body_run, copies them once).
 */
size_t mdx_one_body_workspace_size(mdx_ctx *ctx, const mdx_shells *shells, int32_t npair, const int32_t *pairs,
                                   int flags);
mdx_status mdx_one_body_batch(mdx_ctx *ctx, const mdx_shells *shells, int32_t npair, const int32_t *pairs,
                              int flags, double *S, double *T, void *ws, size_t ws_bytes, mdx_stream_t stream);

/*
 * 1-particle Coulomb (nuclear attraction) integrals of npair shell pairs of
 * one class in the field of ncharge point charges,
 *   V_ab = - sum_I q_I <a| 1/|r - I| |b>        (Eqs. (24), (26), (30), (34))
 * with the sum over charges taken before the Hermite-to-AO transform
 * (Eq. (37), Sec. 2.2.4): per primitive pair the kernel sums the charges'
 * Hermite integrals [r]_I^(0), then transforms that sum once.
 *   pairs   HOST int32[2*npair], as mdx_one_body_batch.
 *   charges DEVICE double[4*ncharge]: x, y, z (bohr), q of charge I at
 *           charges[4I .. 4I+3].  ncharge = 0 gives V = 0.
 *   V       DEVICE double, [ij, ab] column-major: V[ij + npair*ab].
 *   ws      DEVICE, at least mdx_nuclear_workspace_size bytes (the pair
 *           records), 256-byte aligned.
 *   flags   MDX_SPHERICAL or MDX_CARTESIAN.
 * Classes with l_a + l_b <= 6 run one shell pair per lane.  Larger classes
 * run one shell pair per wave, the lanes sharing the Hermite table of order
 * l_a + l_b by columns (u, v) of it.
 * Limits: l_a, l_b <= 6.  Errors: MDX_EINVAL for
 * bad arguments, shell indices, mixed classes, a negative charge count or a
 * null charge array with ncharge > 0; MDX_EWORKSPACE for a short workspace;
 * MDX_EDEVICE for a HIP error.  The size query returns 0 on any error.
 * Like mdx_one_body_batch, the call copies host tables and is refused on a
 * stream under graph capture (prepared form: mdx_nuclear_prepare / run).
 */
size_t mdx_nuclear_workspace_size(mdx_ctx *ctx, const mdx_shells *shells, int32_t npair, const int32_t *pairs,
                                  int32_t ncharge, int flags);
mdx_status mdx_nuclear_batch(mdx_ctx *ctx, const mdx_shells *shells, int32_t npair, const int32_t *pairs,
                             int32_t ncharge, const double *charges, int flags, double *V, void *ws,
                             size_t ws_bytes, mdx_stream_t stream);

/*
 * Schwarz factors Q_ij = sqrt(max_ab |(ab|ab)|) of npair shell pairs of one
 * class (pairs[2i], pairs[2i+1], same (l_a, l_b) for all), from the diagonal
 * 4-centre shellsets (ab|ab) computed by the integral kernels.  |(ab|cd)| <=
 * Q_ab Q_cd (Cauchy-Schwarz for the Coulomb metric), so a quartet with
 * Q_ab Q_cd below a threshold can be skipped -- the screening of batches by
 * sorted factors that Sec. 3.1 describes.
 *   Q DEVICE double[npair]; ws DEVICE, at least mdx_schwarz_workspace_size
 *   bytes, 256-byte aligned.  flags: MDX_SPHERICAL or MDX_CARTESIAN.
 * Errors as mdx_eri_batch.
 */
size_t mdx_schwarz_workspace_size(mdx_ctx *ctx, const mdx_shells *shells, int32_t npair, const int32_t *pairs,
                                  int flags);
mdx_status mdx_schwarz(mdx_ctx *ctx, const mdx_shells *shells, int32_t npair, const int32_t *pairs, int flags,
                       double *Q, void *ws, size_t ws_bytes, mdx_stream_t stream);

/*
 * Prepared batches: the call above planned once, run many times.  Preparing
 * validates the batch exactly as the plain call does (same arguments, flags,
 * limits and errors), chooses its kernels (mdx_set_variant overrides in force
 * at preparation apply) and copies its index tables to device memory owned by
 * the batch (the only allocation; freed by mdx_batch_destroy).  A run then
 * enqueues kernel launches only: no host tables are copied and nothing is
 * allocated, so a run can be captured into a HIP graph (and replayed), and its
 * host cost does not grow with the number of pairs.
 *   Runs take the same shell table as the preparation (same metadata, checked:
 *   MDX_EINVAL otherwise); its DEVICE arrays -- centres, exponents,
 *   coefficients -- are read at run time and may hold new values.
 *   ws: DEVICE, at least mdx_batch_workspace_size bytes, 256-byte aligned
 *   (pair data written by the run; one-body and lane-kernel nuclear batches
 *   need none and accept NULL).  Outputs and layouts as the plain calls;
 *   mdx_batch_output_size gives the doubles of each output array.
 *   mdx_nuclear_prepare fixes the charge count; the charges' positions and
 *   values are read from the DEVICE array given to each run.
 * Runs of one batch may be enqueued on different streams only if they use
 * different workspaces.  A batch refers to its context, which must outlive
 * it.  Errors: as the plain calls, plus MDX_ENOMEM if the table allocation
 * fails and MDX_EINVAL for a batch of another kind (e.g. an ERI batch passed
 * to mdx_one_body_run).  On failure *out is NULL.
 */
typedef struct mdx_batch mdx_batch;
/* 2-electron batch: the arguments of mdx_eri_batch (flags MDX_SPHERICAL or
 * MDX_CARTESIAN, optionally | MDX_PAIRED); out as mdx_eri_batch's */
mdx_status mdx_eri_prepare(mdx_ctx *ctx, const mdx_shells *shells, int ncentre, int32_t nbra,
                           const int32_t *bra, int32_t nket, const int32_t *ket, int flags,
                           mdx_batch **out);
mdx_status mdx_eri_run(const mdx_batch *batch, const mdx_shells *shells, double *out, void *ws,
                       size_t ws_bytes, mdx_stream_t stream);
/* overlap and kinetic energy: the pairs and flags of mdx_one_body_batch;
 * S, T as there (either may be NULL) */
mdx_status mdx_one_body_prepare(mdx_ctx *ctx, const mdx_shells *shells, int32_t npair, const int32_t *pairs,
                                int flags, mdx_batch **out);
mdx_status mdx_one_body_run(const mdx_batch *batch, const mdx_shells *shells, double *S, double *T, void *ws,
                            size_t ws_bytes, mdx_stream_t stream);
/* 1-particle Coulomb: the pairs, charge count and flags of mdx_nuclear_batch;
 * charges (DEVICE double[4*ncharge]) and V as there */
mdx_status mdx_nuclear_prepare(mdx_ctx *ctx, const mdx_shells *shells, int32_t npair, const int32_t *pairs,
                               int32_t ncharge, int flags, mdx_batch **out);
mdx_status mdx_nuclear_run(const mdx_batch *batch, const mdx_shells *shells, const double *charges, double *V,
                           void *ws, size_t ws_bytes, mdx_stream_t stream);
/* workspace bytes of a run (0 for a NULL batch); doubles of each output array */
size_t mdx_batch_workspace_size(const mdx_batch *batch);
int64_t mdx_batch_output_size(const mdx_batch *batch);
/* frees the batch and its device tables (NULL is ignored) */
void mdx_batch_destroy(mdx_batch *batch);

/*
 * Multi-class plans (batch-level screening of Sec. 3.1; mixed classes in one
 * launch).  A plan holds host-side planning and device-side index tables; it
 * is built once and executed many times.
 *
 * Each batch is one class (same rules as mdx_eri_batch) with a ragged
 * outer product: for ket pair kl only the first bra_count[kl] bra pairs are
 * computed (bra_count NULL = all).  Sorting bra pairs by decreasing Schwarz
 * factor turns a Schwarz screen into such prefixes.  Output of batch b:
 *   out[out_offset + base_kl + ij + n_kl*(ab + nab*cd)],
 *   n_kl = bra_count[kl], base_kl = nab*ncd*sum_{k<kl} n_k.
 * All arrays in the descriptor are HOST arrays, copied by mdx_plan_create.
 */
typedef struct {
    int ncentre;
    int32_t nbra;
    const int32_t *bra;
    int32_t nket;
    const int32_t *ket;
    const int32_t *bra_count;
    int64_t out_offset;
} mdx_batch_desc;

typedef struct mdx_plan mdx_plan;

/* flags: MDX_SPHERICAL/MDX_CARTESIAN | MDX_FUSED | MDX_DIGEST (mdx_plan_digest
 * below).  Without MDX_FUSED the plan
 * issues one plain launch per batch (and two pair-data launches per batch);
 * with it, execution is one captured graph: the pair data of all batches,
 * then one persistent work-queue launch per kernel instance, each serving
 * every batch that uses that instance.
 * Batches are taken in kernel orientation as given (no bra/ket swap): give
 * the pair with the larger total angular momentum as the bra (l_a + l_b >=
 * l_c + l_d); other orientations can fail with MDX_EUNSUPPORTED.
 * mdx_plan_create allocates the plan's device index tables (the only
 * allocation of the library outside mdx_create; freed by mdx_plan_destroy);
 * with MDX_FUSED it also creates the streams and events used to capture the
 * graph.  Executions of one plan must not overlap in time (they share its
 * work counters). */
mdx_status mdx_plan_create(mdx_ctx *ctx, const mdx_shells *shells, int nbatch,
                           const mdx_batch_desc *batches, int flags, mdx_plan **out);
size_t mdx_plan_workspace_size(const mdx_plan *plan);
/* total number of doubles the plan writes (max over batches of offset+size) */
int64_t mdx_plan_output_size(const mdx_plan *plan);
/* shells must describe the same basis (same metadata) as at creation, else
 * MDX_EINVAL; its device arrays may hold new values.  out: DEVICE double of at
 * least mdx_plan_output_size doubles.  With MDX_FUSED the graph keeps the
 * device pointers of shells, out and ws: changing any of them rebuilds the
 * graph (which synchronises the stream once); the stream may change freely. */
mdx_status mdx_plan_execute(mdx_plan *plan, const mdx_shells *shells, double *out, void *ws,
                            size_t ws_bytes, mdx_stream_t stream);

/*
 * Digestion over a screened plan (the "consume" use of Sec. 3.1: a Coulomb
 * build over a screened molecule never writes its integrals).  A plan created
 * with MDX_DIGEST (matrix-core classes then run their first, general, kernel
 * shape) is run by this call instead of mdx_plan_execute; with MDX_FUSED as
 * well it runs as one graph of persistent digesting kernels, whose batch
 * descriptors hold the blocks' pointers (new pointers rebuild the graph, which
 * synchronises the stream once).
 * Batch b, with bra pairs ij < nbra_b, ket pairs kl < nket_b and ket pair kl
 * taking the bra prefix ij < n_kl (bra_count), contributes
 *   Jbra[ij + nbra_b*ab] += sum_{kl: ij < n_kl} sum_cd (ab|cd) Dket[kl + nket_b*cd]
 *   Jket[kl + nket_b*cd] += sum_{ij < n_kl} sum_ab (ab|cd) Dbra[ij + nbra_b*ab]
 * with the DEVICE pointers of blocks[b] (a HOST array of nbatch entries);
 * J blocks are ACCUMULATED with atomic adds (the caller zeroes them; several
 * batches may share one), either may be NULL (not computed), and a J needs
 * the other side's density.  With canonical pair lists and a screen these are
 * the two Coulomb contributions of each computed quartet; symmetry factors
 * and the gather/scatter of D and J between AO and pair-blocked layouts are
 * the caller's.  Errors as mdx_plan_execute, plus MDX_EINVAL for a plan made
 * without MDX_DIGEST or a J without its density.
 */
typedef struct {
    const double *Dbra, *Dket;
    double *Jbra, *Jket;
} mdx_digest_block;
/* blocks: HOST array of one mdx_digest_block per batch of the plan */
mdx_status mdx_plan_digest(mdx_plan *plan, const mdx_shells *shells, const mdx_digest_block *blocks, void *ws,
                           size_t ws_bytes, mdx_stream_t stream);
/* frees the plan, its tables, streams and graph */
void mdx_plan_destroy(mdx_plan *plan);

/*
 * Profiling hook.  With nevents >= 2, every integral-kernel launch made
 * through this context records hipEventRecord(events[2i]) just before and
 * hipEventRecord(events[2i+1]) just after the kernel on the call's stream,
 * i = (launch count since this call) mod (nevents/2).  The events are
 * hipEvent_t handles created and owned by the caller.  nevents = 0 (or a null
 * array) switches the hook off.  Returns MDX_EINVAL for a null context or an
 * odd/negative count.
 */
mdx_status mdx_set_profile_events(mdx_ctx *ctx, void *const *events, int nevents);

/*
 * Kernel variant for one class (used by the autotuner).  The class is given
 * by ncentre and the caller's l values (lb / ld ignored for a single-function
 * side) plus MDX_CARTESIAN in flags.  variant 0 = register (one lane per
 * shellset) kernel; 1, 2, ... = matrix-core kernel tile shapes; -1 = back to
 * the default choice.  With MDX_GRADIENT in flags the choice applies to the
 * backward kernel of mdx_eri_grad_batch instead (tile shapes 1, 2, ...; a
 * pass whose kernel has fewer shapes uses shape 1).  Returns MDX_EINVAL if
 * the class has no such variant.  Affects calls and plans made afterwards
 * through this context.
 */
mdx_status mdx_set_variant(mdx_ctx *ctx, int ncentre, int la, int lb, int lc, int ld, int flags,
                           int variant);

#ifdef __cplusplus
}
#endif

#endif /* MDX_H */
