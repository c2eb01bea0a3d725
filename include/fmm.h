/*
 * fmm.h -- C ABI of the MI355X (gfx950) adaptive point-charge Laplace FMM.
 *
 * The library evaluates, for N point charges q_j at positions r_j,
 *
 *     u(r_i)   = -1/(4 pi) * sum_{j : |r_i - r_j| > 0} q_j / |r_i - r_j|
 *     E(r_i)   = -grad u(r_i)
 *
 * (kernel and density of eqs. 2-3 of Kraft et al., "jaxFMM: An Adaptive,
 * GPU-Parallel Implementation of the Fast Multipole Method in JAX",
 * arXiv 2511.15269), approximately, by the paper's fast multipole method:
 * a balanced 2^s-tree built by median splits (Sec. II.A), cross-level
 * interaction lists from the admissibility test R + theta r <= theta d
 * (eq. 4, Sec. II.B), real solid-harmonic expansions of order p
 * (Sec. II.C, App. A) and rotation-based O(p^3) M2M/M2L/L2L operators
 * computed per interaction (Sec. II.D, App. B).  Pairs at distance 0
 * contribute nothing.  Every pass runs as hand-written HIP kernels.
 *
 * Conventions for every entry point:
 *   - Pointers documented "device" must be device memory of the current
 *     HIP device; "host" pointers are ordinary host memory.
 *   - `stream` is a hipStream_t (NULL = the legacy default stream); all
 *     device work is enqueued on it.  fmm_plan_create and the fmm_plan_get_*
 *     calls synchronise that stream; fmm_evaluate does not.
 *   - Every call returns an fmm_status.  On any error no output buffer has
 *     been written, the plan (if any) is unchanged and usable, and
 *     fmm_last_error() returns a message for the calling thread.
 *   - No C++ exception crosses this boundary.
 */
#ifndef FMM_H_
#define FMM_H_

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define FMM_ABI_VERSION 2

typedef enum {
  FMM_OK = 0,
  FMM_EINVAL = 1,  /* bad argument: parameter out of range, NULL pointer,
                      non-finite position, size mismatch                  */
  FMM_ENOMEM = 2,  /* device allocation failed                             */
  FMM_EDEVICE = 3, /* HIP runtime error (launch, copy, wrong device)       */
  FMM_ENOTSUP = 4, /* valid request this build does not implement
                      (e.g. an expansion order without compiled kernels)   */
  FMM_ESTATE = 5   /* plan in a state that does not allow the call         */
} fmm_status;

typedef enum { FMM_FP64 = 0, FMM_FP32 = 1 } fmm_precision;

typedef enum { FMM_TIE_SOURCE = 0, FMM_TIE_TARGET = 1 } fmm_tie;

/* Interaction lists (Sec. II.B).  Cross-level: the level march that
 * refines one side per step, so a source box of level l may pair with a
 * target box of level l or l+1 (the paper's default).  Same-level: the
 * enumerated procedure at the start of Sec. II.B, boxes compared only with
 * boxes of their own level (every step refines both sides); for one point
 * set these lists are symmetric. */
typedef enum { FMM_LISTS_CROSS_LEVEL = 0, FMM_LISTS_SAME_LEVEL = 1 } fmm_lists;

/* Method parameters (Sec. II.A-II.B; Table II). */
typedef struct {
  int p;            /* expansion order p of Sec. II.C (degrees 0..p);
                       FMM_MIN_ORDER <= p <= FMM_MAX_ORDER are compiled;
                       p < 0 is FMM_EINVAL, other p FMM_ENOTSUP            */
  int leaf_max;     /* N_max: levels are added until every box holds at
                       most leaf_max points; must be >= 2^splits            */
  int splits;       /* s: binary splits per level, 1..3 (2^s children)   */
  double theta;     /* separation parameter of eq. 4, 0 < theta < 1        */
  int max_depth;    /* cap on the number of levels L, 0..16                */
  int precision;    /* fmm_precision of charges, expansions and outputs    */
  int tie_refine;   /* fmm_tie: side refined when the level-mean radii of
                       source and target level are equal (Sec. II.B, the
                       enumerated rule 2 says source)                      */
  int max_rhs;      /* largest number of charge vectors per evaluate, >= 1 */
  int lists;        /* fmm_lists: cross-level (0) or same-level (1)        */
} fmm_params;

/* Orders with compiled kernels.  Each translation keeps one interaction's
 * (p+1)^2 coefficients in one lane's registers, fully unrolled per order;
 * above p = 10 that state no longer fits a lane (the FP64 M2L already
 * spills a little at p = 10).  p = 0 (monopoles only) is not built.       */
#define FMM_MIN_ORDER 1
#define FMM_MAX_ORDER 10

typedef struct fmm_plan fmm_plan;

/* Sizes of a built plan. */
typedef struct {
  int64_t n;            /* points                                          */
  int32_t depth;        /* L (leaf level)                                  */
  int32_t splits;       /* s                                               */
  int64_t nbox;         /* boxes over all levels, sum_l 2^{s l}            */
  int64_t nleaf;        /* 2^{s L}                                         */
  int64_t n_m2l;        /* multipole-to-local pairs (all levels)           */
  int64_t n_p2p;        /* leaf-leaf direct pairs (including self pairs)   */
  int64_t p2p_interactions; /* sum over direct pairs of |src| * |tgt|     */
  int64_t device_bytes; /* device memory held by the plan (all of it)      */
  int64_t workspace_bytes; /* of which the evaluation workspace (see
                              fmm_plan_workspace_bytes)                    */
  int64_t p2p_items;    /* near-field work items (direct lists longer than
                           about 2^16 interactions are split into several) */
} fmm_plan_info;

/* Source of the plan's device memory (fmm_plan_create_ex).  alloc returns
 * `bytes` of device memory of the current device, aligned to 256 bytes, or
 * NULL on failure; free releases a block alloc returned.  `stream` is the
 * stream given to the create call (a hipStream_t): the plan uses the
 * memory on it, and frees nothing before its work there is done.  Both
 * callbacks run on the calling thread, inside the create call (the tree and
 * list build also takes its temporaries from alloc and returns them before
 * the call ends), inside fmm_plan_autotune (temporary outputs) and inside
 * fmm_plan_destroy; ctx is passed through.  The per-process operator
 * tables (a few hundred KB per order and precision, shared by all plans)
 * are not plan memory and come from hipMalloc.                           */
typedef struct {
  void* (*alloc)(void* ctx, size_t bytes, void* stream);
  void (*free)(void* ctx, void* ptr, void* stream);
  void* ctx;
} fmm_allocator;

/* Version of this ABI (FMM_ABI_VERSION of the built library). */
int fmm_abi_version(void);

/* Message describing the last error of the calling thread ("" if none). */
const char* fmm_last_error(void);

/* Build the tree, box geometry and interaction lists of `n` points.
 *   pos    device, double[n][3] (x, y, z of point i at pos[3i..3i+2]), read
 *          only; the plan keeps its own copy, so the caller may free or
 *          overwrite pos after the call returns.
 *   n      1 <= n < 2^31.
 *   prm    host, parameters (copied).
 *   out    host, receives the new plan (owned by the caller; free it with
 *          fmm_plan_destroy).  Untouched on error.
 * Tree: Sec. II.A (median split along the longest axis; the lower child
 * takes ceil(n/2) points ordered by (coordinate, input index); the first
 * axis wins ties of the extent).  Geometry: centre = midpoint of the tight
 * bounding box of a box's points, radius = half its diagonal.  Lists: the
 * cross-level level march of Sec. II.B; a pair at distance 0 is never
 * admissible.  Errors: FMM_EINVAL (parameters, n, NULL, non-finite
 * position), FMM_ENOTSUP (p outside FMM_MIN_ORDER..FMM_MAX_ORDER),
 * FMM_ENOMEM, FMM_EDEVICE. */
fmm_status fmm_plan_create(const double* pos, int64_t n, const fmm_params* prm,
                           void* stream, fmm_plan** out);

/* Plan flag (fmm_plan_create_ex, fmm_multi_plan_create_ex,
 * fmm_plan_create_st): hold no evaluation workspace.  Such a plan keeps only
 * its tree and lists; it is evaluated with fmm_evaluate_noalloc, and
 * fmm_evaluate, fmm_evaluate_transposed, fmm_adjoint, fmm_graph_create and
 * fmm_plan_autotune return FMM_ESTATE on it. */
#define FMM_PLAN_NO_WORKSPACE 1u

/* fmm_plan_create with the plan's device memory taken from `allocator`
 * (NULL: hipMalloc/hipFree).  flags: 0 or FMM_PLAN_NO_WORKSPACE.  Errors: as
 * fmm_plan_create, plus FMM_EINVAL for an allocator without both
 * callbacks, other flags or a block not aligned to 256 bytes, and
 * FMM_ENOMEM when alloc returns NULL (everything allocated so far is
 * returned through free). */
fmm_status fmm_plan_create_ex(const double* pos, int64_t n, const fmm_params* prm,
                              const fmm_allocator* allocator, unsigned flags, void* stream,
                              fmm_plan** out);

/* A plan with separate sources and targets (Sec. II.B, the generalisation
 * to distinct source and target points, used by the paper's inverse-design
 * example in Sec. III.B): potentials and fields of charges at the ns points
 * src are evaluated at the nt points tgt.
 *   src    device, double[ns][3], the charge positions (read only, copied)
 *   tgt    device, double[nt][3], the evaluation points (read only, copied)
 * Each point set gets its own tree (Sec. II.A, same parameters; the depths
 * may differ).  The lists come from the cross-level level march between
 * the two trees (Sec. II.B): each step refines the side whose level has the
 * larger mean box radius (the side tie_refine names on equal means), a side
 * that has reached its leaves is no longer refined, and the march starts
 * by testing the pair of roots (two point sets far apart interact through
 * one M2L pair).  A target may coincide with a source: such pairs
 * contribute nothing.  On this plan fmm_evaluate takes q as [nrhs][ns] and
 * writes pot [nrhs][nt] and field [nrhs][nt][3]; fmm_evaluate_transposed
 * takes [nrhs][nt] and writes [nrhs][ns] (the adjoint map, from the
 * targets back to the sources); fmm_adjoint takes g [nrhs][nt], writes
 * grad_q [nrhs][ns] and needs grad_x = NULL (FMM_ENOTSUP otherwise).
 * Every charge vector is evaluated in its own pass (no 32-vector form).
 * fmm_plan_get_info reports n = ns + nt and the boxes and leaves of both
 * trees: the source tree's boxes and leaves come first, then the target
 * tree's; fmm_plan_get_tree's perm gives input indices within each point
 * set, fmm_plan_get_lists global box and leaf ids.  allocator and flags as
 * for fmm_plan_create_ex.  Errors: as fmm_plan_create_ex (ns and nt are
 * each checked as n; ns + nt < 2^31). */
fmm_status fmm_plan_create_st(const double* src, int64_t ns, const double* tgt, int64_t nt,
                              const fmm_params* prm, const fmm_allocator* allocator,
                              unsigned flags, void* stream, fmm_plan** out);

/* Device bytes of the evaluation workspace of a plan of n points with
 * these parameters (fmm_plan_create): the buffers every evaluation writes
 * and reads -- leaf-ordered source records (32 n), multipole and local
 * expansions (2 x nbox x (p+1)^2 values), the near field (4 n values), the
 * adjoint's field (3 n values) and, for FP32 plans with max_rhs > 1, their
 * 32-vector copies -- each rounded up to 256 bytes; the plan takes it as one
 * allocation.  Exact: nbox = sum_{l<=L} 2^{s l} follows from n, leaf_max,
 * splits and max_depth alone.  The tree and the interaction lists (and the
 * batched form's M2L partial rows, one row per work item), whose size
 * depends on where the points are, come on top: fmm_plan_get_info reports
 * both figures of a built plan.  Host only: needs no device, allocates
 * nothing.  Errors: FMM_EINVAL (NULL, n or parameters), FMM_ENOTSUP (p). */
fmm_status fmm_plan_workspace_bytes(int64_t n, const fmm_params* prm, int64_t* bytes);

/* One plan over several independent problems of uneven sizes (beyond the
 * paper, which treats one system per hierarchy; each problem's tree and
 * lists follow Sec. II.A-II.B unchanged).
 *   pos      device, double[offsets[nprob]][3]: the points of problem k are
 *            rows offsets[k] .. offsets[k+1]-1.  Read only, copied.
 *   offsets  host, int64[nprob+1], offsets[0] = 0, strictly increasing
 *            (every problem has at least one point); total below 2^31.
 *   nprob    number of problems, >= 1.
 * Each problem gets its own tree and lists, exactly those fmm_plan_create
 * would build for its points alone (depths may differ); problems never
 * interact.  The plan then behaves as a plan of offsets[nprob] points:
 * every call below takes charges and returns potentials/fields for the
 * concatenated points, and each evaluation stage covers all problems in
 * one launch (M2M and L2L: one launch per level step, the deepest tree
 * setting the count).  fmm_plan_get_tree/get_lists report global box and
 * leaf numbering: problem k's boxes follow those of problems 0..k-1.
 * Errors: as fmm_plan_create, plus FMM_EINVAL for bad offsets. */
fmm_status fmm_multi_plan_create(const double* pos, const int64_t* offsets, int nprob,
                                 const fmm_params* prm, void* stream, fmm_plan** out);

/* fmm_multi_plan_create with device memory from `allocator` (as
 * fmm_plan_create_ex). */
fmm_status fmm_multi_plan_create_ex(const double* pos, const int64_t* offsets, int nprob,
                                    const fmm_params* prm, const fmm_allocator* allocator,
                                    unsigned flags, void* stream, fmm_plan** out);

/* Sizes of the plan (host struct, written on success). */
fmm_status fmm_plan_get_info(const fmm_plan* plan, fmm_plan_info* info);

/* Evaluate potentials (and fields) for `nrhs` charge vectors.
 *   q      device, [nrhs][n] of double (FMM_FP64) or float (FMM_FP32),
 *          in input point order.
 *   pot    device, [nrhs][n], same type: u at every input point.
 *   field  device, [nrhs][n][3], same type: -grad u; may be NULL (then
 *          only potentials are computed).
 * 1 <= nrhs <= max_rhs of the plan.  Enqueued on `stream`; buffers must
 * stay valid until the stream has executed it.  Calls on one plan must be
 * serialised by the caller (they share the plan's expansion workspace).
 * Errors: FMM_EINVAL (NULL q or pot, nrhs out of range), FMM_EDEVICE. */
fmm_status fmm_evaluate(fmm_plan* plan, const void* q, int nrhs, void* pot,
                        void* field, void* stream);

/* fmm_evaluate for callers that cannot allocate device memory (code under
 * HIP graph capture, tight serving loops, harnesses that forbid it): the
 * evaluation workspace of each pass -- source records, multipole and local
 * expansions, near field -- comes from one device array of
 * FMM_NOALLOC_MAX_BYTES that the library holds on every device it runs on
 * until the process ends, shared by all plans, instead of from the plan.
 * Nothing is allocated (the array's address is looked up once per device,
 * on the first call there).  The plan may be one created with
 * FMM_PLAN_NO_WORKSPACE.  Arguments, results and errors as fmm_evaluate;
 * charge vectors are evaluated one pass each; stage profiling is not
 * recorded.  Plans whose pass needs more than FMM_NOALLOC_MAX_BYTES
 * (32 n + 2 nbox (p+1)^2 e + 4 n e bytes, e = 8 for FP64 and 4 for FP32,
 * each part rounded up to 256) are rejected with FMM_EINVAL.  Every call on
 * a device uses the same array: calls that overlap on one device (other
 * streams, other threads) race and must be serialised by the caller.  Each
 * pass writes every part of the array it reads before reading it, so the
 * contents a previous call left do not matter. */
#define FMM_NOALLOC_MAX_BYTES (128u << 20)
fmm_status fmm_evaluate_noalloc(fmm_plan* plan, const void* q, int nrhs, void* pot,
                                void* field, void* stream);

/* Transposed evaluation: the adjoint operator G-hat^T of fmm_evaluate's
 * linear map q -> u-hat (tree, lists and centres frozen), i.e. the same FMM
 * run over the transposed interaction lists (every M2L and P2P pair
 * reversed).  Needed because the cross-level lists of Sec. II.B pair a
 * source level with a different target level, so G-hat is not symmetric;
 * the truncated two-centre kernel with the square truncation n, k <= p is
 * symmetric under exchanging source and target with the shift reversed
 * (App. B.3 operators), which makes the transposed-list FMM the exact
 * transpose.  Arguments and errors as for fmm_evaluate. */
fmm_status fmm_evaluate_transposed(fmm_plan* plan, const void* q, int nrhs,
                                   void* pot, void* field, void* stream);

/* Backward pass of u-hat = FMM(q, x) with frozen hierarchy, for upstream
 * gradients g = dL/du-hat (autodiff of the evaluation, Sec. III.B):
 *   grad_q = G-hat^T g
 *   grad_x = g * grad u-hat(x) + q * grad (G-hat^T g)(x)   (per point, [n][3])
 *   q          device [nrhs][n]: the charges of the forward pass
 *   g          device [nrhs][n]
 *   field_fwd  device [nrhs][n][3]: the field (-grad u-hat) of the forward pass
 *   grad_q     device [nrhs][n] (written)
 *   grad_x     device [nrhs][n][3] or NULL (then q and field_fwd may be NULL)
 * For E = 1/2 q^T u-hat use g = q/2 and add u-hat/2 to grad_q.  Types follow
 * the plan's precision.  Errors: FMM_EINVAL, FMM_EDEVICE. */
fmm_status fmm_adjoint(fmm_plan* plan, const void* q, const void* g, int nrhs,
                       const void* field_fwd, void* grad_q, void* grad_x,
                       void* stream);

/* Copy the tree to host buffers (any may be NULL):
 *   perm       int64[n]: leaf-ordered slot i holds input point perm[i]
 *   leaf_start int64[nleaf+1]: leaf j holds slots [leaf_start[j],
 *              leaf_start[j+1]); points inside a leaf by input index
 *   centre     double[nbox][3], radius double[nbox]; box b of level l has
 *              global id (2^{s l} - 1)/(2^s - 1) + b, children of b are
 *              b * 2^s + c. */
fmm_status fmm_plan_get_tree(const fmm_plan* plan, int64_t* perm,
                             int64_t* leaf_start, double* centre,
                             double* radius);

/* Copy the interaction lists to host buffers (any may be NULL), each
 * sorted by (target, source):
 *   m2l_src/m2l_tgt  int64[n_m2l], global box ids
 *   p2p_src/p2p_tgt  int64[n_p2p], leaf indices */
fmm_status fmm_plan_get_lists(const fmm_plan* plan, int64_t* m2l_src,
                              int64_t* m2l_tgt, int64_t* p2p_src,
                              int64_t* p2p_tgt);

/* Direct summation of the potential (and field) at selected points, the
 * reference the paper measures FMM errors against (Sec. III.A; eqs. 1-3):
 *   pos      device, double[n][3], all sources
 *   q        device, [n] double (FMM_FP64) or float (FMM_FP32)
 *   targets  device, int64[ntargets] indices into pos, or NULL for all n
 *            points (then ntargets must equal n); an index outside [0, n)
 *            reads no memory and gives NaN outputs (the indices live on the
 *            device, so they are checked there)
 *   pot      device, [ntargets] of the charge type
 *   field    device, [ntargets][3] (-grad u) or NULL
 * Pairs at distance 0 are skipped.  O(n * ntargets) work, enqueued on
 * `stream`.  Errors: FMM_EINVAL (NULL, sizes, precision), FMM_EDEVICE. */
fmm_status fmm_direct(const double* pos, int64_t n, const void* q, int precision,
                      const int64_t* targets, int64_t ntargets, void* pot,
                      void* field, void* stream);

/* Per-stage timing of evaluations, the breakdown of the paper's Fig. 5
 * (Sec. III.A: sort, mpls, M2M, M2L, L2L, evloc, evdir).  Stage indices:
 *   0 sort (charges to leaf order), 1 P2M, 2 M2M, 3 M2L, 4 L2L,
 *   5 L2P (evloc), 6 P2P (evdir).
 * The P2M kernels also do the sort stage, so its time is counted under
 * P2M and stage 0 holds only the cost of its pair of events.
 * While enabled, every evaluation records a HIP event before and after each
 * stage on its stream.  fmm_plan_read_profile waits for those
 * events, writes the summed milliseconds per stage to
 * stage_ms[FMM_NSTAGES] (host) and the number of evaluated passes to
 * *passes, and clears the record.  Disabling also clears it. */
#define FMM_NSTAGES 7
fmm_status fmm_plan_set_profiling(fmm_plan* plan, int enable);
fmm_status fmm_plan_read_profile(fmm_plan* plan, double* stage_ms,
                                 int64_t* passes);

/* Choose the launch tiles of the single-vector evaluation (fmm_tiles) by
 * timing them on this plan: first the M2L form, the M2M / L2L form (one
 * lane or several waves per translation) and the near field's stream, then
 * the number of source groups of the near-field kernel (1, 2 or 4) together
 * with the number of leaves per wave of P2M and L2P (1, 2, 4 or 8), among
 * the values the plan's largest leaf allows; on plans of the 32-vector form
 * (FP32, max_rhs > 1) also the batched near field's waves per block, timed
 * on passes of max_rhs copies of q.  Every candidate runs one untimed and
 * three timed evaluations of the charges q (device, [n], the plan's
 * precision) on `stream`; the fastest values are stored in the plan
 * and used by every later evaluation (results change only by the summation
 * order inside the near field and the multipole sums).  The chosen groups
 * and leaves per wave are written to *p2p_groups and *leaves_per_wave
 * (host; may be NULL); every chosen value can be read with
 * fmm_plan_get_tiles.  Synchronises `stream`; allocates and frees
 * temporary output buffers.  Errors: FMM_EINVAL (NULL plan or q),
 * FMM_ENOMEM, FMM_EDEVICE. */
fmm_status fmm_plan_autotune(fmm_plan* plan, const void* q, void* stream, int* p2p_groups,
                             int* leaves_per_wave);

/* Launch tiles of the single-vector evaluation, as fmm_plan_autotune
 * chooses them or a caller sets them:
 *   p2p_groups       source groups of the near-field kernel: 1, 2 or 4
 *                    (2 and 4 need leaves of at most 64 / groups points)
 *   leaves_per_wave  leaves per wave of P2M and L2P: 1, 2, 4 or 8 (at most
 *                    64 / value points per leaf)
 *   m2l_waves        waves sharing each M2L translation (Sec. II.D): 1 (one
 *                    lane per translation) or 4, the shared form, which
 *                    exists for FP64 at p = 6, 7 and FP32 at p = 9, 10 and
 *                    is their default.  Both forms give identical results.
 *   chain_waves      waves sharing each M2M and L2L translation: 1 (one
 *                    lane per translation) or 4 (the shared form, built and
 *                    the default for p >= 5).  Identical results.
 *   batch_p2p_waves  waves per block of the 32-vector near field (each
 *                    takes 16 targets of the leaf at a time, the block's
 *                    waves share every staged source chunk): 1, 2, 4 or 8;
 *                    by default set from the plan's largest leaf.  Identical
 *                    results.  Read and set on every plan; used by plans
 *                    with max_rhs > 1 in FP32.
 *   near_stream      2 (default): the near field runs on a second stream
 *                    of the plan beside the far-field chain (M2M, M2L,
 *                    L2L), forked after P2M and joined before L2P; 1: every
 *                    stage on the caller's stream.  Identical results.
 *                    While stage profiling is on, stages run one after
 *                    another on one stream; graphs (fmm_graph_create)
 *                    keep the plan's choice.
 * fmm_plan_set_tiles takes 0 in a field as "the default for this plan" and
 * rejects any other value the plan cannot use (FMM_EINVAL, plan unchanged).
 * fmm_plan_get_tiles writes the values evaluations use (host *tiles).
 * Neither call touches the device. */
typedef struct fmm_tiles {
  int p2p_groups;
  int leaves_per_wave;
  int m2l_waves;
  int chain_waves;
  int near_stream;
  int batch_p2p_waves;
} fmm_tiles;
fmm_status fmm_plan_set_tiles(fmm_plan* plan, const fmm_tiles* tiles);
fmm_status fmm_plan_get_tiles(const fmm_plan* plan, fmm_tiles* tiles);

/* Release the plan and its device memory (NULL is accepted). */
fmm_status fmm_plan_destroy(fmm_plan* plan);

/* A whole evaluation captured once as a HIP graph and replayed with one
 * launch call (the sequence of stage kernels of fmm_evaluate, or of
 * fmm_evaluate_transposed when `transposed` is nonzero, for fixed buffers).
 *   plan   the plan; must outlive the graph and must not be destroyed or
 *          evaluated concurrently with a replay.  Stage profiling is not
 *          recorded inside graphs.
 *   q, pot, field, nrhs   as for fmm_evaluate; the graph keeps these device
 *          addresses: each replay reads q's current contents and rewrites
 *          pot (and field).
 *   out    host, receives the graph (free with fmm_graph_destroy).
 * Nothing runs at creation.  The graph contains kernel launches only; when
 * the plan's near field runs on the second stream (near_stream 2) it is a
 * second branch of the graph, forked after P2M and joined before L2P.
 * Errors: as fmm_evaluate, FMM_EDEVICE if capture or instantiation fails. */
typedef struct fmm_graph fmm_graph;
fmm_status fmm_graph_create(fmm_plan* plan, int transposed, const void* q, int nrhs,
                            void* pot, void* field, fmm_graph** out);

/* Enqueue one replay on `stream`.  Errors: FMM_EINVAL (NULL graph),
 * FMM_EDEVICE. */
fmm_status fmm_graph_launch(fmm_graph* graph, void* stream);

/* Release the graph (NULL is accepted). */
fmm_status fmm_graph_destroy(fmm_graph* graph);

#ifdef __cplusplus
}
#endif

#endif /* FMM_H_ */
