/*
 * fx.h -- C ABI of the MI355X exchange-matrix library (libfx.so).
 *
 * The library builds the Fock exchange matrix of Challacombe & Bock, "An
 * N-Body Solution to the Problem of Fock Exchange", Eq. (6), by the naive
 * hextree traversal of Eqs. (7a-d) with the blocked Almlof-Ahlrichs metric
 * query of Eq. (8), on one AMD Instinct MI355X (gfx950).
 *
 * Conventions shared by every entry point
 *  - Basis: contracted Cartesian Gaussian shells, l = 0 (s), 1 (p), 2 (d).
 *    Functions are numbered shell after shell in the caller's shell order;
 *    the components of a shell follow lexicographic Cartesian order
 *    (p: x, y, z; d: xx, xy, xz, yy, yz, zz).  Every component is
 *    normalised to (phi|phi) = 1.
 *  - K convention (library scale, no -1/2):
 *        K_{mu sig} = sum_{nu, lam} (mu nu|lam sig) P_{nu lam}
 *    summed over the shell quartets (a,b,c,d) that survive the metric query
 *        beta = (||Q_ab||_F * ||Q_cd||_F) * ||P_bc||_F  >  tau,
 *    Q_{mu nu} = (mu nu|mu nu)^{1/2}, ||P_bc||_F the larger of the Frobenius
 *    norms of the (b,c) and (c,b) blocks of P.  The paper's exchange matrix
 *    (factor -1/2, Eq. 6) is obtained with alpha = -0.5 in fx_exchange_ex.
 *    Because block Frobenius norms bound the norms of their sub-blocks (Eq.
 *    8 and the sub-multiplicativity argument after it), the traversal culls
 *    only work whose bound is <= tau, and the computed quartet set is exactly
 *    {q : beta_q > tau}, independent of the tree.
 *  - Matrices P and K are n x n, row-major, FP64, DEVICE memory owned by the
 *    caller, indexed in the caller's function order.
 *  - Every call returns fx_status; arguments are validated before any work
 *    is enqueued; no C++ exception crosses this boundary.  On failure
 *    fx_last_error_message() describes the cause (thread-local).
 *  - hipStream_t is passed as void* so that this header needs no HIP header.
 */
#ifndef FX_H
#define FX_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum fx_status {
    FX_OK = 0,
    FX_ERR_INVALID_ARG = 1,  /* null pointer, bad size, tau < 0 or NaN, ... */
    FX_ERR_UNSUPPORTED = 2,  /* l > 2, more than FX_MAX_PRIM primitives     */
    FX_ERR_OOM = 3,          /* device allocation failed                     */
    FX_ERR_HIP = 4,          /* a HIP runtime call failed                    */
    FX_ERR_INTERNAL = 5
} fx_status;

#define FX_MAX_L 2
#define FX_MAX_PRIM 16

/* Shells, HOST memory, read only during fx_build_quadtree.
 *   l[nshell]        angular momentum 0..2
 *   nprim[nshell]    primitives per shell, 1..FX_MAX_PRIM
 *   center[3*nshell] shell centres in bohr
 *   exps[sum nprim]  primitive exponents (bohr^-2), shell after shell
 *   coefs[sum nprim] weights multiplying NORMALISED primitives; the library
 *                    renormalises each contracted function.                */
typedef struct fx_shells {
    int32_t nshell;
    const int32_t* l;
    const int32_t* nprim;
    const double* center;
    const double* exps;
    const double* coefs;
} fx_shells;

/* Tree options (NULL = defaults).
 *   leaf_max_functions: the ragged bisection of Eq. (1) stops at blocks of
 *     at most this many functions (or a single shell); 0 = default 10, as in
 *     the paper's implementation (Section V: blocks of 10x10 or smaller).
 *     Inside a surviving leaf task the class kernels apply the same Eq. (8)
 *     test to every shell quartet, so K does not depend on this size; 1
 *     continues the traversal itself down to single shells.
 *   ordering: 0 = Hilbert curve on shell centres (Section III, default),
 *             1 = caller order. */
typedef struct fx_tree_opts {
    int32_t leaf_max_functions;
    int32_t ordering;
} fx_tree_opts;

typedef struct fx_tree fx_tree;   /* opaque, immutable after build */

/* Precision of the shell-quartet recursion.
 *   FX_PREC_FP64:  every quartet in FP64.
 *   FX_PREC_MIXED: quartets with beta < fp32_threshold run their VRR/HRR in
 *                  FP32; Boys function, bounds, pair geometry and all
 *                  accumulation into K stay FP64. */
typedef enum fx_precision { FX_PREC_FP64 = 0, FX_PREC_MIXED = 1 } fx_precision;

/* Work scheduling (never changes which quartets are computed, nor K: the
 * per-block reduction is deterministic).
 *   FX_SCHED_BOUND: units ordered by a cost estimate from bounds and counts.
 *   FX_SCHED_MLP:   units ordered by the learned cost model given in
 *                   fx_exchange_opts.costmodel (falls back to BOUND if NULL).
 *   FX_SCHED_NONE:  traversal order. */
typedef enum fx_schedule { FX_SCHED_BOUND = 0, FX_SCHED_MLP = 1, FX_SCHED_NONE = 2 } fx_schedule;

typedef struct fx_costmodel fx_costmodel;

/* Use of the permutational symmetry of the integrals (Section IV, in the
 * form that keeps every K block a gather).  For a symmetric density,
 * (ab|cd) = (dc|ba) gives K_da = K_ad^T, so only the K blocks a <= d (tree
 * order) are built and each also writes its transpose: half the quartets.
 *   FX_SYM_AUTO: the library tests P for bitwise symmetry on the device
 *                (one pass over P) and uses this when it holds;
 *   FX_SYM_OFF:  every K block is built (any P). */
typedef enum fx_symmetry { FX_SYM_AUTO = 0, FX_SYM_OFF = 1 } fx_symmetry;

/* What a surviving leaf task of the traversal computes.
 *   FX_LEAF_SHELL: every shell quartet inside it is tested with the
 *                  shell-level bound of Eq. (8) (default): the computed set
 *                  is exactly {q : beta_q > tau}, independent of the tree;
 *   FX_LEAF_BLOCK: every shell quartet inside it is computed, as the paper's
 *                  implementation evaluates whole leaf blocks (Section V);
 *                  the set then depends on the leaf size. */
typedef enum fx_leaf_screen { FX_LEAF_SHELL = 0, FX_LEAF_BLOCK = 1 } fx_leaf_screen;

/* Options of an exchange call.  Fill with fx_exchange_opts_init() and then
 * change fields: an all-zero struct is NOT the defaults (alpha = 0 would
 * return K = beta*K, and fp32_threshold = 0 would run every quartet in FP64). */
typedef struct fx_exchange_opts {
    int32_t precision;          /* fx_precision, default FX_PREC_FP64        */
    double fp32_threshold;      /* default 1e-5                              */
    int32_t schedule;           /* fx_schedule, default FX_SCHED_BOUND       */
    const fx_costmodel* costmodel;
    double alpha, beta;         /* K <- alpha*K_x + beta*K; default 1, 0     */
    int64_t max_frontier_entries; /* entry capacity of a traversal level; 0 = sized from earlier calls */
    int32_t profile;            /* 1: time every class-kernel launch with HIP events on `stream` (waits) */
    int32_t use_graph;          /* 1: capture the whole call once in a hipGraph and replay the capture on later
                                   calls with the same tree(s), P, K, tau and options */
    int32_t symmetry;           /* fx_symmetry, default FX_SYM_AUTO          */
    int32_t leaf_screen;        /* fx_leaf_screen, default FX_LEAF_SHELL     */
    double tau_ovlp;            /* overlap threshold of Eqs. (3)-(4), default 0 (off): a pair of shells
                                   (or, in the traversal, of blocks) all of whose functions overlap less
                                   than tau_ovlp contributes nothing.  Unlike tau this drops work the
                                   metric query would keep, without a bound on the change of K. */
    int64_t max_workspace_bytes; /* device workspace of a one-system call, in bytes: 0 = the default, 4 GiB
                                   or what 64 K row ranges need if that is more (within 80% of the free
                                   device memory); < 0 = no limit but 80% of the free device memory.  A
                                   traversal that needs more is run over K row ranges (at leaf-block
                                   boundaries) one after another; K does not depend on it.  Below what one
                                   leaf row of K needs the call takes that much (stats.workspace_bytes
                                   tells). */
} fx_exchange_opts;

/* Fill *o with the defaults documented above. */
void fx_exchange_opts_init(fx_exchange_opts* o);

/* Statistics of one fx_exchange_ex call (valid when the call returns). */
#define FX_STATS_MAX_LEVELS 32
typedef struct fx_stats {
    int32_t levels;                              /* tree depth + 1            */
    int64_t frontier[FX_STATS_MAX_LEVELS];       /* surviving tasks per level */
    int64_t leaf_items;                          /* surviving leaf (A,D) pairs */
    int64_t units;                               /* K-block work units        */
    int64_t quartets;                            /* evaluated shell quartets  */
    int64_t quartets_fp32;                       /* of which in FP32          */
    int64_t class_quartets[81];                  /* per (la lb|lc ld), ((la*3+lb)*3+lc)*3+ld */
    double prim_quartets;                        /* primitive quartets        */
    double flops;                                /* algorithmic flops (generated-code count) */
    int32_t chunks;                              /* traversal chunks          */
    int32_t graph_nodes;                         /* graphs launched           */
    /* with opts.profile: per class and precision (index cls*2 + fp32) */
    double class_seconds[162];                   /* summed kernel time (HIP events) */
    int32_t class_launches[162];                 /* launches                   */
    double class_flops[162];                     /* algorithmic flops          */
    int64_t class_prec_quartets[162];            /* computed quartets          */
    double seconds_traversal, seconds_eri, seconds_total; /* host wall clock */
    int64_t quartets_covered;                    /* ordered quartets with beta > tau that K accounts for
                                                    (evaluated ones plus the mirrors they stand for) */
    int32_t symmetric_systems;                   /* systems built on the symmetric path */
    /* Traversal partition (Eqs. 7a-d): sums of |A||B||C||D| (function counts
     * of the four tree nodes) over [0] the surviving leaf tasks, [1] the
     * culled tasks, [2] the tasks skipped because their mirror (D,C,B,A) is
     * traversed (symmetric form).  Every task of the product of the four
     * trees is in exactly one set, so the sum is n^4 per system (modulo
     * 2^64). */
    int64_t partition[3];
    int32_t overflow;                            /* 1: a traversal level exceeded its capacity and the call
                                                    split its K rows and ran them again (K is complete) */
    int64_t workspace_bytes;                     /* device workspace of the call */
    double fp32_beta_sum;                        /* mixed precision: sum of the bounds beta_q (Eq. 8) of the
                                                    quartets evaluated in FP32; with the FP32 unit roundoff
                                                    u = 2^-24 and a per-quartet growth factor c, c*u times
                                                    this bounds the Frobenius change of K a priori */
} fx_stats;

/* Build the basis-function tree for a set of shells: normalisation, shell
 * ordering along a Hilbert curve (Section III), ragged bisection at shell
 * boundaries (Eq. 1), shell-pair Schwarz factors Q and their Frobenius norms
 * at every level of the pair quadtree (Eq. 2).  The handle owns its device
 * memory.  Blocking: returns after the tree is built on `stream`. */
fx_status fx_build_quadtree(const fx_shells* shells, const fx_tree_opts* opts, void* stream,
                            fx_tree** out);

/* K <- K_x(P) with the defaults of fx_exchange_ex (FP64, alpha 1, beta 0).
 * P, K: device, n x n row-major FP64 (n = fx_nbf(tree)), caller order.
 * tau >= 0 (tau = 0 culls only exactly-zero bounds).  K is overwritten; P
 * must not alias K.
 *
 * Asynchronous: the work is enqueued on `stream` and the call returns
 * without waiting for it; P must stay unchanged and K unread until the
 * stream reaches that point.  Every size the traversal produces stays on the
 * device.  Buffers (traversal levels, K-block unit lists) and launch grids
 * are sized from the sizes earlier calls on the same tree needed (with a
 * 25% margin); the first call on a tree learns the traversal sizes in a
 * traversal-only pass, for which it waits.  If a later call needs more than
 * its buffers hold, that call writes NaN into K (and, when it waits for
 * statistics, redoes the work in K row ranges and returns the right K); the
 * next call uses the larger sizes.  Calls on one tree are serialised on the
 * host; the device work of calls on different streams may overlap. */
fx_status fx_exchange(const fx_tree* tree, const double* P, double tau, double* K, void* stream);

/* As fx_exchange with options and statistics.  stats == NULL (and no
 * opts.profile): asynchronous as fx_exchange.  stats != NULL: the call waits
 * for its result, fills *stats, and never returns a NaN K for lack of
 * buffer space (it splits the traversal into K row ranges instead). */
fx_status fx_exchange_ex(const fx_tree* tree, const double* P, double tau, double* K,
                         const fx_exchange_opts* opts, fx_stats* stats, void* stream);

/* Many independent systems in one call: trees[i], P[i], K[i] (host arrays of
 * device pointers), all with the same tau and options.  Every system is
 * traversed, then each class kernel is launched once over the K-block units
 * of all systems (per-unit system descriptors), optionally captured in a
 * hipGraph (opts.use_graph).  Each K[i] equals fx_exchange_ex's result. */
fx_status fx_exchange_batched(const fx_tree* const* trees, const double* const* P, double* const* K,
                              int32_t count, double tau, const fx_exchange_opts* opts,
                              fx_stats* stats, void* stream);

/* Several densities of one system contracted with the same integrals
 * (Eq. 6 for each): K[j] <- K_x(P[j]), j < ndens, ndens in 1..2 (else
 * FX_ERR_UNSUPPORTED).  P, K: host arrays of ndens device pointers to n x n
 * row-major FP64 arrays in caller order; no P may alias a K and the K must be
 * distinct.  The metric query of Eq. (8) uses, for each density block, the
 * largest norm over the densities, so every K[j] contains at least the
 * quartets its own density would select (when all densities are equal,
 * K[j] equals fx_exchange_ex(P[j]): bitwise in FP64, to rounding in mixed
 * precision).  The symmetric path (fx_symmetry) is taken
 * when every density is bitwise symmetric.  Options and stats as in
 * fx_exchange_ex (quartet counts are per quartet, not per density). */
fx_status fx_exchange_multi(const fx_tree* tree, const double* const* P, double* const* K, int32_t ndens,
                            double tau, const fx_exchange_opts* opts, fx_stats* stats, void* stream);

/* For callers that cannot allocate device memory (code under stream
 * capture, serving loops with a fixed memory budget): fx_exchange_ex with
 * every work buffer taken from a device array of the library of
 * fx_noalloc_scratch_bytes() bytes (256 MiB) instead of being allocated;
 * the call allocates nothing (no hipMalloc, no pool allocation).  The
 * traversal capacities are the largest that fit in the array, and an
 * over-large K row block is split as in fx_exchange_ex when stats is given
 * (asynchronous with stats NULL: NaN K if a level does not fit).  Returns
 * FX_ERR_OOM before any work is enqueued when the system's fixed buffers
 * (norm tables, unit lists, the K accumulator when beta != 0) exceed the
 * array, and FX_ERR_INVALID_ARG for opts.use_graph or opts.profile.  Every
 * call on a GPU shares that GPU's array (it keeps the last call's contents;
 * what must start at zero is cleared by each call): calls that overlap on
 * one GPU, on any streams, race and must be serialised by the caller. */
fx_status fx_exchange_noalloc(const fx_tree* tree, const double* P, double tau, double* K,
                              const fx_exchange_opts* opts, fx_stats* stats, void* stream);
size_t fx_noalloc_scratch_bytes(void);

/* Number of basis functions. */
int32_t fx_nbf(const fx_tree* tree);
/* Number of shells. */
int32_t fx_nshell(const fx_tree* tree);
/* perm[i] = caller index of the i-th shell in the tree's (Hilbert) order; host array of nshell. */
fx_status fx_tree_perm(const fx_tree* tree, int32_t* perm);
/* Depth of the tree (number of levels) and nodes per level (host array, may be NULL). */
int32_t fx_tree_levels(const fx_tree* tree, int64_t* nodes_per_level);
/* Copy the shell-pair Schwarz norms ||Q_ab||_F (caller shell order, nshell^2, host). */
fx_status fx_tree_schwarz(const fx_tree* tree, double* Qn_host);
/* Copy the largest |overlap| of the functions of every shell pair (caller shell order, nshell^2, host). */
fx_status fx_tree_overlap(const fx_tree* tree, double* Sm_host);
void fx_tree_free(fx_tree* tree);

/* ---------------------------------------------------------------------------
 * Learned scheduling.  A small MLP (4 -> 64 -> 64 -> 1, FP32, ReLU) predicts
 * the wall time (log2 ns) of one K-block work unit in one class launch from
 * four features: log2 of the class's flops per quartet, log2(nprim_a nprim_d),
 * log10 of the unit's Schwarz row bound, log2(1 + candidate entries).  With
 * FX_SCHED_MLP each class launch dispatches its units heaviest-predicted
 * first (stable 32-bin ordering); FX_SCHED_BOUND uses the bound-only estimate
 * log2(flops * nprim_a nprim_d * entries).  Culling is never affected, and K
 * is bitwise identical under every schedule.
 * ------------------------------------------------------------------------- */
typedef struct fx_task_timings fx_task_timings;   /* (features, log2 ns) samples */

typedef struct fx_train_opts {
    int32_t steps;   /* Adam steps (default 2000)                 */
    int32_t batch;   /* minibatch size (default 8192)             */
    float lr;        /* learning rate (default 3e-3)              */
    uint64_t seed;   /* initialisation and minibatch seed          */
} fx_train_opts;

/* Run one exchange with per-unit timing probes (wall clock of every unit in
 * every class launch) and collect (features, log2 ns) samples; K is computed
 * into library-owned scratch and discarded. */
fx_status fx_record_task_timings(const fx_tree* tree, const double* P, double tau, const fx_exchange_opts* opts,
                                 fx_task_timings** out, void* stream);
/* Samples from host arrays (feats: 4 per sample; cls may be NULL). */
fx_status fx_task_timings_create(const float* feats, const float* log2_ns, const int32_t* cls, int64_t n,
                                 fx_task_timings** out);
int64_t fx_task_timings_count(const fx_task_timings* t);
fx_status fx_task_timings_get(const fx_task_timings* t, float* feats, float* log2_ns, int32_t* cls);
void fx_task_timings_free(fx_task_timings* t);

/* Train on the GPU (hand-written forward, backward and Adam kernels). */
fx_status fx_costmodel_train(const fx_task_timings* data, const fx_train_opts* opts, fx_costmodel** out,
                             float* final_loss, void* stream);
/* Parameters: FX_MLP layout of fx_costmodel_nparams() floats (W1[64][4],
 * b1[64], W2[64][64], b2[64], w3[64], b3); norm[10] = input means, input
 * standard deviations, target mean, target standard deviation. */
int32_t fx_costmodel_nparams(void);
fx_status fx_costmodel_create(const float* params, const float* norm, fx_costmodel** out);
fx_status fx_costmodel_params(const fx_costmodel* m, float* params, float* norm);
/* Predicted log2 ns for host feature arrays (4 per sample). */
fx_status fx_costmodel_predict(const fx_costmodel* m, const float* feats, int64_t n, float* out, void* stream);
/* Mean squared error on standardised targets and its gradient (host arrays). */
fx_status fx_costmodel_loss_grad(const fx_costmodel* m, const float* feats, const float* log2_ns, int64_t n,
                                 float* loss, float* grad, void* stream);
void fx_costmodel_free(fx_costmodel* m);
/* Serialise a model (parameters and normalisation, binary32) to a file, and
 * load one back; the loaded model predicts bitwise as the saved one.  Load
 * returns FX_ERR_INVALID_ARG for a missing, truncated or foreign file. */
fx_status fx_costmodel_save(const fx_costmodel* m, const char* path);
fx_status fx_costmodel_load(const char* path, fx_costmodel** out);

/* Kernel variant of a class (cls = ((la*3+lb)*3+lc)*3+ld) and precision
 * (prec32 0/1): 0 = one quartet per lane, 1 = one quartet per wave with the
 * HGP intermediates in LDS, 2 (FP64 entry only) = in mixed precision with one
 * density, both precisions in one kernel that screens each candidate once
 * (the FP32 entry is then unused).  Defaults are built in per class and the
 * autotuner may change them; all variants give the same quartet set and agree
 * to rounding.  Process-wide setting; FX_ERR_INVALID_ARG for a bad class,
 * precision or variant, FX_ERR_UNSUPPORTED for a variant not built. */
fx_status fx_set_class_variant(int32_t cls, int32_t prec32, int32_t variant);
int32_t fx_get_class_variant(int32_t cls, int32_t prec32);
/* Launch flags of a class and precision: bit 0 = XCD-aware workgroup remap
 * (neighbouring K blocks, which share density and pair data, on one XCD and
 * its L2).  Bit 1 (persistent grid pulling units from an atomic counter) is
 * switched off and returns FX_ERR_UNSUPPORTED.  Chosen by the autotuner; K
 * does not depend on them. */
fx_status fx_set_class_launch(int32_t cls, int32_t prec32, int32_t flags);
int32_t fx_get_class_launch(int32_t cls, int32_t prec32);
/* Logical block of hardware workgroup b of nb under the XCD remap (-1 if out
 * of range); host-callable so the mapping can be checked. */
int64_t fx_xcd_block(int64_t b, int64_t nb);
/* Bit mask of the variants built for a class (bit v = variant v). */
int32_t fx_class_variants_available(int32_t cls);

/* Host-only planning helper (no device work): the cuts that split a row of
 * nleaf leaf blocks into nchunks contiguous, non-empty K row ranges, as a
 * call whose workspace budget needs several ranges takes them.
 * leaf_entries[nleaf] (host, nullable): traversal entries per leaf row; the
 * ranges then hold about equal entries (cut k at the first leaf boundary
 * where the running sum reaches k/nchunks of the total), else about equal
 * leaf counts.  cuts[nchunks + 1] (host, caller-owned): range k is leaves
 * [cuts[k], cuts[k+1]); nchunks above nleaf is reduced to nleaf and the
 * cuts beyond it are nleaf. */
fx_status fx_plan_row_cuts(const int64_t* leaf_entries, int32_t nleaf, int32_t nchunks, int32_t* cuts);

/* Shared screen per (l_a, l_d) group (default off): where every leaf holds at
 * most one shell of each angular momentum, one kernel per group tests each
 * entry's nine (l_b, l_c) candidates with the bound of Eq. (8) and the
 * group's nine class kernels read the outcomes; off, each class kernel tests
 * its own candidates.  The same quartets are computed in the same order
 * either way, so K is bitwise the same.  Off by default because it measured
 * slower (the class kernels' candidate scan is bound by its own loop, not by
 * the norm gathers this removes).  Process-wide; not thread-safe against
 * running calls. */
fx_status fx_set_group_screen(int32_t enabled);
int32_t fx_get_group_screen(void);

/* Device allocator used for all library memory (NULL, NULL restores
 * hipMallocAsync / hipFreeAsync).  Not thread-safe against running calls. */
typedef void* (*fx_alloc_fn)(size_t bytes, void* stream, void* ctx);
typedef void (*fx_free_fn)(void* ptr, void* stream, void* ctx);
fx_status fx_set_allocator(fx_alloc_fn alloc, fx_free_fn free_, void* ctx);

/* Progress of long one-system calls: fn(done, total, ctx) is called on a
 * runtime thread each time the device finishes one K row range of an eager
 * call (`total` counts the ranges planned so far; a replayed graph reports
 * nothing).  The stream waits while fn runs, so fn must return quickly and
 * must not wait for the stream.  NULL removes it.  Process-wide; not
 * thread-safe against running calls.  fx_progress_stderr is a ready-made fn
 * that prints one line per range to stderr (ctx: a NUL-terminated prefix, or
 * NULL for "fx"). */
typedef void (*fx_progress_fn)(int32_t done, int32_t total, void* ctx);
fx_status fx_set_progress(fx_progress_fn fn, void* ctx);
void fx_progress_stderr(int32_t done, int32_t total, void* ctx);

const char* fx_status_string(fx_status s);
const char* fx_last_error_message(void);

#ifdef __cplusplus
}
#endif
#endif /* FX_H */
