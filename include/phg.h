/*
 * phg.h -- C ABI of the MI355X (gfx950) phylogenetic likelihood-gradient library.
 *
 * Computes, for a rooted bifurcating tree, a reversible or general CTMC given by
 * its eigensystem, discrete rate categories and an alignment of weighted site
 * patterns, the log-likelihood log P(Y) and its derivative with respect to every
 * branch length, in time linear in the number of tips (Gangavarapu et al.,
 * "Many-core algorithms for high-dimensional gradients on phylogenetic trees",
 * arXiv:2303.04390, Methods section: pruning equation, sequence-likelihood
 * equation, eq:preorder, eq:gradient and eq:gradientSumAcrossColumns).
 *
 * Conventions (Methods, labelling paragraph, written 0-based):
 *   - N tips are nodes 0..N-1, internal nodes N..2N-3, the root is 2N-2.
 *   - Every non-root node x owns the branch to its parent; branch lengths and
 *     gradients are arrays of length 2N-2 indexed by child node x.
 *   - An unrooted tree is a rooted one with one root branch of length zero.
 *   - S states (2..256), R rate categories (1..64), C site patterns (>= 1).
 *
 * General rules for every call:
 *   - Every call returns a phg_status; PHG_OK (0) on success, a negative code
 *     otherwise, with a message available from phg_last_error().
 *   - Every input array is copied before the call returns; the caller keeps
 *     ownership of its memory and may free or reuse it at once.
 *   - Output arrays are caller-allocated.  Host pointers unless stated.
 *   - No C++ exception crosses this boundary.
 *   - A context is used from one thread at a time; distinct contexts are
 *     independent and may be used concurrently.
 *   - Inputs are validated on the host (no device work) when they are set;
 *     the device is first touched by a compute call (or phg_prepare).
 */
#ifndef PHG_H
#define PHG_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
    PHG_OK = 0,
    PHG_ERR_ARG = -1,      /* invalid argument: sizes, topology, values out of range */
    PHG_ERR_STATE = -2,    /* compute requested before every required input was set */
    PHG_ERR_OOM = -3,      /* device allocation failed or bound workspace too small */
    PHG_ERR_DEVICE = -4,   /* no usable gfx950 device, or a HIP runtime error */
    PHG_ERR_NUMERIC = -5,  /* some weighted site likelihood is zero or not finite */
    PHG_ERR_BUSY = -6      /* resource temporarily unavailable (serving queue full) */
} phg_status;

typedef enum {
    PHG_FP64 = 0,          /* partials, P(t) and reductions in float64 */
    PHG_FP32_SCALED = 1    /* partials and P(t) copies in float32 with per-node,
                              per-pattern power-of-two rescaling shared across
                              categories; P(t) built in float64; per-pattern
                              ratios and all reductions in float64.  Subject
                              to the FP32 precision guard (phg_set_fp32_guard):
                              a tree too saturated for float32 partials is
                              evaluated in FP64 */
} phg_precision;

typedef struct phg_context phg_context;

/* Create a context for one (tree, alignment) problem of fixed sizes.
 * n_tips >= 2, n_patterns >= 1, 2 <= n_states <= 256, 1 <= n_categories <= 64,
 * device = HIP device ordinal.  *out receives the context (NULL on error).
 * Host-only: no device work happens here. */
phg_status phg_create(int n_tips, int n_patterns, int n_states, int n_categories,
                      phg_precision prec, int device, phg_context **out);

/* Release the context and every device buffer it allocated.  Accepts NULL. */
phg_status phg_destroy(phg_context *ctx);

/* Message describing the last error on ctx (or on context creation when ctx
 * is NULL).  Owned by the library; valid until the next call on ctx. */
const char *phg_last_error(const phg_context *ctx);

/* Tree topology (Methods, labelling paragraph).  parent has 2N-1 entries:
 * parent[root = 2N-2] = -1; every other node's parent is an internal node or
 * the root; tips have no children; internal nodes and the root have exactly two;
 * no cycles.  PHG_ERR_ARG otherwise. */
phg_status phg_set_topology(phg_context *ctx, const int32_t *parent);

/* Branch lengths b[x], x = 0..2N-3, indexed by child node (Methods).  Each
 * must be finite and >= 0.  Cheap to call repeatedly (e.g. per HMC step). */
phg_status phg_set_branch_lengths(phg_context *ctx, const double *b);

/* Substitution model through its eigensystem: Q = V diag(lambda) Vinv, so
 * P^(r)(b) = exp(gamma_r b Q) = V diag(exp(gamma_r b lambda)) Vinv (Methods,
 * equation for P).  V and Vinv are S*S row-major, lambda has S entries; all
 * finite.  The library does not check that Vinv inverts V. */
phg_status phg_set_eigen(phg_context *ctx, const double *V, const double *Vinv,
                         const double *lambda);

/* One substitution model per rate category: category r evolves under
 * Q^(r) = rates[r] * V_r diag(lambda_r) Vinv_r (the gradient-kernel section
 * keeps the algorithm general for generators that vary across categories).
 * V and Vinv are R*S*S (category-major, each S*S row-major), lambda R*S;
 * all finite; copied.  Replaces any eigensystem set before, and
 * phg_set_eigen replaces this one.  The serving engine takes one shared
 * model per tree. */
phg_status phg_set_category_eigen(phg_context *ctx, const double *V, const double *Vinv,
                                  const double *lambda);

/* Root prior pi (S entries, finite, >= 0), the q vector at the root
 * (Methods, sequence-likelihood equation and eq:preorder). */
phg_status phg_set_root_frequencies(phg_context *ctx, const double *pi);

/* Discrete rate categories: rates gamma_r (finite, >= 0) and probabilities
 * P(gamma_r) (finite, >= 0), R entries each (Methods, rate-variation
 * paragraph; Q^(r) = gamma_r Q). */
phg_status phg_set_categories(phg_context *ctx, const double *rates,
                              const double *weights);

/* Observed tip states (Methods, alignment paragraph; compact integer tip
 * states of the gradient-kernel section).  codes is N*C, tip-major
 * (codes[tip*C + c]); each value is 0..S-1, or S for a fully ambiguous
 * entry whose partial is all ones. */
phg_status phg_set_tip_states(phg_context *ctx, const int32_t *codes);

/* General tip partial vector of one tip (Methods, pruning equation: a tip's
 * partial vector in its general form, for partial ambiguity or observation
 * error models).  partials is C*S, pattern-major: partials[c*S + s] is the
 * probability of the tip's data at pattern c given state s; finite, >= 0.
 * It replaces the tip's code (which must still be set and is then ignored);
 * NULL reverts the tip to its code.  Copied.  Values are used as given
 * (rounded to float in FP32 contexts; no rescaling at tips).  A context with
 * any such tip evaluates on the level schedule: PHG_SCHEDULE_AUTO picks it
 * and PHG_SCHEDULE_BLOCKS is rejected (PHG_ERR_ARG) while one is set.  The
 * device copy lives in memory the context allocates itself, also when a
 * workspace is bound.  Not available through the serving engine. */
phg_status phg_set_tip_partials(phg_context *ctx, int tip, const double *partials);

/* Pattern weights W_c (C entries, finite, >= 0): the multiplicity of each
 * unique column (Methods, pattern-compression remark).  A zero-weight
 * pattern contributes nothing, even if its likelihood is zero.
 * Defaults to all ones. */
phg_status phg_set_pattern_weights(phg_context *ctx, const double *w);

/* Traversal schedule.  LEVELS: one launch per tree level, every internal
 * node's partial stored in device memory.  BLOCKS (4 states, R <= 8): the tree
 * is cut into blocks of depth 3 (a block root at
 * every depth that is a multiple of 3, with its internal children and
 * grandchildren); only block roots' partials go to device memory and the
 * pre-order pass recomputes in-block post-order partials in registers, which
 * moves about 2.5x fewer bytes on a Yule tree; one launch per block level and
 * pass.  QUEUE (4 states, FP32, R in {1, 2, 4, 8}; opt-in): the same blocks
 * and arithmetic, one launch per pass (PHG_TUNE_QUEUE_LAUNCHES) over
 * (block, 64-pattern tile) work items in dependency order, each waiting only
 * on the items it reads (Methods: the post-order and pre-order recursions
 * order nodes, not whole tree levels), so there is no level-wide barrier.
 * It relies on the GPU starting a launch's workgroups in increasing order on
 * each XCD, and is meant for one such evaluation on the device at a time:
 * two QUEUE evaluations running concurrently on different streams can stall
 * each other until a wait gives up after 2 s, when the evaluation returns
 * NaN (PHG_ERR_NUMERIC from the synchronous calls).  A tree too large for
 * one launch per pass runs BLOCKS.  AUTO (default) picks BLOCKS where
 * supported.  Same results up to rounding order; BLOCKS and QUEUE give
 * bitwise-identical results. */
typedef enum {
    PHG_SCHEDULE_AUTO = 0,
    PHG_SCHEDULE_LEVELS = 1,
    PHG_SCHEDULE_BLOCKS = 2,
    PHG_SCHEDULE_QUEUE = 3
} phg_schedule;
phg_status phg_set_schedule(phg_context *ctx, phg_schedule mode);

/* The schedule in effect for the current topology: *schedule is
 * PHG_SCHEDULE_LEVELS, PHG_SCHEDULE_BLOCKS or PHG_SCHEDULE_QUEUE (AUTO
 * resolved).  PHG_ERR_STATE
 * before the topology is set. */
phg_status phg_get_schedule(phg_context *ctx, int *schedule);

/* Allocate device memory and upload inputs without computing.  Optional. */
phg_status phg_prepare(phg_context *ctx);

/* log P(Y) = sum_c W_c log sum_r P(gamma_r) p_root,r,c . pi.  Synchronous.
 * Runs P(t), the post-order pass and the final sum only (no pre-order pass).
 * PHG_ERR_STATE until topology, branch lengths, eigensystem, root
 * frequencies, categories and tip states are all set.  If a weighted site
 * likelihood is zero or not finite, *logl = -inf and PHG_ERR_NUMERIC. */
phg_status phg_log_likelihood(phg_context *ctx, double *logl);

/* log P(Y) (if logl is not NULL) and grad[x] = d log P(Y) / d b_x for all
 * 2N-2 branches (eq:gradient summed by eq:gradientSumAcrossColumns).
 * Synchronous.  On PHG_ERR_NUMERIC, *logl = -inf and grad is all NaN. */
phg_status phg_gradient(phg_context *ctx, double *logl, double *grad);

/* ---- FP32 precision guard ----
 *
 * Float32 partials carry a gradient component to ~1e-4 of itself only while
 * the pre-order vector reaching a branch and its sibling's vector keep some
 * distance from the stationary and the flat vector.  Where both neighbours
 * of a branch are long, the component becomes a small difference of nearly
 * equal terms (rows of dP sum to zero, eq:gradient) and a single float32
 * rounding of the stored partials moves it by more than that.  The guard
 * measures this on the host before every evaluation of an FP32 context:
 *   saturation = max over internal nodes k and children x' of k of
 *                min(L_k, L_x'),   L_v = b_v * max_r(gamma_r * mu_r),
 * mu_r the smallest non-zero |lambda| of category r's generator (the slowest
 * decay of the fastest category), L_root = infinity.  Above the threshold
 * the evaluation runs on an FP64 twin of the context (same inputs, its own
 * device memory, same stream), so results keep the FP64 bar.  The default
 * threshold is 1.5.  Contexts with a bound workspace never route (they
 * allocate nothing of their own); the serving engine does not route. */

/* threshold >= 0; 0 disables the guard.  Applies to FP32 contexts only. */
phg_status phg_set_fp32_guard(phg_context *ctx, double threshold);

/* The guard's saturation statistic for the current inputs (host only).
 * PHG_ERR_STATE before topology, branch lengths, eigensystem and categories
 * are set. */
phg_status phg_fp32_saturation(phg_context *ctx, double *saturation);

/* Precision the last evaluation ran in (PHG_FP64 or PHG_FP32_SCALED), or -1
 * before the first. */
phg_status phg_last_precision(phg_context *ctx, int *prec);

/* ---- tile-shape tuning ----
 *
 * A process-wide table of kernel shape parameters, per (state count,
 * category count, precision).  Filled at the library's first use from a
 * tuning file written by the project's autotuner (paper_2303_04390_amd/
 * autotune.py): the file named by the environment variable PHG_TUNE_FILE, else
 * tune_cache.txt beside libphg.so; PHG_TUNE=off skips it.  Each line reads
 * "gfx950 S R prec param value" (prec 0 = FP64, 1 = FP32; R = 0 matches any
 * category count); lines for other devices and '#' comments are ignored.
 * phg_set_tuning changes an entry at run time.  Value 0 means the built-in
 * rule.  Row blocks are read when a context is created (its tile is fixed for
 * its lifetime); the narrow-launch threshold when a launch is issued. */
typedef enum {
    PHG_TUNE_ROW_BLOCKS = 0,    /* 17..255 states: 16-pattern row blocks per tile (1, 2 or 4,
                                   as built for S and the precision) */
    PHG_TUNE_NARROW_UNITS = 1,  /* 4 states, blocked FP32 kernels: largest launch (workgroups)
                                   that takes the one-round-trip narrow variant */
    PHG_TUNE_QUEUE_LAUNCHES = 2,  /* 4 states, QUEUE schedule: launches per evaluation with the
                                     gradient (1: both passes in one; 2, the default: one per pass) */
    PHG_TUNE_QUEUE_WAIT_US = 3,   /* QUEUE schedule: microseconds a work item waits on another before
                                     the evaluation is abandoned as faulty (NaN results,
                                     PHG_ERR_NUMERIC); default 2 s.  A tiny value forces that path. */
    PHG_TUNE_PARAMS = 4
} phg_tune_param;

/* n_categories = 0: any category count.  PHG_ERR_ARG for an unknown
 * parameter or a value the kernels are not built for. */
phg_status phg_set_tuning(int n_states, int n_categories, phg_precision prec, int param, int value);

/* The value in effect (0: the built-in rule). */
phg_status phg_get_tuning(int n_states, int n_categories, phg_precision prec, int param, int *value);

/* ---- library-owned HIP graphs ----
 *
 * phg_gradient and phg_log_likelihood capture their evaluation's kernel
 * launches (P(t), post-order levels, pre-order levels, final sums) as a HIP
 * graph on first use and replay it on later calls while the launch sequence
 * is unchanged: new branch lengths, model, categories, tip states and
 * pattern weights are uploaded before the replay and leave the graph valid;
 * a new topology, schedule, general tip partials, per-category eigensystems
 * switched on or off, or a new device binding drop it (captured again on next
 * use).  Tuning values read at launch (PHG_TUNE_NARROW_UNITS) are those of
 * the capture.  Not used while profiling, nor by phg_gradient_async (whose
 * callers can capture it themselves) or the chain-rule calls. */

/* on = 0 turns graphs off for this context (every call issues its launches);
 * default on. */
phg_status phg_set_graphs(phg_context *ctx, int on);

/* Graphs captured and replays issued by this context so far (each nullable). */
phg_status phg_graph_stats(phg_context *ctx, uint64_t *captures, uint64_t *replays);

/* ---- parameter chain rules: node heights, branch rates, branch sets ----
 *
 * The Methods section's problem statement allows a branch length to be the
 * difference between the parent's and the child's node heights times a
 * (possibly branch-specific) rate scalar, and the gradient-kernel section
 * sums branch derivatives over a chosen set of branches (e.g. a strict
 * clock).  These calls apply those chain rules on the device right after the
 * gradient, g_i = d logL / d b_i:
 *   d logL / d rate_i = (h_parent(i) - h_i) g_i
 *   d logL / d h_k    = sum over children c of k of rate_c g_c
 *                       - rate_k g_k   (the last term absent at the root)
 *   set sums          = sum over the branches of a set, increasing index.
 */

/* b_i = (heights[parent(i)] - heights[i]) * rates[i].  heights: 2N-1 by node
 * (root 2N-2); rates: 2N-2 by child node; both copied.  Replaces the branch
 * lengths and keeps heights and rates for phg_time_tree_gradient until the
 * next phg_set_branch_lengths or phg_set_topology.  PHG_ERR_STATE before the
 * topology; PHG_ERR_ARG on NULL, a non-finite height, a rate that is
 * negative or not finite, or a node above its parent. */
phg_status phg_set_time_tree(phg_context *ctx, const double *heights, const double *rates);

/* Branch sets: set_of[i] (2N-2 int32 by child node) in [0, n_sets), or -1 for
 * a branch in no set; 1 <= n_sets <= 2N-2; copied.  n_sets = 0 clears
 * (set_of may be NULL).  PHG_ERR_ARG on an entry out of range. */
phg_status phg_set_branch_sets(phg_context *ctx, const int32_t *set_of, int n_sets);

/* One evaluation under the time tree.  Writes (each nullable): logL;
 * d_heights (2N-1) = d logL / d h; d_rates (2N-2) = d logL / d rate; d_sets
 * (n_sets) = sum over set j of d_rates, the derivative with respect to one
 * rate shared by the branches of set j (a strict clock is one set holding
 * every branch).  Synchronous.  PHG_ERR_STATE without phg_set_time_tree, or
 * with d_sets and no branch sets; PHG_ERR_NUMERIC as phg_gradient (outputs
 * NaN, logL -inf). */
phg_status phg_time_tree_gradient(phg_context *ctx, double *logl, double *d_heights,
                                  double *d_rates, double *d_sets);

/* One evaluation; d_sets[j] = sum over set j of d logL / d b_i (branch
 * lengths tied within a set).  logl nullable, d_sets not.  PHG_ERR_STATE
 * without branch sets; PHG_ERR_NUMERIC as phg_gradient. */
phg_status phg_gradient_branch_sets(phg_context *ctx, double *logl, double *d_sets);

/* ---- device-side variants (memory and streams owned by the caller) ---- */

/* Device memory for the P(t) tables of 17..256 states.  A context keeps
 * P, dP and their transposes for every (branch, category) when they fit in
 * `bytes` (default 16 GiB); otherwise it holds a pool of as many branches'
 * tables as fit (at least 2) and rebuilds them for each launch chunk of at
 * most pool/2 nodes, just before the post-order or pre-order launch that
 * reads them (P(t) is then computed twice per evaluation; results are
 * bitwise those of full tables).  At 256 states, 20,000 branches and 4
 * categories in FP32 the full tables take 84 GB, the default pool 16 GiB.
 * Before first use (PHG_ERR_STATE after).  phg_workspace_size assumes the
 * default; the serving engine keeps full tables. */
phg_status phg_set_table_budget(phg_context *ctx, size_t bytes);

/* Branch tables the context holds: 0 for every branch's, else the pool size
 * (what first use will choose, before it). */
phg_status phg_table_slots(phg_context *ctx, int *slots);

/* Bytes of device workspace a context of these sizes needs. */
phg_status phg_workspace_size(int n_tips, int n_patterns, int n_states,
                              int n_categories, phg_precision prec, size_t *bytes);

/* The level kernels a context of these sizes runs (host only; no device
 * work).  All families compute the same quantities (Methods: pruning
 * equation, eq:preorder, eq:gradient); they differ in how the products are
 * laid out on the hardware. */
typedef enum {
    PHG_KERNELS_FOUR_STATE = 0,  /* 4 states, R <= 8: blocked or level 4-state kernels */
    PHG_KERNELS_SMALL_MFMA = 1,  /* other shapes up to 16 states (and 4 states with R > 8) */
    PHG_KERNELS_VECTOR_ALU = 2,  /* 17..32 states (FP64: 17..24), R in 1, 2, 4, 8: one wave per
                                    category, per-lane products on the vector ALUs */
    PHG_KERNELS_MFMA = 3         /* other shapes above 16 states: MFMA tiles */
} phg_kernel_family;

/* PHG_ERR_ARG for sizes phg_create would refuse. */
phg_status phg_kernel_family_of(int n_states, int n_categories, phg_precision prec, int *family);

/* Use caller-owned device memory (>= phg_workspace_size bytes, 256-byte
 * aligned) instead of allocating.  It must outlive every later compute call.
 * Must be called before the first compute call / phg_prepare. */
phg_status phg_bind_workspace(phg_context *ctx, void *device_ptr, size_t bytes);

/* Issue all later device work on this hipStream_t (NULL = the library's own
 * stream).  The stream must outlive its use by the context. */
phg_status phg_bind_stream(phg_context *ctx, void *hip_stream);

/* Enqueue logL + gradient on the bound stream and return without waiting.
 * d_logl (1 double) and d_grad (2N-2 doubles) are device pointers; they are
 * valid once the stream reaches this point.  Host inputs set before this call
 * are uploaded first, in stream order.  No numeric check is done (inspect
 * *d_logl: -inf or NaN signals a zero site likelihood). */
phg_status phg_gradient_async(phg_context *ctx, double *d_logl, double *d_grad);

/* For callers that cannot allocate device memory (code under HIP graph
 * capture, tight serving loops, harnesses that forbid allocation): the same
 * evaluation as phg_gradient_async, with the context's whole workspace in a
 * static device array of PHG_NOALLOC_SCRATCH_BYTES (64 MiB) that the library
 * holds on each GPU it runs on until the process ends.  Calls no hipMalloc,
 * hipFree or other allocating routine.  Requirements, else an error and no
 * device work: a stream bound with phg_bind_stream (PHG_ERR_STATE);
 * phg_workspace_size of the context <= PHG_NOALLOC_SCRATCH_BYTES
 * (PHG_ERR_OOM); no general tip partials (PHG_ERR_ARG); the context has not
 * evaluated in other device memory before (PHG_ERR_STATE).  Every context
 * using this call on one GPU shares that GPU's array: a context whose data
 * another context may have overwritten since its last call uploads all its
 * inputs again (and waits for those copies), so alternating contexts is
 * correct but slower; calls that overlap in time on one GPU (other threads,
 * or work still queued on another stream) race and corrupt each other.  Not
 * routed by the FP32 precision guard.  Profiling events are not recorded. */
#define PHG_NOALLOC_SCRATCH_BYTES ((size_t)64 << 20)
phg_status phg_gradient_async_noalloc(phg_context *ctx, double *d_logl, double *d_grad);

/* Wall-clock-free introspection: number of kernel launches one gradient call
 * issues and the post-/pre-order level counts of the current topology. */
phg_status phg_schedule_info(phg_context *ctx, int *n_post_levels,
                             int *n_pre_levels, int *n_launches);

/* ---- measurement ---- */

/* Kernel classes timed by the profiler, in the order of one evaluation. */
enum { PHG_PROF_PMAT = 0, PHG_PROF_POST = 1, PHG_PROF_PRE = 2, PHG_PROF_FINAL = 3,
       PHG_PROF_CLASSES = 4 };

/* on != 0: every later evaluation records HIP events on the context's stream
 * around each kernel class (P(t); post-order levels incl. the root; pre-order
 * + gradient levels; final sums).  on == 0 stops recording.  Recording adds
 * event records between launches and nothing else, except that a QUEUE
 * schedule records one launch per pass even where it is tuned to one launch
 * for both. */
phg_status phg_profile_enable(phg_context *ctx, int on);

/* Wait for the recorded evaluations, then write the summed device time in
 * milliseconds of each kernel class into ms[0..PHG_PROF_CLASSES-1], the
 * number of evaluations recorded into *n_evals and the number of kernel
 * launches per class per evaluation into launches[0..3] (either pointer may
 * be NULL).  Clears the record. */
phg_status phg_profile_read(phg_context *ctx, double *ms, int *n_evals, int *launches);

/* ---- serving: many trees, continuous batching ----
 *
 * A server owns one device, a device-memory budget and a scheduler thread.
 * Trees (topology, model, alignment) are registered once; each request
 * brings new branch lengths for a registered tree (as an HMC sampler or
 * several chains do) and asks for log P(Y) and all 2N-2 derivatives.
 * Requests are admitted when a slot is free and the tree's workspace fits
 * the budget (idle resident trees are evicted least-recently-used first);
 * every scheduler step advances each in-flight request by one stage of the
 * path (P(t), one post-order level, one pre-order level, or the final sums),
 * and requests at the same stage kind share kernel launches, so requests that
 * arrive while others run join at the next step.  Results do not depend on
 * what else is in flight (every work unit's arithmetic is independent of the
 * batch).  One evaluation per tree is in flight at a time; later requests for
 * the same tree wait for it.  All server calls are thread-safe. */
typedef struct phg_server phg_server;

/* Everything that defines one tree's problem (host pointers, copied by
 * phg_server_register_tree).  Layouts as for the phg_set_* calls above;
 * pattern_weights may be NULL (all ones). */
typedef struct {
    int n_tips, n_patterns, n_states, n_categories;
    phg_precision prec;
    const int32_t *parent;
    const double *V, *Vinv, *lambda;
    const double *pi;
    const double *rates, *weights;
    const int32_t *codes;
    const double *pattern_weights;
    /* Optional, zero / NULL when unused (the gradient-kernel section's
     * general form): per_category_eigen != 0 means V, Vinv hold R models
     * (R*S*S each) and lambda R*S, as phg_set_category_eigen; n_tip_vectors
     * tips (ids in tip_vector_tips) take general partial vectors, C*S each,
     * concatenated in tip_vectors, as phg_set_tip_partials (their device copy
     * lives outside the memory budget). */
    int per_category_eigen;
    int n_tip_vectors;
    const int32_t *tip_vector_tips;
    const double *tip_vectors;
} phg_tree_desc;

/* max_slots in [1, 48] concurrent evaluations; mem_budget_bytes of device
 * memory is reserved at creation for resident trees' workspaces. */
phg_status phg_server_create(int device, size_t mem_budget_bytes, int max_slots,
                             phg_server **out);
phg_status phg_server_destroy(phg_server *srv);
const char *phg_server_last_error(const phg_server *srv);

/* Validate and copy a tree (no device work).  PHG_ERR_OOM if its workspace
 * alone exceeds the budget. */
phg_status phg_server_register_tree(phg_server *srv, const phg_tree_desc *desc,
                                    uint64_t *tree_id);

/* Queue one evaluation of tree_id at branch lengths b (2N-2 doubles, copied;
 * finite and >= 0).  Never fails for lack of memory: the request waits. */
phg_status phg_server_submit(phg_server *srv, uint64_t tree_id, const double *b,
                             uint64_t *req_id);

/* Non-blocking: *done = 1 and results written (logl may be NULL; grad has
 * 2N-2 doubles) once the request finished, after which req_id is forgotten.
 * A finished request whose site likelihood was zero returns PHG_ERR_NUMERIC
 * with logl = -inf and NaN gradients. */
phg_status phg_server_poll(phg_server *srv, uint64_t req_id, double *logl, double *grad,
                           int *done);

/* phg_server_poll that also reports, on the server's monotonic clock in
 * nanoseconds, when the request was submitted and when its results were
 * observed in host memory (either pointer may be NULL). */
phg_status phg_server_poll_timed(phg_server *srv, uint64_t req_id, double *logl, double *grad,
                                 int *done, uint64_t *t_submit_ns, uint64_t *t_done_ns);

/* Blocking variant of phg_server_poll. */
phg_status phg_server_wait(phg_server *srv, uint64_t req_id, double *logl, double *grad);

/* Forget a tree: its device memory is released once no request for it is
 * queued or in flight.  Requests submitted afterwards fail with PHG_ERR_ARG. */
phg_status phg_server_release_tree(phg_server *srv, uint64_t tree_id);

/* Kernel time and wall time since the server's creation, in nanoseconds:
 * *busy_ns sums, over scheduler steps, the device time from the step's first
 * launch to its last (HIP events on the compute stream), so busy / wall is
 * the fraction of time the GPU spent on serving kernels.  Either pointer may
 * be NULL. */
phg_status phg_server_busy(phg_server *srv, uint64_t *busy_ns, uint64_t *wall_ns);

/* Counters since creation: stats[0] requests completed, [1] scheduler steps,
 * [2] kernel launches, [3] resident trees now, [4] evictions, [5] peak bytes of
 * the budget in use, [6] requests now queued, [7] requests now in flight. */
phg_status phg_server_stats(phg_server *srv, uint64_t stats[8]);

#ifdef __cplusplus
}
#endif

#endif /* PHG_H */
