/*
 * epochlik — epoch-model (time-inhomogeneous) phylogenetic likelihood on
 * AMD Instinct MI355X (gfx950).
 *
 * The method (Bielejec et al., "Inferring heterogeneous evolutionary processes
 * through time"):
 *   - S rate matrices Q_s; a change-point process with fixed boundaries picks
 *     which Q_s is active in each time interval (Methods, "Relaxing
 *     time-homogeneity").
 *   - A branch that crosses boundaries gets the ordered product of per-interval
 *     exponentials, parent-side interval first (Eq. 5-7, Fig. 1); each factor
 *     is V_s diag(exp(lambda_s * rho_c * r_b * t_bk)) V_s^-1, reusing one
 *     eigensystem for any rate and time (Appendix A).
 *   - Felsenstein pruning over every node, pattern and rate category (Eq. 4),
 *     then the root sum over pi and categories, aggregated over patterns with
 *     integer weights (text after Eq. 4).
 *   - Additions the paper does not contain: per-(node, pattern) power-of-two
 *     rescaling, an adjoint (pre-order) pass giving dlogL/d(branch length) and
 *     dlogL/dQ_s, an FP32 bulk path next to FP64, and batched evaluation.
 *
 * Conventions
 *   - Times are HEIGHTS (time before the youngest tip, >= 0 or any real).
 *     Interval k covers heights [b_k, b_{k+1}) with b_0 = -inf, b_M = +inf;
 *     interval 0 is the youngest.  A zero-length stretch (a node exactly on a
 *     boundary) contributes no factor.
 *   - Nodes: tips 0..N-1, internal nodes N..2N-2 in any order; exactly one
 *     node has parent -1 (the root).  The tree must be binary.
 *   - Matrices passed in are row-major K x K, rows = the earlier (parent-side)
 *     state.  Transition matrices read back are row-major too.
 *   - The library pads K internally (4 -> 4, up to 64 -> multiple of 16);
 *     padding is invisible at the ABI.
 *
 * Ownership: every host pointer is borrowed for the duration of the call and
 * copied; the library owns all device memory it allocates.  Device pointers
 * are never taken or returned, except by epoch_eigen_residual_noalloc, which
 * works on caller-owned device memory only.  An instance is
 * not thread-safe; distinct instances are independent.  All device work runs
 * on the stream given in EpochConfig (NULL = the default stream); calls that
 * return host results synchronise that stream.
 *
 * Errors: functions return EPOCH_OK (0), a negative error code, or a positive
 * warning.  epoch_last_error() returns a thread-local message for the last
 * non-zero return on the calling thread.
 */
#ifndef EPOCHLIK_H
#define EPOCHLIK_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define EPOCH_OK 0
#define EPOCH_ERR_ARG (-1)       /* invalid argument (shape, range, non-finite value) */
#define EPOCH_ERR_STATE (-2)     /* call-order violation (a required set_/update_ step missing) */
#define EPOCH_ERR_OOM (-3)       /* device allocation failed */
#define EPOCH_ERR_HIP (-4)       /* a HIP runtime call failed */
#define EPOCH_ERR_NUMERIC (-5)   /* NaN or +inf likelihood (non-finite inputs), or a gradient asked
                                  * for a state whose log-likelihood is -inf */
#define EPOCH_WARN_EIGEN_RESIDUAL 1 /* eigensystem reconstruction residual above 1e-8 (relative) */
#define EPOCH_WARN_UNDERFLOW 2   /* some pattern's likelihood is zero in the working precision:
                                  * logL = -inf is returned (see root_log_likelihood) */

#define EPOCH_FP32 1
#define EPOCH_FP64 2

#define EPOCH_GRAD_BRANCH 0x1u   /* keep what log_likelihood_gradient needs for dlogL/dl_b */
#define EPOCH_GRAD_Q 0x2u        /* ... and for dlogL/dQ_s */
#define EPOCH_GRAD_TIME 0x4u     /* ... and for epoch_time_gradient (implies EPOCH_GRAD_BRANCH; the
                                  * 4-state kernels then run per tree level, and an HBM budget on the
                                  * 4-state path is refused) */

#define EPOCH_KERNEL_AUTO 0      /* pick the specialised kernels where they exist */
#define EPOCH_KERNEL_GENERIC 1   /* force the generic any-K kernels (reference GPU path) */

typedef struct EpochInstance EpochInstance;

typedef struct EpochConfig {
  int32_t n_tips;          /* N >= 2 */
  int32_t n_patterns;      /* P >= 1 (unique site patterns) */
  int32_t n_states;        /* K, 2 <= K <= 64 */
  int32_t n_categories;    /* C, 1 <= C <= 8 (among-site rate categories) */
  int32_t n_processes;     /* S >= 1 (distinct rate matrices) */
  int32_t max_intervals;   /* upper bound on M passed to set_tree_epochs, >= 1 */
  int32_t precision;       /* EPOCH_FP32 or EPOCH_FP64: arithmetic of P matrices and partials */
  uint32_t flags;          /* EPOCH_GRAD_* */
  int32_t kernel_path;     /* EPOCH_KERNEL_AUTO or EPOCH_KERNEL_GENERIC */
  int32_t reserved;        /* must be 0 */
  int64_t hbm_budget_bytes; /* 0 = unlimited.  > 0: device bytes allowed for intermediate
                             * partials (and their scale rows and gradient partial sums):
                             * - n_states == 4 with EPOCH_KERNEL_AUTO, no EPOCH_GRAD_Q (with it,
                             *   EPOCH_ERR_ARG; EPOCH_KERNEL_GENERIC takes the chunked form below):
                             *   the tree walk stores only the partials of the largest subtrees that fit
                             *   and recomputes the others from the tip states in the gradient
                             *   pass; set_tree_epochs returns EPOCH_ERR_OOM when even the root
                             *   alone does not fit.
                             * - every other configuration (the 64-state kernels and the generic
                             *   kernels, EPOCH_GRAD_Q allowed): the patterns are evaluated in
                             *   chunks (a multiple of 64 patterns) whose partials, outside
                             *   vectors, scale exponents (and 64-state dlogL/dP partial sums)
                             *   fit; update_partials forms each chunk's partials and its share
                             *   of logL, and the gradient call forms them again chunk by chunk.
                             *   epoch_create returns EPOCH_ERR_ARG when one chunk of
                             *   min(64, n_patterns) patterns does not fit. */
  void* stream;            /* hipStream_t to run on, or NULL for the default stream */
  void* workspace;         /* NULL, or caller-owned device memory (e.g. a torch tensor) of
                            * workspace_bytes bytes that holds the pattern-sized buffers (tip
                            * states, weights, partials, outside vectors, scale exponents,
                            * per-pattern log-likelihoods); it must stay allocated until
                            * epoch_destroy.  Not combinable with hbm_budget_bytes. */
  int64_t workspace_bytes; /* >= epoch_workspace_bytes(cfg) when workspace is set */
} EpochConfig;

/* Message for the last non-zero return on this thread ("" if none). */
const char* epoch_last_error(void);

/* Library version string. */
const char* epoch_version(void);

/* Bytes of caller-owned device memory (EpochConfig.workspace) that hold this
 * configuration's pattern-sized buffers; *out receives it.  No device work. */
int epoch_workspace_bytes(const EpochConfig* cfg, int64_t* out);

/* Create an instance (Methods, coarse-grain parallel implementation: an
 * instance holds a fixed set of device buffers, allocated when it is created
 * and not grown afterwards).  Validates cfg (before any HIP call), then
 * allocates the device buffers whose size depends only on cfg (the
 * pattern-sized ones inside cfg->workspace when it is set); the tree-sized
 * ones follow at set_tree_epochs.  *out receives the handle. */
int epoch_create(const EpochConfig* cfg, EpochInstance** out);

/* Free every device buffer of the instance (the buffer pool of the same
 * passage); NULL is accepted. */
int epoch_destroy(EpochInstance* inst);

/* Tip data (text after Eq. 4: tips are 0/1 indicators of the (partially)
 * observed state).
 * states: host [N][P] row-major int32; value in [0, K) = observed state,
 * value K = missing (all-ones vector), value K + 1 + a = ambiguity set a of
 * epoch_set_tip_ambiguities (the indicator of the states in the set).  Any
 * other value -> EPOCH_ERR_ARG. */
int epoch_set_tip_states(EpochInstance* inst, const int32_t* states);

/* Ambiguity sets for partially observed tips (text after Eq. 4): sets: host
 * [n_codes] bit masks, bit j = state j possible (non-empty, states < K), so
 * that tip code K + 1 + a stands for set a.  n_codes in [0, 255 - K].  The tip
 * states must be set (again) afterwards. */
int epoch_set_tip_ambiguities(EpochInstance* inst, int32_t n_codes, const uint64_t* sets);

/* Pattern weights w_p: host [P], finite and >= 0. */
int epoch_set_pattern_weights(EpochInstance* inst, const double* weights);

/* Among-site rate categories (text after Eq. 4): rates rho_c > 0 and weights
 * w_c >= 0 summing to 1 (within 1e-9), host [C] each. */
int epoch_set_categories(EpochInstance* inst, const double* rates, const double* weights);

/* Root distribution pi (text after Eq. 4: L = sum_i pi_i L_root(i)): host [K],
 * entries >= 0, summing to 1 within 1e-9. */
int epoch_set_root_frequencies(EpochInstance* inst, const double* pi);

/* Eigensystem of process s (Appendix A: one decomposition reused for every
 * rate and time): Q_s = V diag(lambda) V^-1 in real form.
 *   V, Vinv: host K x K row-major.  lambda_re, lambda_im: host [K].
 *   lambda_im may be NULL (all eigenvalues real).  A complex pair occupies two
 *   consecutive columns j, j+1 with lambda_im[j] = b > 0, lambda_im[j+1] = -b,
 *   lambda_re[j] = lambda_re[j+1] = a; V[:, j] and V[:, j+1] hold the real and
 *   imaginary parts of the eigenvector of a + ib, so that Q V = V B with the
 *   2x2 block B = [[a, b], [-b, a]].
 *   Q: host K x K or NULL.  If given, an FP64 device kernel measures
 *   max|V B V^-1 - Q| / max|Q| and max|V V^-1 - I|; the larger is written to
 *   *residual_out (if not NULL) and EPOCH_WARN_EIGEN_RESIDUAL is returned when
 *   it exceeds 1e-8; the call then waits for the check.  Without Q it does not
 *   wait: the host arrays are converted into a library-owned pinned staging
 *   buffer and uploaded asynchronously on the instance's stream (they may be
 *   reused as soon as the call returns).  Invalidates transition matrices. */
int set_epoch_eigensystems(EpochInstance* inst, int32_t s, const double* V, const double* Vinv,
                           const double* lambda_re, const double* lambda_im, const double* Q,
                           double* residual_out);

/* Tree and epoch structure (Methods, change-point process; Coarse-grain
 * implementation: per-branch times spent in each interval).
 *   parent: host [2N-1], -1 at the root; height: host [2N-1] finite,
 *   height[parent[v]] >= height[v]; branch_rate: host [2N-1] > 0 (entry v is
 *   the rate r_v of the branch above v; the root entry is ignored) or NULL = 1.
 *   n_intervals M in [1, max_intervals]; boundaries: host [M-1] strictly
 *   ascending finite heights (NULL when M = 1); interval_process: host [M],
 *   values in [0, S).
 * The host planner splits every branch into its per-interval segments and
 * builds the traversal schedules.  Invalidates everything downstream. */
int set_tree_epochs(EpochInstance* inst, const int32_t* parent, const double* height,
                    const double* branch_rate, int32_t n_intervals, const double* boundaries,
                    const int32_t* interval_process);

/* Transition matrices of every branch and category (Eq. 3, 6, 7), plus their
 * derivatives with respect to the branch length when EPOCH_GRAD_BRANCH is set.
 * Requires all eigensystems, categories and the tree. */
int update_transition_matrices(EpochInstance* inst);

/* Post-order partial likelihoods with rescaling (Eq. 4).  Requires
 * update_transition_matrices, tip states. */
int update_partials(EpochInstance* inst);

/* logL = sum_p w_p log L_p (text after Eq. 4), reduced in FP64.
 *   logL: host double (required); site_logL: host [P] or NULL.
 * Requires update_partials, pattern weights, root frequencies.
 * Underflow: partials are rescaled per pattern by a power of two shared by
 * the rate categories (Eq. 4 is evaluated with the largest entry over states
 * and categories kept near 1), so a category far less likely than the best
 * one at some node is flushed to zero there; when, for one pattern, a
 * category that dominates one subtree and another that dominates a second
 * subtree are each flushed in the other, the pattern's likelihood is zero in
 * the working precision (FP32 reaches this far sooner than FP64).  Data that
 * are impossible under the model (a zero-length branch between different
 * states) give the same zero.  Either way logL = -inf and the site values are
 * written, EPOCH_WARN_UNDERFLOW is returned, and gradients of this state are
 * refused (EPOCH_ERR_NUMERIC).  A NaN or +inf logL returns EPOCH_ERR_NUMERIC. */
int root_log_likelihood(EpochInstance* inst, double* logL, double* site_logL);

/* Gradient of logL (an addition to the paper):
 *   d_branch: host [2N-1] or NULL: entry v = dlogL/dl_v for l_v = r_v * tau_v,
 *     the per-interval fractions of the branch held fixed; root entry 0.
 *     Needs EPOCH_GRAD_BRANCH.
 *   d_Q: host [S][K][K] or NULL: dlogL/dQ_s entrywise, for the Q_s whose
 *     eigensystems were set.  Needs EPOCH_GRAD_Q.
 * Requires root_log_likelihood for the current state, with a finite
 * log-likelihood (EPOCH_ERR_NUMERIC after EPOCH_WARN_UNDERFLOW). */
int log_likelihood_gradient(EpochInstance* inst, double* d_branch, double* d_Q);

/* Node-height and epoch-boundary gradients (an addition: the paper fixes the
 * transition times and names estimating them as the natural next step,
 * Discussion).  Heights and boundaries enter logL only through the stretch
 * durations of Eq. 7; branch rates are held fixed.
 *   d_height: host [2N-1] or NULL: dlogL/dh_v for every node height (tips too).
 *   d_boundary: host [M-1] or NULL: dlogL/db_m for every boundary.
 * Intervals are half-open [b_{m-1}, b_m), so for a node exactly on a boundary
 * (a tie) the value is the one-sided derivative for an increasing height or
 * boundary.  Needs EPOCH_GRAD_TIME and root_log_likelihood for the current
 * state; runs the branch-gradient pass first when it has not run for this
 * state.  Computed in FP64 from the branch adjoints of that pass. */
int epoch_time_gradient(EpochInstance* inst, double* d_height, double* d_boundary);

/* One whole evaluation with a single host synchronisation: the transition
 * matrices (Eq. 3, 6, 7), the post-order partials (Eq. 4), the root
 * log-likelihood and, on request, the gradients, enqueued back to back on the
 * instance's stream; equivalent to update_transition_matrices, update_partials,
 * root_log_likelihood and log_likelihood_gradient in turn, without the host
 * round trip between the log-likelihood and the gradient pass.
 *   what: EPOCH_EVAL_* bits (the log-likelihood is always computed).
 *   logL: host out; site_logL: host [P] out or NULL;
 *   d_branch, d_Q: host outs as in log_likelihood_gradient, required when
 *     EPOCH_EVAL_GRAD_BRANCH / EPOCH_EVAL_GRAD_Q are set (ignored otherwise).
 * Needs every input set (as the separate calls do) and the instance flags for
 * the requested gradients (EPOCH_ERR_STATE otherwise).  A logL of -inf
 * returns EPOCH_WARN_UNDERFLOW with logL and the site values written and the
 * requested gradient outputs filled with NaN; a NaN or +inf logL returns
 * EPOCH_ERR_NUMERIC after the outputs are written. */
#define EPOCH_EVAL_LOGL 0x1u
#define EPOCH_EVAL_GRAD_BRANCH 0x2u
#define EPOCH_EVAL_GRAD_Q 0x4u
int epoch_evaluate(EpochInstance* inst, uint32_t what, double* logL, double* site_logL, double* d_branch,
                   double* d_Q);

/* Kernel family the instance runs (fixed at creation): *out = 0 generic any-K
 * kernels, 1 the 4-state kernels, 2 the matrix-core kernels (49..64 states
 * padded to 64, and 17..32 states padded to 32; FP32 or FP64; any number of
 * rate categories; under an HBM budget FP32 with one category). */
int epoch_get_kernel_path(EpochInstance* inst, int32_t* out);

/* Read back the transition matrices: host [2N-1][C][K][K] doubles (row-major,
 * entry v = branch above node v; root block left as zeros).  Requires
 * update_transition_matrices. */
int epoch_get_transition_matrices(EpochInstance* inst, double* out);

/* Per-phase device timing (tracing): when enabled, the library brackets each
 * phase with HIP events on the instance's stream and accumulates their elapsed
 * times.  Phases: 0 transition matrices, 1 post-order partials, 2 root
 * reduction, 3 pre-order + dlogL/dP accumulation, 4 gradient reduction and
 * dlogL/dl, 5 dlogL/dQ.  enable != 0 resets the accumulators. */
#define EPOCH_N_PHASES 6
int epoch_set_timing(EpochInstance* inst, int32_t enable);

/* Accumulated milliseconds and launch-group counts per phase, host [EPOCH_N_PHASES]
 * each (either may be NULL).  Synchronises the stream. */
int epoch_get_timing(EpochInstance* inst, double* ms_out, int64_t* counts_out);

/* Kernel-selection options of an instance (performance and rounding only:
 * every setting computes the same quantities).  Takes effect for the next evaluation; a key
 * that changes the schedule re-plans the current tree.
 *   EPOCH_OPT_TREE_WALK (fixed at 1 under hbm_budget_bytes): 1 = 4-state pruning and branch gradients as one
 *     traversal of the whole tree per tile of patterns; 0 = one launch per
 *     tree level; -1 (default) = the traversal for FP32 instances with at
 *     most 1024 tiles of 16 patterns (where per-level launches cannot fill the
 *     GPU), else per level.  dlogL/dQ always uses the level kernels.
 *   EPOCH_OPT_WALK_RECOMPUTE: value >= 2 (default 2): in the tree walk,
 *     internal nodes whose subtree holds at most this many tips are recomputed
 *     from tip states in the pre-order pass instead of being stored (2 when the
 *     instance has EPOCH_GRAD_Q).
 *   EPOCH_OPT_WALK_BLOCKS: value >= 0: cap on the blocks of a tree-walk launch
 *     (0 = one group of tiles per wavefront).
 *   EPOCH_OPT_WALK_TILES: 1 (default) or 2: FP32 pattern tiles carried
 *     together by one wavefront of the tree walk.
 *   EPOCH_OPT_LEVEL_MIN_TILES: 1..64 (default 8): fewest pattern tiles a
 *     wavefront of the 4-state pre-order level kernels walks; smaller values
 *     give narrow levels more wavefronts and more dlogL/dP partial sums.
 *   EPOCH_OPT_CHAIN_SPLIT: 0..2^30 (default 16): on the matrix-core P stage
 *     and dlogL/dQ chain, a branch whose ordered product has at least this many
 *     segments is computed as two halves in parallel and combined (the same
 *     quantities, rounded differently); 0 = never.
 *   EPOCH_OPT_TARGET_BLOCKS: 1..2^30 (default 1024): on the 64-state path,
 *     the blocks each tree-level launch aims for (it sets how many 64-pattern
 *     tiles a block walks, and so the number of dlogL/dP partial sums).
 *   EPOCH_OPT_INCREMENTAL: 0 or 1 (default 1): restricted re-evaluation after
 *     epoch_set_branch_rates / set_epoch_eigensystems (see below).
 *   EPOCH_OPT_SPLIT_BLOCKS: 0..2^30 (default 256): on the 64-state path, a
 *     pre-order tree level launched with at most this many blocks runs each
 *     child branch on its own wavefronts (same results, shorter per-wavefront
 *     work for levels too narrow to fill the GPU); 0 = never.
 *   EPOCH_OPT_EIGEN_PRECISION: 0, 1 or 2 (default 0), FP32 instances only:
 *     the arithmetic of the transition matrices V exp(r t Lambda) V^-1 and
 *     their ordered products (Eq. 6-7) and of the dlogL/dQ chains.  0 = FP64
 *     when some process's eigenvector matrix has infinity-norm condition
 *     number cond(V) = |V| |V^-1| above 32 (FP32 rounding of the
 *     reconstruction grows like cond(V) 2^-24), else FP32; 1 = FP32 always;
 *     2 = FP64 always.  The matrices are stored in FP32 either way.
 * Returns EPOCH_ERR_ARG for an unknown key or a value out of range. */
#define EPOCH_OPT_TREE_WALK 1
#define EPOCH_OPT_WALK_RECOMPUTE 2
#define EPOCH_OPT_WALK_BLOCKS 3
#define EPOCH_OPT_WALK_TILES 4
#define EPOCH_OPT_LEVEL_MIN_TILES 5
#define EPOCH_OPT_SPLIT_BLOCKS 6
#define EPOCH_OPT_TARGET_BLOCKS 7
#define EPOCH_OPT_CHAIN_SPLIT 8
#define EPOCH_OPT_INCREMENTAL 9
#define EPOCH_OPT_EIGEN_PRECISION 10
int epoch_set_option(EpochInstance* inst, int32_t key, int64_t value);

/* ---- Incremental re-evaluation for MCMC proposals (Introduction: the method
 * runs inside a Markov chain Monte Carlo sampler that proposes one change at a
 * time; Methods, "Coarse-grain parallel implementation": the front end tracks
 * which branches need new transition matrices).  The instance remembers which
 * branches changed since its last post-order pass: the listed branches of
 * epoch_set_branch_rates, and every branch with a stretch in an interval of
 * process s after set_epoch_eigensystems(s) (Eq. 6-7).  The next
 * update_transition_matrices / update_partials (or epoch_evaluate) then forms
 * only those branches' transition matrices and the partials of the nodes on
 * their paths to the root (Eq. 4: a partial depends on its subtree only); the
 * root log-likelihood and any gradient pass run in full.  Any other setter, a
 * new tree, an option or a batch evaluation makes the next evaluation full.
 * Restricted passes are taken by instances without EPOCH_GRAD_Q on the
 * 4-state level kernels, the 64-state kernels and the generic kernels when all
 * patterns are evaluated at once (not under an HBM budget, not on the tree
 * walk); otherwise the evaluation is full.  EPOCH_OPT_INCREMENTAL 0 turns the
 * restriction off (default 1).  Results equal a full evaluation, except that a
 * long epoch chain the full matrix-core P stage would cut into parts is formed
 * whole (different rounding). */

/* New rates r_v for the branches above nodes[0..n) (each > 0 and finite; an
 * entry for the root is ignored), as set_tree_epochs' branch_rate would give
 * them, without re-planning the tree.  Host arrays [n].  Needs the tree;
 * invalidates the transition matrices. */
int epoch_set_branch_rates(EpochInstance* inst, int32_t n, const int32_t* nodes, const double* rates);

/* Work of the last evaluation: out[0] = transition matrices (branch x category)
 * formed by the last P stage, out[1] = internal-node partials formed by the
 * last post-order pass (the 4-state kernels never store cherries).  Host [2]. */
int epoch_get_work_counts(EpochInstance* inst, int64_t* out);

/* ---- Batched evaluation (an addition to the paper: many independent
 * evaluations in one replayed HIP graph).
 * A batch references n distinct, fully set-up instances (eigensystems, tree,
 * tips, weights, categories, root frequencies); it does not own them and they
 * must outlive it.  Members on the 64-state path share merged per-level
 * launches; every other member's launches (and each member's dlogL/dQ) form
 * independent branches of the graph, which the GPU runs concurrently; a member's
 * results are the bits of its single evaluation.  The graph is captured at the
 * first evaluation and replayed, and
 * captured again when a member's tree or eigen-reconstruction precision
 * changes or epoch_set_option is called on a member.  tune_cache_path (or NULL) names a text file caching the tuned
 * launch shape per device and batch shape; it is read, and written after
 * tuning on the first evaluation. */
typedef struct EpochBatch EpochBatch;
int epoch_batch_create(EpochInstance* const* insts, int32_t n, const char* tune_cache_path, EpochBatch** out);

/* Evaluate every member: logL: host [n] out.  what: EPOCH_EVAL_* bits (logL
 * is always computed).  Gradients stay on the device; read them with
 * epoch_batch_gradients.  Synchronises the batch's own stream.  As for one
 * instance (root_log_likelihood): a member whose logL is -inf makes the call
 * return EPOCH_WARN_UNDERFLOW (every logL written) and has no gradient; a NaN
 * or +inf logL returns EPOCH_ERR_NUMERIC. */
int epoch_batch_evaluate(EpochBatch* batch, uint32_t what, double* logL);

/* Gradients of member i from the last evaluation (host arrays as in
 * log_likelihood_gradient; either may be NULL).  EPOCH_ERR_NUMERIC for a
 * member whose logL was -inf. */
int epoch_batch_gradients(EpochBatch* batch, int32_t i, double* d_branch, double* d_Q);

/* Tuned launch shape in use (for reporting): blocks each merged level launch
 * aims for, and the widest pre-order level (in blocks) that runs each child
 * branch on its own wavefronts (0 = none). */
int epoch_batch_target_blocks(EpochBatch* batch, int32_t* out);
int epoch_batch_split_blocks(EpochBatch* batch, int32_t* out);

int epoch_batch_destroy(EpochBatch* batch);

/* Attainable HBM bandwidth on the current device: a plain stream over a
 * library-allocated buffer of `bytes` (1 MiB .. 64 GiB), repeated `iters`
 * times on the default stream and timed with HIP events, for each of eight
 * launch shapes (grid-stride or block-contiguous ranges, 1,024 to 65,536
 * blocks); *gbs receives the best rate in GB/s (1e9 bytes per second).
 * kind: 0 = copy (counts read + write bytes), 1 = read-only, 2 = write-only.
 * Allocates and frees its own buffers. */
int epoch_bandwidth_probe(int64_t bytes, int32_t kind, int32_t iters, double* gbs);

/* For callers that cannot allocate device memory (code under HIP graph capture,
 * tight serving loops, harnesses that forbid hipMalloc): the FP64 eigensystem
 * check of set_epoch_eigensystems, for n_systems eigensystems at once, on device
 * memory the caller owns.  It calls no allocating routine and does not
 * synchronise: the kernels are enqueued on `stream` (a hipStream_t of the current
 * device, NULL = the default stream) and the residuals are ready when it completes.
 *   n_states K in [2, 64]; n_systems >= 1.
 *   V, Vinv: device [n_systems][K][K] row-major doubles; lambda_re: device
 *   [n_systems][K]; lambda_im: device [n_systems][K] or NULL (all real), complex
 *   pairs laid out as in set_epoch_eigensystems; Q: device [n_systems][K][K].
 *   residual: device [n_systems] out: max(max|V B V^-1 - Q| / max|Q|, max|V V^-1 - I|)
 *   per system, the value set_epoch_eigensystems reports for the same columns.
 * Every pointer must be device memory of the current device (EPOCH_ERR_ARG
 * otherwise, checked before any launch).  The per-tile maxima live in a fixed
 * 1 MiB device array per GPU (131072 doubles; a system of K states takes
 * 3 * ceil(K/16)^2 of them): more systems than fit in one call -> EPOCH_ERR_ARG.
 * Every row of that array a call reads is written by the same call first, so
 * nothing needs clearing; calls that overlap on one GPU (concurrent streams or
 * threads) share the array and race. */
int epoch_eigen_residual_noalloc(int32_t n_states, int32_t n_systems, const double* V, const double* Vinv,
                                 const double* lambda_re, const double* lambda_im, const double* Q,
                                 double* residual, void* stream);

/* Host planner only (no device work, usable without a GPU): the per-interval
 * segments of every branch, parent side first.
 *   seg_offset: host [2N] out (CSR offsets indexed by child node);
 *   seg_process, seg_time: host [capacity] out; *n_segments receives the total.
 * Returns EPOCH_ERR_ARG if capacity is too small (n_segments still set). */
int epoch_plan_segments(int32_t n_tips, const int32_t* parent, const double* height,
                        int32_t n_intervals, const double* boundaries,
                        const int32_t* interval_process, int32_t n_processes,
                        int32_t capacity, int32_t* seg_offset, int32_t* seg_process,
                        double* seg_time, int32_t* n_segments);

/* Host planner only (no device work, usable without a GPU): the two programs
 * of the 4-state tree walk for a tree (the pre-order pass that follows
 * Felsenstein's recursion, Eq. 4, down from the root).  parent/height as in
 * set_tree_epochs; recompute_tips >= 2.  ops: host [capacity][4] int32 out,
 * the post-order program followed by the pre-order program; counts: host [4]
 * out = {post ops, pre ops, post stack slots, pre stack slots}.  Each
 * operation is {info, a, b, u}: info bit 0 = pre-order operation, bit 1 =
 * root, bit 2 = store the partial, bits 3-4 / 5-6 = source of child a / b
 * (0 tip, 1 stored partial, 2 stack slot), bits 8-13 / 14-19 = stack slots of
 * a / b, bits 20-25 = output slot (post) or outside-vector slot (pre), bits
 * 26-31 = slot of q_b (pre); an output that nothing reads (the root's partial,
 * the outside vector of a tip) names the slot just past the program's slot
 * count.  Returns EPOCH_ERR_ARG if capacity is too small (counts still set) or
 * the tree needs more than 62 stack slots. */
int epoch_plan_walk(int32_t n_tips, const int32_t* parent, const double* height, int32_t recompute_tips,
                    int32_t capacity, int32_t* ops, int32_t* counts);

#ifdef __cplusplus
}
#endif

#endif /* EPOCHLIK_H */
