// Instance state shared by the ABI implementation and the kernel launchers.
#pragma once
#include <hip/hip_runtime.h>

#include <cstdint>
#include <string>
#include <vector>

#include "../../include/epochlik.h"
#include "planner.h"

namespace epochlik {

// One growable device allocation owned by the instance.
struct DevBuf {
  void* ptr = nullptr;
  size_t bytes = 0;
  bool borrowed = false;  // part of a caller-owned workspace: never freed or reallocated
};

// Device-visible description of one problem for the 64-state kernels (one
// instance, or one member of a batch).
struct CodonProblem {
  const float* Pm;
  const uint8_t* tips;
  float* part;
  float* pre;
  int32_t* scales;
  float* weightsT;         // FP32 pattern weights (with several categories: w_p times the category's posterior share)
  const double* weights;
  const double* pi;
  float* Gpart;
  const float* dPm;
  double* G;
  double* dbranch;
  double* site;
  double* blocksum;
  double* result;
  const int32_t* left;
  const int32_t* right;
  const uint64_t* amb;    // [256] state sets of the ambiguity codes K + 1 + a (bit j = state j)
  const int32_t* gslots;  // [2 n_nodes]: dlogL/dP partial slots written per branch, then each branch's first slot
  const double* cat;      // [2 kMaxCategories]: category rates, then weights
  int N, P, K, root, n_nodes;
  int tip_stride;         // row stride of tips (the instance's pattern count; P is this chunk's)
  int pm_stride;          // floats from one node's transition matrix (and G, dP) to the next: C x 64 x 64
  int cat_index, n_cats;  // this descriptor's rate category and the instance's category count; the
                          // descriptors of one instance's categories are consecutive, category 0 first
};

// Device pointers of one problem's P stage (one instance, or one member of a batch).
constexpr int kChainMaxParts = 8;  // parts a long epoch-product chain is cut into, at most

struct PStageDesc {
  const void* V;
  const void* Vi;
  const void* lr;
  const void* li;
  const int32_t* seg_offset;
  const int32_t* seg_process;
  const int4* items;           // work items (node, k0, k1, kind | slot << 2) of this launch, longest first
  void* scratch;               // per split, category and part: X_j, dX_j, prefix, suffix, suffix^T
  const double* seg_time;
  const double* seg_frac;
  const double* rate;
  const double* cat_rates;
  void* Pout;
  void* dPout;
  void* Ubuf;   // or null: A_k V of every segment term, kept for the dlogL/dQ adjoint chain
  int n_items;  // work items x categories
  int C;
  bool grad;
};

// Merged level schedule: work items (problem, internal node) grouped by level.
struct CodonSchedule {
  std::vector<int2> items;         // level l (1-based) occupies [level_off[l-1], level_off[l])
  std::vector<int> level_off;
  std::vector<int> level_R;        // 64-pattern tiles per block of the launches of each level
  std::vector<int2> reduce_items;  // every (problem, node)
  std::vector<size_t> slot_total;  // dlogL/dP partial slots of each problem
  std::vector<int> desc_inst, desc_cat;  // each problem's instance (index in the list given) and rate category
  int n_levels = 0, max_tiles = 0, max_pattern_blocks = 0, n_problems = 0;
  int split_blocks = 0;  // pre-order levels of at most this many blocks put each child branch on its own wavefronts
  bool amb = false;      // some problem has tips with ambiguity codes (the kernels' ambiguity instantiation)
  bool fp64 = false;     // FP64 problems (the FP64 matrix-core instantiation; every problem of a schedule alike)
  int nt = 4;            // 16-state tiles of the padded states: 4 (64 states) or 2 (32); every problem alike
};

// Incremental re-evaluation (MCMC proposals): the work of one restricted pass.
struct IncrementalPlan {
  std::vector<int32_t> pnodes;          // branches (child nodes) whose transition matrices are formed again
  std::vector<int4> chain_items;        // the same as whole-chain work items of the matrix-core P stage
  std::vector<int32_t> post_nodes;      // internal nodes whose partials are formed again, grouped by level
  std::vector<int32_t> post_level_off;  // [n_levels + 2]: level l occupies [off[l], off[l + 1])
  CodonSchedule codon;                  // the 64-state schedule restricted to post_nodes
  size_t off_chain = 0, off_post = 0, off_codon = 0;  // byte offsets in the device copy
};

}  // namespace epochlik

struct EpochInstance {
  EpochConfig cfg{};
  int N = 0, P = 0, K = 0, Kp = 0, C = 0, S = 0, n_nodes = 0, n_int = 0;
  bool fp64 = false;
  size_t real_size = 4;  // bytes of the compute type
  hipStream_t stream = nullptr;
  int device = 0;

  // host-side copies and validity flags
  std::vector<double> h_V, h_Vinv, h_lre, h_lim;  // padded [S][Kp][Kp], [S][Kp]
  std::vector<char> have_eig;
  bool any_complex = false;
  std::vector<double> cond;  // infinity-norm condition number of each V
  // FP32 instances reconstruct exp(tQ) from the eigensystem in FP64 when some
  // V is ill-conditioned (the FP32 rounding error grows like cond(V) * 2^-24).
  bool eig_fp64 = false;
  int eig_mode = 0;  // EPOCH_OPT_EIGEN_PRECISION
  double h_cat_rates[8] = {0}, h_cat_weights[8] = {0};
  bool have_tips = false, have_weights = false, have_cats = false, have_pi = false;
  bool have_tree = false;
  bool P_valid = false, partials_valid = false, logL_valid = false;
  bool logL_underflow = false;  // the last logL was -inf (EPOCH_WARN_UNDERFLOW): no gradient of this state
  bool grad_ready = false, gradQ_ready = false;  // gradients left on the device by a batch evaluation
  uint64_t tree_generation = 0;                   // bumped by set_tree_epochs
  uint64_t option_generation = 0;                 // bumped by every epoch_set_option call
  bool eig_dirty = true;
  epochlik::TreePlan plan;
  int n_chunks = 1;  // pattern chunks of the generic gradient accumulation
  int path = 0;        // 0 generic, 1 four-state kernels, 2 64-state MFMA kernels
  int nuc_rmin = 8;    // minimum pattern tiles per wavefront in the four-state gradient
  int nuc_slots = 1;   // partial-sum slots per branch of the four-state gradient
  std::vector<int> nuc_fuse;   // per level: pre-order nodes with a cherry child (listed first in nuc_nodes)
  epochlik::DevBuf nuc_nodes;  // int32 [N-1]: level order of the four-state pre-order launches
  // four-state tree-walk kernels (kernels_walk.hip)
  int walk_enable = -1;        // tree-walk kernels for the 4-state pruning and branch gradients: 1 on, 0 off,
                               // -1 when the level kernels cannot fill the GPU (FP32, at most kWalkAutoTiles tiles)
  int walk_recompute = 2;      // subtrees with at most this many tips are recomputed, not stored
  int walk_blocks = 0;         // > 0: cap on the blocks of a walk launch (tiles are then strided)
  int walk_nt = 1;             // FP32: pattern tiles per wavefront (1 or 2)
  bool walk_ok = false;        // programs built for the current tree
  bool walk_pre_ok = false;    // the pre-order program's LDS fits (else the level kernels take the gradient)
  epochlik::WalkProgram walk;
  epochlik::DevBuf walk_ops;   // int4 post-order program, then pre-order program
  epochlik::DevBuf walk_tcol;  // T [2][N][C][5][4] columns of the tip branches' P and dP/dl
  epochlik::DevBuf walk_dpart; // T [tile groups][n_nodes] shares of dlogL/dl, then double [32][n_nodes]
  epochlik::DevBuf walk_dummy; // stand-in operands of the walk kernels (never read back)
  epochlik::DevBuf walk_slots; // int32 [n_nodes]: partial slot of each stored node (-1: not stored)
  int64_t budget = 0;          // hbm_budget_bytes (0: every internal node has a slot, slot = node - N)
  int root_slot = 0;           // partial slot of the root; its scale exponents are scales row root_slot

  // device buffers (compute type T unless noted)
  epochlik::DevBuf eigT;       // V[S][Kp][Kp], Vinv[S][Kp][Kp], lre[S][Kp], lim[S][Kp]
  epochlik::DevBuf eig64;      // the same in double
  epochlik::DevBuf eigTT;      // V^T[S][Kp][Kp], (V^-1)^T[S][Kp][Kp] in the compute type
  epochlik::DevBuf eig64T;     // the same in double
  epochlik::DevBuf check;      // double scratch for the eigen check
  epochlik::DevBuf tips;       // uint8 [N][P]: state codes (4-state kernels: state sets, bit i = state i)
  epochlik::DevBuf amb;        // uint64 [256]: state sets of the ambiguity codes K + 1 .. K + n_amb
  std::vector<uint64_t> h_amb; // the same on the host (n_amb entries)
  bool tips_amb = false;       // some tip state is an ambiguity code
  epochlik::DevBuf weights;    // double [P]
  epochlik::DevBuf weightsT;   // T [P]
  epochlik::DevBuf pi;         // double [Kp]
  epochlik::DevBuf cat;        // double rates[8], weights[8]
  epochlik::DevBuf tree_i;     // int32: parent, left, right [n], level_nodes [N-1], seg_offset [n+1], seg_process [nseg]
  epochlik::DevBuf tree_d;     // double: rate [n], tau [n], seg_time [nseg], seg_frac [nseg]
  epochlik::DevBuf Pm;         // T [n][C][Kp][Kp]
  epochlik::DevBuf dPm;        // T [n][C][Kp][Kp]
  epochlik::DevBuf partials;   // T [N-1][C][P][Kp]
  epochlik::DevBuf scales;     // int32 [N-1][P]
  epochlik::DevBuf pre;        // T [N-1][C][P][Kp]
  epochlik::DevBuf site;       // double [P]
  epochlik::DevBuf blocksum;   // double [ceil(P/256)+1]
  epochlik::DevBuf result;     // double [4]
  epochlik::DevBuf Gpart;      // double [chunks][n][C][Kp][Kp]
  epochlik::DevBuf G;          // double [n][C][Kp][Kp]
  epochlik::DevBuf dbranch;    // double [n]
  epochlik::DevBuf qseg;       // double complex per segment [nseg][C][Kp][Kp][2]
  epochlik::DevBuf qscratch;   // T prefix products [nseg][C][Kp][Kp]
  // matrix-core chains: work items (node, first segment, end segment, info), longest first:
  // [whole list: one per node][split list: long chains cut into parts][per split: node, m, parts, slot];
  // info = kind (0 whole, 1 part) | part << 2 | parts << 5 | slot << 9
  epochlik::DevBuf chain_items;
  // per split, category and part: X_j, dX_j, prefix X_0..X_{j-1}, suffix X_{j+1}..X_{J-1} and its
  // transpose [Kp][Kp] (compute type)
  epochlik::DevBuf chain_scratch;
  int n_chain_split_items = 0, n_chain_splits = 0, chain_max_tail = 0;
  int chain_split_min = 16;        // chains of at least this many segments are cut in two (0: never)
  bool pstage_split = false;       // the last P stage launched ran the split items (the dQ chain follows it)
  epochlik::DevBuf dQ;         // double [S][Kp][Kp]
  epochlik::DevBuf qtau;       // double [nseg][C] tau of each segment term of dlogL/dQ, then complex [nseg][C][Kp] e^{tau lambda}
  int q_chunks = 1;            // segment chunks per process of the dlogL/dQ sums
  int q_chunk_items = 32;      // segment terms per chunk
  epochlik::DevBuf seglist;    // int32 segments grouped by process: offsets [S+1], items [nseg*C]
  epochlik::DevBuf gslots;     // int32 [n]: partial-sum slots written per branch (4-state / 64-state gradient)
  epochlik::DevBuf codon_dev;  // 64-state path: descriptor + work items
  epochlik::DevBuf codon_aux;  // 64-state path: per-chunk shares of dlogL/dl (double)
  epochlik::CodonSchedule codon_sched;
  int codon_target_blocks = 1024;  // blocks per pre-order launch the 64-state schedule aims for
  int codon_pc = 0;                // 64-state path under an HBM budget: patterns per chunk (0: all at once)
  int codon_nchunks = 1;           // pattern chunks evaluated one after another
  int gen_pc = 0;                  // generic path under an HBM budget: patterns per chunk (0: all at once)
  int gen_nchunks = 1;
  // the pattern chunk the generic launches work on (view_P == 0: all patterns)
  int view_P = 0, view_p0 = 0, view_j = 0;
  bool view_accumulate = false;    // dlogL/dP of this chunk adds to the earlier chunks
  int codon_split_blocks = 256;    // narrow pre-order levels (at most this many blocks) use the side-split kernel

  // incremental re-evaluation (epoch_set_branch_rates, set_epoch_eigensystems on one process)
  int inc_enable = 1;              // EPOCH_OPT_INCREMENTAL
  bool dirty_all = true;           // every transition matrix and partial must be formed again
  bool inc_base = false;           // the partials hold a complete post-order pass (the state changes apply to)
  bool inc_active = false;         // the last P stage was restricted: the post-order pass follows it
  std::vector<uint8_t> dirty;      // [n_nodes]: the branch above the node changed since the last post-order pass
  epochlik::IncrementalPlan inc;
  epochlik::DevBuf inc_dev;        // device copy of the restricted lists
  int64_t work_P = 0, work_partials = 0;  // matrices and node partials formed by the last P stage / post-order pass

  // node-height and boundary gradients (EPOCH_GRAD_TIME)
  epochlik::DevBuf tg_i;           // int32 process above / below each node, crossing offsets, phi; int4 crossings
  epochlik::DevBuf tg_d;           // double Q_s, end terms, crossing terms, outputs, scratch
  size_t tg_cross_offset = 0;      // byte offset of the crossings in tg_i
  int tg_n_cross = 0, tg_n_bound = 0;
  uint64_t eval_gen = 0;           // bumped by every post-order pass and root reduction
  uint64_t G_gen = ~0ull;          // eval_gen of the last gradient pass (the branch adjoints G on the device)

  // per-phase timing (epoch_set_timing)
  bool timing = false;
  hipEvent_t ev[EPOCH_N_PHASES][2] = {};
  // pinned staging of set_epoch_eigensystems' copies (enqueued without waiting)
  void* stage_host = nullptr;
  size_t stage_bytes = 0;
  hipEvent_t stage_event = nullptr;
  bool stage_pending = false;
  bool ev_pending[EPOCH_N_PHASES] = {};
  double phase_ms[EPOCH_N_PHASES] = {};
  int64_t phase_count[EPOCH_N_PHASES] = {};

  // device pointers into tree_i / tree_d
  int32_t *d_parent = nullptr, *d_left = nullptr, *d_right = nullptr, *d_level_nodes = nullptr,
          *d_seg_offset = nullptr, *d_seg_process = nullptr;
  double *d_rate = nullptr, *d_tau = nullptr, *d_seg_time = nullptr, *d_seg_frac = nullptr;
};

namespace epochlik {

// incremental re-evaluation (incremental.hip)
void mark_dirty_all(EpochInstance* in);
void mark_dirty_process(EpochInstance* in, int s);
bool incremental_eligible(const EpochInstance* in);
int launch_pstage_incremental(EpochInstance* in);  // builds the restricted lists, forms the dirty branches' P
int launch_post_incremental(EpochInstance* in);    // partials of the dirty branches' ancestors
void incremental_done(EpochInstance* in);           // after a complete post-order pass

// phase timing brackets (no-ops unless timing is enabled)
int phase_begin(EpochInstance* in, int phase);
int phase_end(EpochInstance* in, int phase);

// error helpers (thread-local message)
int set_error(int code, const char* fmt, ...);
int hip_check(hipError_t e, const char* what);

// grows a device buffer (contents not preserved); returns EPOCH_OK or an error code
int ensure(DevBuf& b, size_t bytes);

// kernel launchers (kernels_generic.hip); all return EPOCH_OK or an error code
// FP64 eigensystem check (kernels_eigcheck.hip): d_out[0] receives the residual, scratch follows it
int launch_eigen_check(EpochInstance* in, int s, const double* dQ, double* d_out);
int eigen_check_tiles(int K);  // scratch rows (3 doubles each) per system
int launch_q_reconstruct(EpochInstance* in, double* d_Q, double* part);  // Q_s = V B V^-1, FP64 [S][Kp][Kp]
// node-height and boundary gradients (kernels_tgrad.hip)
int tgrad_prepare(EpochInstance* in);
int launch_time_gradient(EpochInstance* in, double** d_height, double** d_bound);
int launch_eigen_check_n(hipStream_t st, int K, int n, int ld, long mat_stride, int vec_stride, const double* V,
                         const double* Vi, const double* lr, const double* li, const double* Q, double* part,
                         double* out);
int launch_pstage_generic(EpochInstance* in);
int launch_pstage_generic_nodes(EpochInstance* in, const int32_t* d_nodes, int n);  // listed branches only
int launch_post_generic_nodes(EpochInstance* in, const int32_t* d_nodes, const int32_t* level_off);
int launch_pstage_mfma_items(EpochInstance* in, const int4* d_items, int n_items);  // whole chains listed
int launch_pstage_mfma(EpochInstance* in);
bool pstage_mfma_supported(const EpochInstance* in);
int launch_pstage(EpochInstance* in);  // matrix-core kernel where it applies, else generic
PStageDesc pstage_descriptor(const EpochInstance* in);
int launch_pstage_mfma_multi(const EpochInstance* like, const PStageDesc* d_descs, int n, int max_items,
                             hipStream_t st);
int launch_grad_Q_mfma(EpochInstance* in);
bool grad_Q_mfma_supported(const EpochInstance* in);
int launch_grad_Q(EpochInstance* in);  // matrix-core kernels where they apply, else generic
int launch_post_generic(EpochInstance* in);
int launch_root_generic(EpochInstance* in);
int launch_pre_generic(EpochInstance* in);
int launch_grad_branch_generic(EpochInstance* in);
int launch_grad_Q_generic(EpochInstance* in);
int launch_final_sum(EpochInstance* in, int n_blocks);
int launch_chunk_sum(EpochInstance* in, int n);  // result[0] = result[1] + ... + result[n], in order
int launch_grad_reduce(EpochInstance* in, int n_chunks, const int32_t* chunks_per_node);

// 4-state kernels (kernels_nuc.hip)
int launch_nuc_post(EpochInstance* in);
int launch_nuc_post_nodes(EpochInstance* in, const int32_t* d_nodes, const int32_t* level_off);
int launch_nuc_root(EpochInstance* in);
int launch_nuc_pre_grad(EpochInstance* in);
int nuc_slots(int P, int C, int rmin);
void nuc_pre_order_nodes(const EpochInstance* in, std::vector<int32_t>& nodes, std::vector<int>& fuse);
void nuc_slots_per_node(const EpochInstance* in, const std::vector<int32_t>& nodes, const std::vector<int>& fuse,
                        std::vector<int32_t>& out);

// 4-state tree-walk kernels (kernels_walk.hip)
int walk_prepare(EpochInstance* in);  // builds and uploads the programs (walk_ok)
int walk_tiles(const EpochInstance* in);
size_t walk_tcol_bytes(const EpochInstance* in);
size_t walk_dpart_rows_bytes(const EpochInstance* in);
int launch_walk_tipcol(EpochInstance* in);
int launch_walk_post(EpochInstance* in);
int launch_walk_pre_grad(EpochInstance* in);

// 64-state MFMA kernels (kernels_codon.hip)
int launch_codon_post(EpochInstance* in);
int launch_codon_post_schedule(EpochInstance* in, const CodonSchedule& sc, const int2* d_items);
int launch_codon_root(EpochInstance* in);
int launch_codon_pre_grad(EpochInstance* in);
int codon_prepare(EpochInstance* in);
CodonProblem codon_descriptor(const EpochInstance* in, int c, const int32_t* gslots, float* gpart);
constexpr size_t kCodonSlotBytes = 64 * 64 * sizeof(float);  // one FP32 64x64 partial of dlogL/dP (FP64: twice)
void codon_build_schedule(const std::vector<const EpochInstance*>& insts, int target_blocks, CodonSchedule& out,
                          std::vector<std::vector<int32_t>>& gslots);
int codon_launch_post(const CodonSchedule& sc, const CodonProblem* d_probs, const int2* d_items, hipStream_t st);
int codon_launch_root(const CodonSchedule& sc, const CodonProblem* d_probs, hipStream_t st);
size_t codon_dpart_bytes(const CodonSchedule& sc);
int codon_launch_pre_grad(const CodonSchedule& sc, const CodonProblem* d_probs, const int2* d_items,
                          const int2* d_reduce_items, double* dpart, hipStream_t st, bool accumulate, bool finish);

}  // namespace epochlik
