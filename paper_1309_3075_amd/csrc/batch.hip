// Batched evaluation: many independent likelihood problems in one replayed
// HIP graph.
//
// Problems on the 64-state MFMA path share merged launches: one launch per
// tree level (counted from the tips) carries the nodes of that level of every
// problem as (problem, node) work items, so small problems do not leave the
// chip idle.  Transition matrices and dlogL/dQ are launched per problem inside
// the same graph.  The graph is captured on the first evaluation and replayed
// afterwards; it is captured again when a tree topology (level structure) or
// the precision of the eigen reconstruction of a member changes.  The number
// of blocks each pre-order launch aims for is tuned on the device the first
// time a shape is seen and kept in a JSON cache file.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <limits>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <fstream>
#include <sstream>
#include <string>
#include <vector>

#include "fastpath.h"
#include "instance.h"

using namespace epochlik;

struct EpochBatch {
  std::vector<EpochInstance*> insts;
  hipStream_t stream = nullptr;
  bool merged = false;  // every member is on the 64-state path
  int target_blocks = 1024;
  int split_blocks = 256;  // narrow pre-order levels use the side-split kernel
  std::string tune_path;
  CodonSchedule sched;
  DevBuf dev;                  // descriptors + items + reduce items
  std::vector<DevBuf> gslots;  // per member
  DevBuf gpart;                // dlogL/dP slot partials of every member
  DevBuf dpart;                // per-chunk shares of dlogL/dl
  DevBuf results;              // double [n]
  // P-stage groups: members sharing Kp, precision, eigen arithmetic and gradient flag run in one launch
  struct PGroup {
    std::vector<size_t> members;
    int max_items = 0;
    size_t desc_offset = 0;  // index of the group's first descriptor in pdescs
  };
  std::vector<PGroup> pgroups;
  std::vector<size_t> p_single;  // members that run their own P stage (generic, or a matrix-core group of one)
  DevBuf pdescs;
  std::vector<uint64_t> signature;
  hipGraph_t graph[8] = {};
  hipGraphExec_t exec[8] = {};
  bool tuned = false;
  bool own_stream = false;
  // branch streams of the captured graph: members whose launches are their own (not the
  // merged levels) run on kBatchBranches streams forked from and joined back to `stream`
  static constexpr int kBatchBranches = 16;
  hipStream_t branch[kBatchBranches] = {};
  hipEvent_t fork_ev = nullptr;
  hipEvent_t join_ev[kBatchBranches] = {};
};

namespace {

constexpr uint32_t kLogL = 1u, kGradBranch = 2u, kGradQ = 4u;

__global__ __launch_bounds__(64) void gather_results(const double* const* __restrict__ src, int n,
                                                     double* __restrict__ dst) {
  for (int i = threadIdx.x; i < n; i += 64) dst[i] = *src[i];
}

uint64_t member_signature(const EpochInstance* in) {
  uint64_t h = (uint64_t)in->tree_generation * 1000003ull + (in->eig_fp64 ? 7 : 0) + (in->tips_amb ? 11 : 0);
  return h ^ (in->option_generation * 0x9E3779B97F4A7C15ull);
}

void release_buf(DevBuf& b) {
  if (b.ptr) (void)hipFree(b.ptr);
  b.ptr = nullptr;
  b.bytes = 0;
}

void drop_graphs(EpochBatch* b) {
  for (int k = 0; k < 8; ++k) {
    if (b->exec[k]) (void)hipGraphExecDestroy(b->exec[k]);
    if (b->graph[k]) (void)hipGraphDestroy(b->graph[k]);
    b->exec[k] = nullptr;
    b->graph[k] = nullptr;
  }
}

// Group the members' P stages by kernel instantiation and upload their descriptors.
int build_pstage_groups(EpochBatch* b) {
  b->pgroups.clear();
  b->p_single.clear();
  std::vector<int> key_of(b->insts.size(), -1);
  std::vector<std::vector<int>> keys;  // Kp, fp64, eig_fp64, grad
  for (size_t q = 0; q < b->insts.size(); ++q) {
    const EpochInstance* in = b->insts[q];
    if (in->cfg.kernel_path != EPOCH_KERNEL_AUTO || !pstage_mfma_supported(in)) {
      b->p_single.push_back(q);
      continue;
    }
    const std::vector<int> k = {in->Kp, in->fp64 ? 1 : 0, in->eig_fp64 ? 1 : 0,
                                (in->cfg.flags & (EPOCH_GRAD_BRANCH | EPOCH_GRAD_Q)) ? 1 : 0};
    size_t g = 0;
    while (g < keys.size() && keys[g] != k) ++g;
    if (g == keys.size()) {
      keys.push_back(k);
      b->pgroups.emplace_back();
    }
    b->pgroups[g].members.push_back(q);
    b->pgroups[g].max_items = std::max(b->pgroups[g].max_items, in->n_nodes * in->C);
  }
  // A group of one gains nothing from the shared launch, which runs whole chains:
  // that member runs its own P stage, with long epoch chains split into parts.
  for (size_t g = b->pgroups.size(); g-- > 0;)
    if (b->pgroups[g].members.size() == 1) {
      b->p_single.push_back(b->pgroups[g].members[0]);
      b->pgroups.erase(b->pgroups.begin() + g);
    }
  std::vector<PStageDesc> descs;
  for (auto& g : b->pgroups) {
    g.desc_offset = descs.size();
    for (size_t q : g.members) descs.push_back(pstage_descriptor(b->insts[q]));
  }
  if (descs.empty()) return EPOCH_OK;
  int rc = ensure(b->pdescs, descs.size() * sizeof(PStageDesc));
  if (rc) return rc;
  return hip_check(hipMemcpy(b->pdescs.ptr, descs.data(), descs.size() * sizeof(PStageDesc), hipMemcpyHostToDevice),
                   "batch P-stage descriptors");
}

int build_schedule(EpochBatch* b) {
  std::vector<const EpochInstance*> cin(b->insts.begin(), b->insts.end());
  std::vector<std::vector<int32_t>> gs;
  codon_build_schedule(cin, b->target_blocks, b->sched, gs);
  b->sched.split_blocks = b->split_blocks;
  const auto& sc = b->sched;
  const size_t n = (size_t)sc.n_problems;  // one problem per member and rate category
  size_t total = 0;
  for (size_t q = 0; q < n; ++q) total += sc.slot_total[q];
  const size_t slot_floats = (size_t)(16 * sc.nt) * (16 * sc.nt) * (sc.fp64 ? 2 : 1);  // one slot, in floats
  int rc0 = ensure(b->gpart, std::max<size_t>(1, total) * slot_floats * sizeof(float));
  if (!rc0) rc0 = ensure(b->dpart, codon_dpart_bytes(sc));
  if (rc0) return rc0;
  b->gslots.resize(n);
  std::vector<CodonProblem> desc(n);
  size_t off = 0;
  for (size_t q = 0; q < n; ++q) {
    int rc = ensure(b->gslots[q], gs[q].size() * sizeof(int32_t));
    if (rc) return rc;
    rc = hip_check(hipMemcpy(b->gslots[q].ptr, gs[q].data(), gs[q].size() * sizeof(int32_t), hipMemcpyHostToDevice),
                   "batch gslots upload");
    if (rc) return rc;
    float* region = static_cast<float*>(b->gpart.ptr) + off * slot_floats;
    desc[q] = codon_descriptor(b->insts[sc.desc_inst[q]], sc.desc_cat[q], static_cast<const int32_t*>(b->gslots[q].ptr),
                               region);
    off += sc.slot_total[q];
  }
  const size_t bytes = sizeof(CodonProblem) * n + sizeof(int2) * (sc.items.size() + sc.reduce_items.size());
  int rc = ensure(b->dev, bytes);
  if (rc) return rc;
  std::vector<char> h(bytes);
  memcpy(h.data(), desc.data(), sizeof(CodonProblem) * n);
  memcpy(h.data() + sizeof(CodonProblem) * n, sc.items.data(), sizeof(int2) * sc.items.size());
  memcpy(h.data() + sizeof(CodonProblem) * n + sizeof(int2) * sc.items.size(), sc.reduce_items.data(),
         sizeof(int2) * sc.reduce_items.size());
  return hip_check(hipMemcpy(b->dev.ptr, h.data(), bytes, hipMemcpyHostToDevice), "batch schedule upload");
}

int ensure_branches(EpochBatch* b) {
  for (int k = 0; k < EpochBatch::kBatchBranches; ++k) {
    if (!b->branch[k] && hipStreamCreateWithFlags(&b->branch[k], hipStreamNonBlocking) != hipSuccess) {
      b->branch[k] = nullptr;
      return set_error(EPOCH_ERR_HIP, "batch branch stream creation failed");
    }
    if (!b->join_ev[k] && hipEventCreateWithFlags(&b->join_ev[k], hipEventDisableTiming) != hipSuccess) {
      b->join_ev[k] = nullptr;
      return set_error(EPOCH_ERR_HIP, "batch event creation failed");
    }
  }
  if (!b->fork_ev && hipEventCreateWithFlags(&b->fork_ev, hipEventDisableTiming) != hipSuccess) {
    b->fork_ev = nullptr;
    return set_error(EPOCH_ERR_HIP, "batch event creation failed");
  }
  return EPOCH_OK;
}

// fn(q) for every member q in qs, member i of the list on branch stream i mod kBatchBranches (its
// launches go to in->stream), after everything already on b->stream; b->stream then waits for
// every branch.  Members touch only their own buffers, so the branches are independent.
template <typename F>
int fork_join(EpochBatch* b, const std::vector<size_t>& qs, F fn) {
  if (qs.empty()) return EPOCH_OK;
  const int K = (int)std::min<size_t>(EpochBatch::kBatchBranches, qs.size());
  int rc = hip_check(hipEventRecord(b->fork_ev, b->stream), "batch fork");
  for (int k = 0; k < K && !rc; ++k) rc = hip_check(hipStreamWaitEvent(b->branch[k], b->fork_ev, 0), "batch fork");
  for (size_t i = 0; i < qs.size() && !rc; ++i) {
    EpochInstance* in = b->insts[qs[i]];
    const hipStream_t own = in->stream;
    in->stream = b->branch[i % K];
    rc = fn(qs[i]);
    in->stream = own;
  }
  for (int k = 0; k < K; ++k) {  // join every forked branch, also after a failure (a capture must end joined)
    int r = hip_check(hipEventRecord(b->join_ev[k], b->branch[k]), "batch join");
    if (!r) r = hip_check(hipStreamWaitEvent(b->stream, b->join_ev[k], 0), "batch join");
    if (!rc) rc = r;
  }
  return rc;
}

// Enqueue one evaluation of every member on b->stream (no host synchronisation).
int enqueue(EpochBatch* b, uint32_t what, const double* const* d_result_ptrs) {
  const size_t n = b->insts.size();
  for (const auto& g : b->pgroups) {
    int rc = launch_pstage_mfma_multi(b->insts[g.members[0]], static_cast<const PStageDesc*>(b->pdescs.ptr) + g.desc_offset,
                                      (int)g.members.size(), g.max_items, b->stream);
    if (rc) return rc;
    for (size_t q : g.members) b->insts[q]->pstage_split = false;  // whole chains: the dQ chains follow suit
  }
  const bool grad = (what & (kGradBranch | kGradQ)) != 0;
  if (!b->merged) {
    // every member on its own: P stage (unless its group ran above), partials, root and gradient
    // on one branch, the members spread over the branches
    std::vector<bool> single(n, false);
    for (size_t q : b->p_single) single[q] = true;
    std::vector<size_t> all(n);
    for (size_t q = 0; q < n; ++q) all[q] = q;
    int rc = fork_join(b, all, [&](size_t q) {
      EpochInstance* in = b->insts[q];
      int r = single[q] ? launch_pstage(in) : EPOCH_OK;
      if (!r && single[q]) r = fastpath_after_pstage(in);
      if (!r) r = fastpath_post(in);
      if (!r) r = fastpath_root(in);
      if (!r && grad) r = fastpath_gradient(in, (what & kGradQ) != 0);
      return r;
    });
    if (rc) return rc;
    hipLaunchKernelGGL(gather_results, dim3(1), dim3(64), 0, b->stream, d_result_ptrs, (int)n,
                       static_cast<double*>(b->results.ptr));
    return hip_check(hipGetLastError(), "batch gather launch");
  }
  {
    int rc = fork_join(b, b->p_single, [&](size_t q) {
      int r = launch_pstage(b->insts[q]);
      return r ? r : fastpath_after_pstage(b->insts[q]);
    });
    if (rc) return rc;
  }
  if (b->merged && (what & (kGradBranch | kGradQ))) {
    // the gradient launches write through these buffers: refuse a capture without them
    for (size_t q = 0; q < n; ++q) {
      const EpochInstance* in = b->insts[q];
      if (!in->pre.ptr || !in->dPm.ptr || !in->G.ptr || !in->dbranch.ptr)
        return set_error(EPOCH_ERR_STATE, "batch member %zu has no gradient buffers", q);
    }
  }
  if (b->merged) {
    const CodonProblem* probs = static_cast<const CodonProblem*>(b->dev.ptr);
    const int2* items = reinterpret_cast<const int2*>(static_cast<const char*>(b->dev.ptr) +
                                                      sizeof(CodonProblem) * b->sched.n_problems);
    const int2* red = items + b->sched.items.size();
    int rc = codon_launch_post(b->sched, probs, items, b->stream);
    if (!rc) rc = codon_launch_root(b->sched, probs, b->stream);
    if (!rc && (what & (kGradBranch | kGradQ))) rc = codon_launch_pre_grad(b->sched, probs, items, red, static_cast<double*>(b->dpart.ptr), b->stream, false, true);
    if (rc) return rc;
  }
  if (what & kGradQ) {  // dlogL/dQ of each member, on the branches
    std::vector<size_t> all(n);
    for (size_t q = 0; q < n; ++q) all[q] = q;
    int rc = fork_join(b, all, [&](size_t q) { return launch_grad_Q(b->insts[q]); });
    if (rc) return rc;
  }
  hipLaunchKernelGGL(gather_results, dim3(1), dim3(64), 0, b->stream, d_result_ptrs, (int)n,
                     static_cast<double*>(b->results.ptr));
  return hip_check(hipGetLastError(), "batch gather launch");
}

int check_members(EpochBatch* b, uint32_t what) {
  for (size_t q = 0; q < b->insts.size(); ++q) {
    EpochInstance* in = b->insts[q];
    if (!in->have_tree || !in->have_cats || !in->have_tips || !in->have_weights || !in->have_pi)
      return set_error(EPOCH_ERR_STATE, "batch member %zu is missing inputs", q);
    for (int s = 0; s < in->S; ++s)
      if (!in->have_eig[s]) return set_error(EPOCH_ERR_STATE, "batch member %zu: eigensystem %d not set", q, s);
    if ((what & kGradBranch) && !(in->cfg.flags & EPOCH_GRAD_BRANCH))
      return set_error(EPOCH_ERR_STATE, "batch member %zu created without EPOCH_GRAD_BRANCH", q);
    if ((what & kGradQ) && !(in->cfg.flags & EPOCH_GRAD_Q))
      return set_error(EPOCH_ERR_STATE, "batch member %zu created without EPOCH_GRAD_Q", q);
  }
  return EPOCH_OK;
}

int capture(EpochBatch* b, uint32_t what) {
  const size_t n = b->insts.size();
  // pointers to every member's result[0], kept after the results array
  int rc = ensure(b->results, n * sizeof(double) + n * sizeof(double*));
  if (rc) return rc;
  std::vector<const double*> ptrs(n);
  for (size_t q = 0; q < n; ++q) ptrs[q] = static_cast<const double*>(b->insts[q]->result.ptr);
  const double** d_ptrs = reinterpret_cast<const double**>(static_cast<char*>(b->results.ptr) + n * sizeof(double));
  rc = hip_check(hipMemcpy(d_ptrs, ptrs.data(), n * sizeof(double*), hipMemcpyHostToDevice), "batch pointers");
  if (rc) return rc;
  // members launch on the batch stream while captured, without phase timing
  std::vector<hipStream_t> saved(n);
  std::vector<bool> timing(n);
  for (size_t q = 0; q < n; ++q) {
    saved[q] = b->insts[q]->stream;
    timing[q] = b->insts[q]->timing;
    b->insts[q]->stream = b->stream;
    b->insts[q]->timing = false;
  }
  rc = ensure_branches(b);
  if (rc) return rc;
  rc = hip_check(hipStreamBeginCapture(b->stream, hipStreamCaptureModeThreadLocal), "begin capture");
  if (!rc) {
    int erc = enqueue(b, what, d_ptrs);
    hipGraph_t g = nullptr;
    int crc = hip_check(hipStreamEndCapture(b->stream, &g), "end capture");
    rc = erc ? erc : crc;
    if (!rc) {
      rc = hip_check(hipGraphInstantiate(&b->exec[what], g, nullptr, nullptr, 0), "graph instantiate");
      b->graph[what] = g;
    } else if (g) {
      (void)hipGraphDestroy(g);
    }
  }
  for (size_t q = 0; q < n; ++q) {
    b->insts[q]->stream = saved[q];
    b->insts[q]->timing = timing[q];
  }
  return rc;
}

int replay(EpochBatch* b, uint32_t what) {
  std::vector<uint64_t> sig;
  for (auto* in : b->insts) sig.push_back(member_signature(in));
  if (sig != b->signature) {
    drop_graphs(b);
    int rc = build_pstage_groups(b);
    if (rc) return rc;
    if (b->merged) {
      rc = build_schedule(b);
      if (rc) return rc;
    }
    b->signature = sig;
  }
  if (!b->exec[what]) {
    int rc = capture(b, what);
    if (rc) return rc;
  }
  return hip_check(hipGraphLaunch(b->exec[what], b->stream), "graph launch");
}

// ---- tuning cache: lines "key value" in a small text/JSON-like file
std::string tune_key(EpochBatch* b) {
  hipDeviceProp_t prop;
  std::string arch = "unknown";
  if (hipGetDeviceProperties(&prop, b->insts[0]->device) == hipSuccess) arch = prop.gcnArchName;
  long tot_p = 0, tot_c = 0;
  for (auto* in : b->insts) {
    tot_p += in->P;
    tot_c += in->C;
  }
  std::ostringstream k;
  k << arch.substr(0, arch.find(':')) << "/codon/K" << b->insts[0]->K << (b->insts[0]->fp64 ? "/fp64" : "/fp32")
    << "/n" << b->insts.size() << "/P"
    << (tot_p / (long)b->insts.size() / 1000);
  if (tot_c != (long)b->insts.size()) k << "/C" << tot_c;  // rate categories multiply the work
  return k.str();
}

bool tune_lookup(const std::string& path, const std::string& key, int& value) {
  std::ifstream f(path);
  if (!f) return false;
  std::string line;
  while (std::getline(f, line)) {
    // format: "key": value,
    const size_t q1 = line.find('"'), q2 = line.find('"', q1 + 1);
    if (q1 == std::string::npos || q2 == std::string::npos) continue;
    if (line.substr(q1 + 1, q2 - q1 - 1) != key) continue;
    const size_t c = line.find(':', q2);
    if (c == std::string::npos) continue;
    value = atoi(line.c_str() + c + 1);
    return value > 0;
  }
  return false;
}

void tune_store(const std::string& path, const std::string& key, int value) {
  std::vector<std::string> entries;
  {
    std::ifstream f(path);
    std::string line;
    while (f && std::getline(f, line)) {
      const size_t q1 = line.find('"'), q2 = line.find('"', q1 + 1);
      if (q1 == std::string::npos || q2 == std::string::npos) continue;
      if (line.substr(q1 + 1, q2 - q1 - 1) == key) continue;
      std::string e = line;
      while (!e.empty() && (e.back() == ',' || e.back() == ' ')) e.pop_back();
      entries.push_back(e);
    }
  }
  std::ostringstream e;
  e << "  \"" << key << "\": " << value;
  entries.push_back(e.str());
  std::ofstream f(path);
  f << "{\n";
  for (size_t i = 0; i < entries.size(); ++i) f << entries[i] << (i + 1 < entries.size() ? ",\n" : "\n");
  f << "}\n";
}

// Timed replays of one launch shape (warm-up and capture first); ms of 3 replays.
int time_shape(EpochBatch* b, uint32_t what, hipEvent_t e0, hipEvent_t e1, float* ms) {
  b->signature.clear();  // forces a new schedule and capture
  int rc = replay(b, what);
  if (!rc) rc = hip_check(hipEventRecord(e0, b->stream), "tune record");
  for (int k = 0; k < 3 && !rc; ++k) rc = replay(b, what);
  if (!rc) rc = hip_check(hipEventRecord(e1, b->stream), "tune record");
  if (!rc) rc = hip_check(hipEventSynchronize(e1), "tune sync");
  if (!rc) rc = hip_check(hipEventElapsedTime(ms, e0, e1), "tune elapsed");
  return rc;
}

// The launch shape of the merged 64-state levels, measured on this device: first the blocks
// each level launch aims for (tiles per block follow from it), then, at the best of those,
// the widest pre-order level that still takes the side-split kernel (each child branch on its
// own wavefronts).  Cached per architecture, state count and batch shape.
int autotune(EpochBatch* b) {
  const std::string key = tune_key(b);
  int v = 0, sv = 0;
  if (!b->tune_path.empty() && tune_lookup(b->tune_path, key + "/target_blocks", v) &&
      tune_lookup(b->tune_path, key + "/split_blocks", sv)) {
    b->target_blocks = v;
    b->split_blocks = sv - 1;  // stored + 1 (0 is a valid choice)
    return EPOCH_OK;
  }
  // tune the evaluation every member supports: the branch gradient only when every member keeps
  // its buffers (a log-likelihood-only member has no outside vectors or dlogL/dP slots)
  bool all_grad = true;
  for (auto* in : b->insts)
    if (!(in->cfg.flags & EPOCH_GRAD_BRANCH)) all_grad = false;
  const uint32_t what = kLogL | (all_grad ? kGradBranch : 0u);
  int rc0 = check_members(b, what);
  if (rc0) return rc0;
  hipEvent_t e0, e1;
  int rc = hip_check(hipEventCreate(&e0), "tune event");
  if (!rc) rc = hip_check(hipEventCreate(&e1), "tune event");
  if (rc) return rc;
  float best = 1e30f;
  int best_t = b->target_blocks, best_s = b->split_blocks;
  for (int t : {512, 1024, 2048, 4096, 8192, 16384}) {
    b->target_blocks = t;
    float ms = 0.f;
    rc = time_shape(b, what, e0, e1, &ms);
    if (rc) break;
    if (ms < best) {
      best = ms;
      best_t = t;
    }
  }
  b->target_blocks = best_t;
  if (!rc && all_grad)  // the split kernel is a pre-order kernel: only the gradient replays see it
    for (int sb : {0, 64, 1024, 4096}) {
      b->split_blocks = sb;
      float ms = 0.f;
      rc = time_shape(b, what, e0, e1, &ms);
      if (rc) break;
      if (ms < best) {
        best = ms;
        best_s = sb;
      }
    }
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
  if (rc) return rc;
  b->split_blocks = best_s;
  b->signature.clear();
  if (!b->tune_path.empty()) {
    tune_store(b->tune_path, key + "/target_blocks", best_t);
    tune_store(b->tune_path, key + "/split_blocks", best_s + 1);
  }
  return EPOCH_OK;
}

}  // namespace

extern "C" {

int epoch_batch_create(EpochInstance* const* insts, int32_t n, const char* tune_cache_path, EpochBatch** out) {
  if (!insts || !out || n < 1) return set_error(EPOCH_ERR_ARG, "batch needs n >= 1 instances and an output");
  *out = nullptr;
  for (int i = 0; i < n; ++i)
    if (!insts[i]) return set_error(EPOCH_ERR_ARG, "batch member %d is NULL", i);
  for (int i = 0; i < n; ++i)
    for (int j = 0; j < i; ++j)
      if (insts[i] == insts[j]) return set_error(EPOCH_ERR_ARG, "batch member %d repeats member %d", i, j);
  auto* b = new EpochBatch();
  b->insts.assign(insts, insts + n);
  // graph capture needs a stream of its own (the legacy default stream cannot be captured)
  if (hipStreamCreateWithFlags(&b->stream, hipStreamNonBlocking) != hipSuccess) {
    delete b;
    return set_error(EPOCH_ERR_HIP, "batch stream creation failed");
  }
  b->own_stream = true;
  b->merged = true;
  for (int i = 0; i < n; ++i) {
    if (insts[i]->path != 2 || insts[i]->codon_nchunks > 1 || insts[i]->fp64 != insts[0]->fp64 ||
        insts[i]->Kp != insts[0]->Kp)
      b->merged = false;
    if (insts[i]->device != insts[0]->device) {
      (void)hipStreamDestroy(b->stream);
      delete b;
      return set_error(EPOCH_ERR_ARG, "batch members must share one device");
    }
  }
  if (tune_cache_path) b->tune_path = tune_cache_path;
  *out = b;
  return EPOCH_OK;
}

int epoch_batch_evaluate(EpochBatch* b, uint32_t what, double* logL) {
  if (!b || !logL) return set_error(EPOCH_ERR_ARG, "batch and logL must not be NULL");
  if (what & ~(kLogL | kGradBranch | kGradQ)) return set_error(EPOCH_ERR_ARG, "unknown evaluation flags");
  what |= kLogL;
  int rc = check_members(b, what);
  if (rc) return rc;
  if (b->merged && !b->tuned) {
    rc = autotune(b);
    if (rc) return rc;
    b->tuned = true;
  }
  rc = replay(b, what);
  if (rc) return rc;
  const size_t n = b->insts.size();
  rc = hip_check(hipMemcpyAsync(logL, b->results.ptr, n * sizeof(double), hipMemcpyDeviceToHost, b->stream), "batch logL");
  if (!rc) rc = hip_check(hipStreamSynchronize(b->stream), "batch sync");
  if (rc) return rc;
  for (size_t q = 0; q < n; ++q) {
    EpochInstance* in = b->insts[q];
    mark_dirty_all(in);  // the graph's launches are not tracked: the member's next single evaluation is full
    in->P_valid = in->partials_valid = true;
    const bool under = logL[q] == -std::numeric_limits<double>::infinity();
    in->logL_valid = std::isfinite(logL[q]) || under;
    in->logL_underflow = under;
    in->grad_ready = (what & (kGradBranch | kGradQ)) != 0 && !under;
    in->gradQ_ready = (what & kGradQ) != 0 && !under;
  }
  int first_under = -1;
  for (size_t q = 0; q < n; ++q) {
    if (std::isnan(logL[q]) || logL[q] == std::numeric_limits<double>::infinity())
      return set_error(EPOCH_ERR_NUMERIC, "batch member %zu: log-likelihood not finite", q);
    if (first_under < 0 && logL[q] == -std::numeric_limits<double>::infinity()) first_under = (int)q;
  }
  if (first_under >= 0)
    return set_error(EPOCH_WARN_UNDERFLOW, "batch member %d: a pattern's likelihood is zero in the working precision "
                     "(logL = -inf; no gradient for that member)", first_under);
  return EPOCH_OK;
}

int epoch_batch_gradients(EpochBatch* b, int32_t i, double* d_branch, double* d_Q) {
  if (!b || i < 0 || i >= (int)b->insts.size()) return set_error(EPOCH_ERR_ARG, "bad batch member index");
  EpochInstance* in = b->insts[i];
  if ((d_branch || d_Q) && in->logL_valid && in->logL_underflow)
    return set_error(EPOCH_ERR_NUMERIC, "batch member %d: the log-likelihood is -inf: no gradient", i);
  if (d_branch && !in->grad_ready) return set_error(EPOCH_ERR_STATE, "the last batch evaluation had no gradient");
  if (d_Q && !in->gradQ_ready) return set_error(EPOCH_ERR_STATE, "the last batch evaluation had no dlogL/dQ");
  int rc = EPOCH_OK;
  if (d_branch)
    rc = hip_check(hipMemcpyAsync(d_branch, in->dbranch.ptr, (size_t)in->n_nodes * sizeof(double), hipMemcpyDeviceToHost,
                                  b->stream), "batch gradient copy");
  if (!rc && d_Q)
    rc = hip_check(hipMemcpyAsync(d_Q, in->dQ.ptr, (size_t)in->S * in->K * in->K * sizeof(double), hipMemcpyDeviceToHost,
                                  b->stream), "batch gradient copy");
  if (!rc) rc = hip_check(hipStreamSynchronize(b->stream), "batch sync");
  return rc;
}

int epoch_batch_target_blocks(EpochBatch* b, int32_t* out) {
  if (!b || !out) return set_error(EPOCH_ERR_ARG, "NULL argument");
  *out = b->target_blocks;
  return EPOCH_OK;
}

int epoch_batch_split_blocks(EpochBatch* b, int32_t* out) {
  if (!b || !out) return set_error(EPOCH_ERR_ARG, "NULL argument");
  *out = b->split_blocks;
  return EPOCH_OK;
}

int epoch_batch_destroy(EpochBatch* b) {
  if (!b) return EPOCH_OK;
  drop_graphs(b);
  release_buf(b->dev);
  release_buf(b->gpart);
  release_buf(b->dpart);
  release_buf(b->pdescs);
  release_buf(b->results);
  for (auto& g : b->gslots) release_buf(g);
  for (int k = 0; k < EpochBatch::kBatchBranches; ++k) {
    if (b->branch[k]) (void)hipStreamDestroy(b->branch[k]);
    if (b->join_ev[k]) (void)hipEventDestroy(b->join_ev[k]);
  }
  if (b->fork_ev) (void)hipEventDestroy(b->fork_ev);
  if (b->own_stream) (void)hipStreamDestroy(b->stream);
  delete b;
  return EPOCH_OK;
}

}  // extern "C"
