// C ABI of the epoch-model likelihood library: instance lifecycle, argument
// validation (always before any HIP call), host->device uploads and the
// dispatch of the kernels.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <limits>
#include <string>
#include <vector>

#include "instance.h"
#include "fastpath.h"
#include "device_common.h"

using namespace epochlik;

namespace epochlik {

thread_local std::string g_error;

int set_error(int code, const char* fmt, ...) {
  char buf[512];
  va_list ap;
  va_start(ap, fmt);
  vsnprintf(buf, sizeof(buf), fmt, ap);
  va_end(ap);
  g_error = buf;
  return code;
}

int hip_check(hipError_t e, const char* what) {
  if (e == hipSuccess) return EPOCH_OK;
  return set_error(EPOCH_ERR_HIP, "%s: %s", what, hipGetErrorString(e));
}

int ensure(DevBuf& b, size_t bytes) {
  if (bytes == 0) bytes = 256;
  if (b.ptr && b.bytes >= bytes) return EPOCH_OK;
  if (b.borrowed) return set_error(EPOCH_ERR_OOM, "a workspace buffer of %zu bytes cannot grow to %zu", b.bytes, bytes);
  if (b.ptr) {
    (void)hipFree(b.ptr);
    b.ptr = nullptr;
    b.bytes = 0;
  }
  hipError_t e = hipMalloc(&b.ptr, bytes);
  if (e != hipSuccess) {
    b.ptr = nullptr;
    (void)hipGetLastError();
    return set_error(EPOCH_ERR_OOM, "hipMalloc of %zu bytes failed: %s", bytes, hipGetErrorString(e));
  }
  b.bytes = bytes;
  return EPOCH_OK;
}

namespace {
int collect_phase(EpochInstance* in, int k) {
  if (!in->ev_pending[k]) return EPOCH_OK;
  int rc = hip_check(hipEventSynchronize(in->ev[k][1]), "timing event sync");
  if (rc) return rc;
  float ms = 0.f;
  rc = hip_check(hipEventElapsedTime(&ms, in->ev[k][0], in->ev[k][1]), "timing elapsed");
  if (rc) return rc;
  in->phase_ms[k] += ms;
  in->ev_pending[k] = false;
  return EPOCH_OK;
}
}  // namespace

int phase_begin(EpochInstance* in, int k) {
  if (!in->timing) return EPOCH_OK;
  int rc = collect_phase(in, k);
  if (rc) return rc;
  return hip_check(hipEventRecord(in->ev[k][0], in->stream), "timing record");
}

int phase_end(EpochInstance* in, int k) {
  if (!in->timing) return EPOCH_OK;
  int rc = hip_check(hipEventRecord(in->ev[k][1], in->stream), "timing record");
  in->ev_pending[k] = true;
  in->phase_count[k]++;
  return rc;
}

}  // namespace epochlik

namespace {

// Above this condition number of V the FP32 path reconstructs exp(tQ) in FP64.
// FP32 reconstruction errs by about cond(V) 2^-24 of the largest entry, which
// is large next to the small entries of P and dP/dt that weigh most in the
// gradients.  Measured against the FP64 oracle with FP32 products throughout:
// the 61-state codon systems (cond 50-65) keep logL within 4e-7 but put one
// branch-gradient component of a 64-problem batch 1.9e-3 off (the FP32
// tolerance is 1e-3), and the 40-state asymmetric trait systems (cond 250-2,800,
// 48 intervals) miss logL by 3e-3 on 200 taxa and give NaN on 2,000.
constexpr double kCondFP32 = 32.0;

void release(DevBuf& b) {
  if (b.ptr && !b.borrowed) (void)hipFree(b.ptr);
  b.borrowed = false;
  b.ptr = nullptr;
  b.bytes = 0;
}

// The pattern-sized buffers a caller-owned workspace holds, in order, with their sizes.
struct WorkspaceItem {
  DevBuf EpochInstance::*buf;
  size_t bytes;
};
size_t scale_sets(const EpochConfig& c);
std::vector<WorkspaceItem> workspace_items(const EpochConfig& c, int Kp) {
  const size_t N = c.n_tips, P = c.n_patterns, C = c.n_categories, R = c.precision == EPOCH_FP64 ? 8 : 4;
  const bool grad = (c.flags & (EPOCH_GRAD_BRANCH | EPOCH_GRAD_Q | EPOCH_GRAD_TIME)) != 0;
  std::vector<WorkspaceItem> v = {{&EpochInstance::tips, N * P},
                                  {&EpochInstance::weights, P * sizeof(double)},
                                  {&EpochInstance::weightsT, P * R * scale_sets(c)},
                                  {&EpochInstance::partials, (N - 1) * C * P * Kp * R},
                                  {&EpochInstance::scales, (N - 1) * P * sizeof(int32_t) * scale_sets(c)},
                                  {&EpochInstance::site, P * sizeof(double)}};
  if (grad) v.push_back({&EpochInstance::pre, (N - 1) * C * P * Kp * R});
  return v;
}
size_t aligned256(size_t b) { return (b + 255) / 256 * 256; }
size_t workspace_total(const EpochConfig& c, int Kp) {
  size_t t = 0;
  for (const auto& it : workspace_items(c, Kp)) t += aligned256(it.bytes);
  return t;
}

int padded_states(int K) {
  if (K <= 4) return 4;
  if (K <= 8) return 8;
  return (K + 15) / 16 * 16;
}

// Problems of 49..64 states (padded to 64), and of 17..32 states (a 20-state amino-acid
// model, say, padded to 32: the padding states are never observed and their transition
// rows are the identity), run on the matrix-core 64- / 32-state kernels, FP32 or FP64,
// with any number of rate categories; under an HBM budget (pattern chunks) FP32 with
// one category.
bool codon_config(const EpochConfig& c) {
  return ((c.n_states > 48 && c.n_states <= 64) || (c.n_states > 16 && c.n_states <= 32)) &&
         c.kernel_path == EPOCH_KERNEL_AUTO &&
         (c.hbm_budget_bytes == 0 || (c.n_categories == 1 && c.precision == EPOCH_FP32));
}
int padded_states(const EpochConfig& c) { return padded_states(c.n_states); }
// The 64-state kernels keep one scale exponent and one weight row per rate category.
size_t scale_sets(const EpochConfig& c) { return codon_config(c) ? (size_t)c.n_categories : 1; }

#define EPOCH_TRY(expr)          \
  do {                           \
    int _rc = (expr);            \
    if (_rc != EPOCH_OK) return _rc; \
  } while (0)

int upload(EpochInstance* in, void* dst, const void* src, size_t bytes) {
  if (bytes == 0) return EPOCH_OK;
  EPOCH_TRY(hip_check(hipMemcpyAsync(dst, src, bytes, hipMemcpyHostToDevice, in->stream), "upload"));
  return hip_check(hipStreamSynchronize(in->stream), "upload sync");
}

int download(EpochInstance* in, void* dst, const void* src, size_t bytes) {
  if (bytes == 0) return EPOCH_OK;
  EPOCH_TRY(hip_check(hipMemcpyAsync(dst, src, bytes, hipMemcpyDeviceToHost, in->stream), "download"));
  return hip_check(hipStreamSynchronize(in->stream), "download sync");
}

bool all_finite(const double* x, size_t n) {
  for (size_t i = 0; i < n; ++i)
    if (!std::isfinite(x[i])) return false;
  return true;
}

int choose_chunks(EpochInstance* in) {
  int q = 4;
  while (q < in->Kp) q <<= 1;
  const int TP = 256 / q;
  const long tiles = (in->P + TP - 1) / TP;
  const size_t per_chunk = (size_t)in->n_nodes * in->C * in->Kp * in->Kp * sizeof(double);
  long cap = (long)std::max<size_t>(1, (size_t)(256u << 20) / std::max<size_t>(per_chunk, 1));
  long n = std::min<long>({tiles, 64L, cap});
  return (int)std::max<long>(1, n);
}

// The 64-state path takes an HBM budget by evaluating the patterns in chunks.
bool codon_budget_config(const EpochConfig& c) {
  return ((c.n_states > 48 && c.n_states <= 64) || (c.n_states > 16 && c.n_states <= 32)) &&
         c.precision == EPOCH_FP32 && c.n_categories == 1 && c.kernel_path == EPOCH_KERNEL_AUTO;
}
// Device bytes one pattern of a chunk costs on the 64-state path: partials and
// scale exponents of every internal node, outside vectors with a gradient, and
// the dlogL/dP slots (at most one 64 x 64 FP32 slot per child branch and tile
// of 64 patterns).
size_t codon_bytes_per_pattern(const EpochConfig& c) {
  const bool grad = (c.flags & (EPOCH_GRAD_BRANCH | EPOCH_GRAD_Q | EPOCH_GRAD_TIME)) != 0;
  const size_t Nm1 = (size_t)c.n_tips - 1, Kp = padded_states(c.n_states);
  return Nm1 * (Kp * sizeof(float) + sizeof(int32_t)) +
         (grad ? Nm1 * Kp * sizeof(float) + 2 * Nm1 * Kp * Kp * sizeof(float) / 64 : 0);
}

// Device bytes one pattern of a chunk costs on the generic path: partials and
// scale exponents of every internal node, and outside vectors with a gradient.
size_t generic_bytes_per_pattern(const EpochConfig& c) {
  const bool grad = (c.flags & (EPOCH_GRAD_BRANCH | EPOCH_GRAD_Q | EPOCH_GRAD_TIME)) != 0;
  const size_t Nm1 = (size_t)c.n_tips - 1, R = c.precision == EPOCH_FP64 ? 8 : 4;
  const size_t row = (size_t)c.n_categories * padded_states(c) * R;
  return Nm1 * (row * (grad ? 2 : 1) + sizeof(int32_t));
}

void invalidate_downstream(EpochInstance* in) {
  in->P_valid = false;
  in->partials_valid = false;
  in->logL_valid = false;
}

// Host-to-device copies of one set_epoch_eigensystems call, staged in the
// instance's pinned host buffer and enqueued on its stream without waiting; the
// next call waits for them (stage_event) before it reuses the buffer.
struct EigStage {
  EpochInstance* in;
  size_t off = 0;
  int rc = EPOCH_OK;
  template <typename D>
  void put(void* dst, const double* src, size_t n) {  // n doubles, copied as D
    if (rc) return;
    off = (off + 15) / 16 * 16;
    D* h = reinterpret_cast<D*>(static_cast<char*>(in->stage_host) + off);
    for (size_t i = 0; i < n; ++i) h[i] = (D)src[i];
    rc = hip_check(hipMemcpyAsync(dst, h, n * sizeof(D), hipMemcpyHostToDevice, in->stream), "eigensystem upload");
    off += n * sizeof(D);
  }
};
int stage_reserve(EpochInstance* in, size_t bytes) {
  if (in->stage_pending) {
    EPOCH_TRY(hip_check(hipEventSynchronize(in->stage_event), "eigensystem staging wait"));
    in->stage_pending = false;
  }
  if (!in->stage_event) EPOCH_TRY(hip_check(hipEventCreateWithFlags(&in->stage_event, hipEventDisableTiming), "staging event"));
  if (in->stage_bytes >= bytes) return EPOCH_OK;
  if (in->stage_host) (void)hipHostFree(in->stage_host);
  in->stage_host = nullptr;
  in->stage_bytes = 0;
  if (hipHostMalloc(&in->stage_host, bytes, hipHostMallocDefault) != hipSuccess) {
    in->stage_host = nullptr;
    return set_error(EPOCH_ERR_OOM, "pinned staging buffer of %zu bytes", bytes);
  }
  in->stage_bytes = bytes;
  return EPOCH_OK;
}

}  // namespace

extern "C" {

const char* epoch_last_error(void) { return g_error.c_str(); }

const char* epoch_version(void) { return "epochlik 0.1.0 (gfx950)"; }

int epoch_create(const EpochConfig* cfg, EpochInstance** out) {
  g_error.clear();
  if (!cfg || !out) return set_error(EPOCH_ERR_ARG, "cfg and out must not be NULL");
  *out = nullptr;
  const EpochConfig& c = *cfg;
  if (c.n_tips < 2) return set_error(EPOCH_ERR_ARG, "n_tips must be >= 2 (got %d)", c.n_tips);
  if (c.n_tips > (1 << 24)) return set_error(EPOCH_ERR_ARG, "n_tips too large (%d)", c.n_tips);
  if (c.n_patterns < 1) return set_error(EPOCH_ERR_ARG, "n_patterns must be >= 1 (got %d)", c.n_patterns);
  if (c.n_states < 2 || c.n_states > 64)
    return set_error(EPOCH_ERR_ARG, "n_states must be in [2, 64] (got %d)", c.n_states);
  if (c.n_categories < 1 || c.n_categories > kMaxCategories)
    return set_error(EPOCH_ERR_ARG, "n_categories must be in [1, 8] (got %d)", c.n_categories);
  if (c.n_processes < 1) return set_error(EPOCH_ERR_ARG, "n_processes must be >= 1");
  if (c.max_intervals < 1) return set_error(EPOCH_ERR_ARG, "max_intervals must be >= 1");
  if (c.precision != EPOCH_FP32 && c.precision != EPOCH_FP64)
    return set_error(EPOCH_ERR_ARG, "precision must be EPOCH_FP32 or EPOCH_FP64");
  if (c.flags & ~(EPOCH_GRAD_BRANCH | EPOCH_GRAD_Q | EPOCH_GRAD_TIME)) return set_error(EPOCH_ERR_ARG, "unknown flags");
  if (c.kernel_path != EPOCH_KERNEL_AUTO && c.kernel_path != EPOCH_KERNEL_GENERIC)
    return set_error(EPOCH_ERR_ARG, "unknown kernel_path");
  if (c.reserved != 0) return set_error(EPOCH_ERR_ARG, "reserved must be 0");
  if (c.hbm_budget_bytes < 0) return set_error(EPOCH_ERR_ARG, "hbm_budget_bytes must be >= 0");
  // HBM budgets: the 4-state tree walk recomputes subtrees; the 64-state and generic
  // paths evaluate the patterns in chunks
  const bool nuc_budget = c.hbm_budget_bytes > 0 && c.n_states == 4 && c.kernel_path == EPOCH_KERNEL_AUTO;
  const bool codon_budget = c.hbm_budget_bytes > 0 && codon_budget_config(c);
  const bool gen_budget = c.hbm_budget_bytes > 0 && !nuc_budget && !codon_budget;
  if (nuc_budget && (c.flags & EPOCH_GRAD_TIME))
    return set_error(EPOCH_ERR_ARG, "hbm_budget_bytes with the 4-state kernels cannot be combined with EPOCH_GRAD_TIME "
                                    "(the time gradient needs the branch adjoints of the level kernels)");
  if (nuc_budget && (c.flags & EPOCH_GRAD_Q))
    return set_error(EPOCH_ERR_ARG,
                     "hbm_budget_bytes with the 4-state kernels cannot be combined with EPOCH_GRAD_Q "
                     "(EPOCH_KERNEL_GENERIC evaluates pattern chunks instead)");
  const size_t chunk_pattern_bytes = codon_budget ? codon_bytes_per_pattern(c) : generic_bytes_per_pattern(c);
  if ((codon_budget || gen_budget) &&
      (size_t)c.hbm_budget_bytes < chunk_pattern_bytes * (size_t)std::min(c.n_patterns, 64))
    return set_error(EPOCH_ERR_ARG, "hbm_budget_bytes %lld is below the %zu bytes one chunk of 64 patterns needs",
                     (long long)c.hbm_budget_bytes, chunk_pattern_bytes * (size_t)std::min(c.n_patterns, 64));
  if (c.workspace && c.hbm_budget_bytes > 0)
    return set_error(EPOCH_ERR_ARG, "a workspace cannot be combined with hbm_budget_bytes");
  if (c.workspace && (c.workspace_bytes < 0 || (size_t)c.workspace_bytes < workspace_total(c, padded_states(c))))
    return set_error(EPOCH_ERR_ARG, "workspace_bytes %lld is below the %zu bytes epoch_workspace_bytes asks for",
                     (long long)c.workspace_bytes, workspace_total(c, padded_states(c)));
  if (c.workspace && (reinterpret_cast<uintptr_t>(c.workspace) & 255))
    return set_error(EPOCH_ERR_ARG, "workspace must be 256-byte aligned");
  const size_t N = c.n_tips, P = c.n_patterns;
  if ((N - 1) * P > ((size_t)1 << 40)) return set_error(EPOCH_ERR_ARG, "problem too large");

  int ndev = 0;
  const hipError_t derr = hipGetDeviceCount(&ndev);
  if (derr != hipSuccess || ndev < 1) {
    (void)hipGetLastError();
    return set_error(EPOCH_ERR_HIP, "no HIP device available (hipGetDeviceCount: %s, count %d)",
                     hipGetErrorString(derr), ndev);
  }
  auto* in = new EpochInstance();
  in->cfg = c;
  if (c.flags & EPOCH_GRAD_TIME) in->cfg.flags |= EPOCH_GRAD_BRANCH;  // the time gradient reads the branch adjoints
  in->N = c.n_tips;
  in->P = c.n_patterns;
  in->K = c.n_states;
  in->Kp = padded_states(c);
  in->C = c.n_categories;
  in->S = c.n_processes;
  in->n_nodes = 2 * c.n_tips - 1;
  in->n_int = c.n_tips - 1;
  in->fp64 = c.precision == EPOCH_FP64;
  in->real_size = in->fp64 ? 8 : 4;
  in->stream = static_cast<hipStream_t>(c.stream);
  (void)hipGetDevice(&in->device);
  const size_t Kp = in->Kp, KK = Kp * Kp, S = in->S, C = in->C, n = in->n_nodes, R = in->real_size;
  const bool grad = (c.flags & (EPOCH_GRAD_BRANCH | EPOCH_GRAD_Q | EPOCH_GRAD_TIME)) != 0;
  in->h_V.assign(S * KK, 0.0);
  in->h_Vinv.assign(S * KK, 0.0);
  in->h_lre.assign(S * Kp, 0.0);
  in->h_lim.assign(S * Kp, 0.0);
  in->have_eig.assign(S, 0);
  in->cond.assign(S, 1.0);
  in->n_chunks = choose_chunks(in);
  int rc = EPOCH_OK;
  if (c.workspace) {  // pattern-sized buffers inside the caller's memory
    size_t off = 0;
    for (const auto& it : workspace_items(c, (int)Kp)) {
      DevBuf& b = in->*(it.buf);
      b.ptr = static_cast<char*>(c.workspace) + off;
      b.bytes = std::max<size_t>(it.bytes, 256);
      b.borrowed = true;
      off += aligned256(it.bytes);
    }
  }
  auto A = [&](DevBuf& b, size_t bytes) {
    if (rc == EPOCH_OK) rc = ensure(b, bytes);
  };
  A(in->eigT, (2 * S * KK + 2 * S * Kp) * R);
  A(in->eig64, (2 * S * KK + 2 * S * Kp) * sizeof(double));
  A(in->eigTT, 2 * S * KK * R);
  A(in->eig64T, 2 * S * KK * sizeof(double));
  A(in->check, (KK + 1 + 3 * (size_t)eigen_check_tiles(in->K)) * sizeof(double));  // Q, residual, tile maxima
  A(in->tips, N * P);
  A(in->amb, 256 * sizeof(uint64_t));
  A(in->weights, P * sizeof(double));
  A(in->weightsT, P * R * scale_sets(c));
  A(in->pi, Kp * sizeof(double));
  A(in->cat, 2 * kMaxCategories * sizeof(double));
  A(in->Pm, n * C * KK * R);
  if (grad) A(in->dPm, n * C * KK * R);
  in->budget = c.hbm_budget_bytes;
  if (codon_budget || gen_budget) {
    // 64-state and generic paths: the patterns run in chunks whose partials, outside
    // vectors, scale exponents (and 64-state dlogL/dP slots) fit the budget
    const size_t pc = std::min<size_t>(P, (size_t)in->budget / chunk_pattern_bytes / 64 * 64);
    const int nc = (int)((P + pc - 1) / pc);
    if (codon_budget) {
      in->codon_pc = (int)pc;
      in->codon_nchunks = nc;
    } else {
      in->gen_pc = (int)pc;
      in->gen_nchunks = nc;
    }
    A(in->partials, (N - 1) * C * pc * Kp * R);
    A(in->scales, (N - 1) * pc * sizeof(int32_t));
    if (grad) A(in->pre, (N - 1) * C * pc * Kp * R);
  } else if (in->budget > 0) {
    in->walk_enable = 1;  // partials are sized at set_tree_epochs, within the budget
  } else {
    A(in->partials, (N - 1) * C * P * Kp * R);
    A(in->scales, (N - 1) * P * sizeof(int32_t) * scale_sets(c));
    if (grad) A(in->pre, (N - 1) * C * P * Kp * R);
  }
  A(in->site, P * sizeof(double));
  A(in->blocksum, ((P + 63) / 64 + 1) * sizeof(double));
  A(in->result, std::max<size_t>(8, std::max(in->codon_nchunks, in->gen_nchunks) + 1) * sizeof(double));
  if (grad) {
    A(in->Gpart, (size_t)in->n_chunks * n * C * KK * sizeof(double));
    A(in->G, n * C * KK * sizeof(double));
    A(in->dbranch, n * sizeof(double));
  }
  if (c.flags & EPOCH_GRAD_Q) A(in->dQ, S * KK * sizeof(double));
  if (rc == EPOCH_OK) rc = fastpath_init(in);
  if (rc != EPOCH_OK) {
    std::string keep = g_error;
    epoch_destroy(in);
    g_error = keep;
    return rc;
  }
  // zero the eigen buffers so padding is well defined
  rc = hip_check(hipMemsetAsync(in->eigT.ptr, 0, in->eigT.bytes, in->stream), "memset");
  if (rc == EPOCH_OK) rc = hip_check(hipMemsetAsync(in->eig64.ptr, 0, in->eig64.bytes, in->stream), "memset");
  if (rc == EPOCH_OK) rc = hip_check(hipMemsetAsync(in->eigTT.ptr, 0, in->eigTT.bytes, in->stream), "memset");
  if (rc == EPOCH_OK) rc = hip_check(hipMemsetAsync(in->eig64T.ptr, 0, in->eig64T.bytes, in->stream), "memset");
  if (rc == EPOCH_OK) rc = hip_check(hipMemsetAsync(in->amb.ptr, 0, in->amb.bytes, in->stream), "memset");
  if (rc == EPOCH_OK) rc = hip_check(hipStreamSynchronize(in->stream), "create sync");
  if (rc != EPOCH_OK) {
    std::string keep = g_error;
    epoch_destroy(in);
    g_error = keep;
    return rc;
  }
  *out = in;
  return EPOCH_OK;
}

int epoch_set_timing(EpochInstance* in, int32_t enable) {
  if (!in) return set_error(EPOCH_ERR_ARG, "NULL instance");
  if (enable && !in->ev[0][0]) {
    for (int k = 0; k < EPOCH_N_PHASES; ++k)
      for (int j = 0; j < 2; ++j) EPOCH_TRY(hip_check(hipEventCreate(&in->ev[k][j]), "hipEventCreate"));
  }
  EPOCH_TRY(hip_check(hipStreamSynchronize(in->stream), "timing sync"));
  for (int k = 0; k < EPOCH_N_PHASES; ++k) {
    in->ev_pending[k] = false;
    in->phase_ms[k] = 0.0;
    in->phase_count[k] = 0;
  }
  in->timing = enable != 0;
  return EPOCH_OK;
}

int epoch_get_timing(EpochInstance* in, double* ms_out, int64_t* counts_out) {
  if (!in) return set_error(EPOCH_ERR_ARG, "NULL instance");
  if (in->timing)
    for (int k = 0; k < EPOCH_N_PHASES; ++k) {
      int rc = EPOCH_OK;
      if (in->ev_pending[k]) {
        rc = hip_check(hipEventSynchronize(in->ev[k][1]), "timing event sync");
        float ms = 0.f;
        if (!rc) rc = hip_check(hipEventElapsedTime(&ms, in->ev[k][0], in->ev[k][1]), "timing elapsed");
        if (rc) return rc;
        in->phase_ms[k] += ms;
        in->ev_pending[k] = false;
      }
    }
  for (int k = 0; k < EPOCH_N_PHASES; ++k) {
    if (ms_out) ms_out[k] = in->phase_ms[k];
    if (counts_out) counts_out[k] = in->phase_count[k];
  }
  return EPOCH_OK;
}

int epoch_destroy(EpochInstance* in) {
  if (!in) return EPOCH_OK;
  if (in->stage_pending) (void)hipEventSynchronize(in->stage_event);  // staged copies still in flight
  if (in->stage_event) (void)hipEventDestroy(in->stage_event);
  if (in->stage_host) (void)hipHostFree(in->stage_host);
  for (int k = 0; k < EPOCH_N_PHASES; ++k)
    for (int j = 0; j < 2; ++j)
      if (in->ev[k][j]) (void)hipEventDestroy(in->ev[k][j]);
  fastpath_release(in);
  for (DevBuf* b : {&in->eigT, &in->eig64, &in->check, &in->tips, &in->weights, &in->weightsT, &in->pi,
                    &in->cat, &in->tree_i, &in->tree_d, &in->Pm, &in->dPm, &in->partials, &in->scales,
                    &in->pre, &in->site, &in->blocksum, &in->result, &in->Gpart, &in->G, &in->dbranch,
                    &in->qseg, &in->qscratch, &in->chain_items, &in->chain_scratch, &in->dQ, &in->seglist, &in->gslots, &in->codon_dev, &in->codon_aux,
                    &in->eigTT, &in->eig64T, &in->qtau, &in->nuc_nodes, &in->walk_ops,
                    &in->walk_tcol, &in->walk_dpart, &in->walk_dummy, &in->walk_slots, &in->inc_dev, &in->tg_i,
                    &in->tg_d, &in->amb})
    release(*b);
  delete in;
  return EPOCH_OK;
}

int epoch_set_tip_ambiguities(EpochInstance* in, int32_t n_codes, const uint64_t* sets) {
  if (!in) return set_error(EPOCH_ERR_ARG, "NULL instance");
  if (n_codes < 0 || n_codes > 255 - in->K)
    return set_error(EPOCH_ERR_ARG, "n_codes must be in [0, %d] (codes K + 1 .. K + n_codes fit a byte)", 255 - in->K);
  if (n_codes > 0 && !sets) return set_error(EPOCH_ERR_ARG, "sets must not be NULL");
  const uint64_t all = in->K == 64 ? ~0ull : ((1ull << in->K) - 1);
  for (int a = 0; a < n_codes; ++a)
    if (sets[a] == 0 || (sets[a] & ~all))
      return set_error(EPOCH_ERR_ARG, "ambiguity set %d is empty or names a state >= %d", a, in->K);
  std::vector<uint64_t> h(256, 0);
  std::copy(sets, sets + n_codes, h.begin());
  EPOCH_TRY(upload(in, in->amb.ptr, h.data(), h.size() * sizeof(uint64_t)));
  in->h_amb.assign(sets, sets + n_codes);
  in->have_tips = false;  // the tip states are read with the new table: set them again
  mark_dirty_all(in);
  in->partials_valid = in->logL_valid = false;
  return EPOCH_OK;
}

int epoch_set_tip_states(EpochInstance* in, const int32_t* states) {
  if (!in || !states) return set_error(EPOCH_ERR_ARG, "instance and states must not be NULL");
  const size_t n = (size_t)in->N * in->P;
  const int max_code = in->K + (int)in->h_amb.size();
  std::vector<uint8_t> h(n);
  for (size_t k = 0; k < n; ++k) {
    const int32_t s = states[k];
    if (s < 0 || s > max_code)
      return set_error(EPOCH_ERR_ARG, "tip state %d at (%zu, %zu) outside [0, %d]", s, k / in->P,
                       k % in->P, max_code);
    h[k] = (uint8_t)s;
  }
  in->tips_amb = false;
  for (size_t k = 0; k < n && !in->tips_amb; ++k) in->tips_amb = h[k] > in->K;
  if (in->path == 1) {
    // the 4-state kernels read a tip as its state set (bit i = state i): one state, all four
    // when missing, or the caller's ambiguity set
    uint8_t code_set[256];
    for (int s = 0; s <= max_code; ++s)
      code_set[s] = (uint8_t)(s < 4 ? 1u << s : (s == 4 ? 15u : (unsigned)in->h_amb[s - 5]));
    for (size_t k = 0; k < n; ++k) h[k] = code_set[h[k]];
  }
  EPOCH_TRY(upload(in, in->tips.ptr, h.data(), n));
  mark_dirty_all(in);
  in->have_tips = true;
  in->partials_valid = false;
  in->logL_valid = false;
  return fastpath_tips_changed(in);
}

int epoch_set_pattern_weights(EpochInstance* in, const double* w) {
  if (!in || !w) return set_error(EPOCH_ERR_ARG, "instance and weights must not be NULL");
  for (int p = 0; p < in->P; ++p)
    if (!std::isfinite(w[p]) || w[p] < 0) return set_error(EPOCH_ERR_ARG, "weight %d is negative or not finite", p);
  EPOCH_TRY(upload(in, in->weights.ptr, w, (size_t)in->P * sizeof(double)));
  if (in->fp64) {
    EPOCH_TRY(upload(in, in->weightsT.ptr, w, (size_t)in->P * sizeof(double)));
  } else {
    std::vector<float> f(w, w + in->P);
    EPOCH_TRY(upload(in, in->weightsT.ptr, f.data(), f.size() * sizeof(float)));
  }
  in->have_weights = true;
  in->logL_valid = false;
  return EPOCH_OK;
}

int epoch_set_categories(EpochInstance* in, const double* rates, const double* weights) {
  if (!in || !rates || !weights) return set_error(EPOCH_ERR_ARG, "NULL argument");
  double sum = 0;
  for (int c = 0; c < in->C; ++c) {
    if (!std::isfinite(rates[c]) || !(rates[c] > 0)) return set_error(EPOCH_ERR_ARG, "category rate %d must be > 0", c);
    if (!std::isfinite(weights[c]) || weights[c] < 0) return set_error(EPOCH_ERR_ARG, "category weight %d must be >= 0", c);
    sum += weights[c];
  }
  if (std::fabs(sum - 1.0) > 1e-9) return set_error(EPOCH_ERR_ARG, "category weights sum to %.17g, not 1", sum);
  double h[2 * kMaxCategories] = {0};
  for (int c = 0; c < in->C; ++c) {
    h[c] = rates[c];
    h[kMaxCategories + c] = weights[c];
    in->h_cat_rates[c] = rates[c];
    in->h_cat_weights[c] = weights[c];
  }
  EPOCH_TRY(upload(in, in->cat.ptr, h, sizeof(h)));
  mark_dirty_all(in);
  in->have_cats = true;
  invalidate_downstream(in);
  return EPOCH_OK;
}

int epoch_set_root_frequencies(EpochInstance* in, const double* pi) {
  if (!in || !pi) return set_error(EPOCH_ERR_ARG, "NULL argument");
  double sum = 0;
  std::vector<double> h(in->Kp, 0.0);
  for (int i = 0; i < in->K; ++i) {
    if (!std::isfinite(pi[i]) || pi[i] < 0) return set_error(EPOCH_ERR_ARG, "pi[%d] must be >= 0", i);
    sum += pi[i];
    h[i] = pi[i];
  }
  if (std::fabs(sum - 1.0) > 1e-9) return set_error(EPOCH_ERR_ARG, "pi sums to %.17g, not 1", sum);
  EPOCH_TRY(upload(in, in->pi.ptr, h.data(), h.size() * sizeof(double)));
  in->have_pi = true;
  in->logL_valid = false;
  return EPOCH_OK;
}

// Arithmetic of exp(tQ) = V exp(t Lambda) V^-1 and of the dlogL/dQ chains in an
// FP32 instance: FP64 when some eigenvector matrix has infinity-norm condition
// number above kCondFP32 (EPOCH_OPT_EIGEN_PRECISION 0), always FP32 (1), or
// always FP64 (2).  Returns whether it changed.
static bool choose_eig_precision(EpochInstance* in) {
  const bool was = in->eig_fp64;
  in->eig_fp64 = in->eig_mode == 2;
  if (in->eig_mode == 0)
    for (int k = 0; k < in->S; ++k)
      if (in->cond[k] > kCondFP32) in->eig_fp64 = true;
  return was != in->eig_fp64;
}

int set_epoch_eigensystems(EpochInstance* in, int32_t s, const double* V, const double* Vinv,
                           const double* lambda_re, const double* lambda_im, const double* Q,
                           double* residual_out) {
  if (!in || !V || !Vinv || !lambda_re) return set_error(EPOCH_ERR_ARG, "NULL argument");
  if (s < 0 || s >= in->S) return set_error(EPOCH_ERR_ARG, "process index %d outside [0, %d)", s, in->S);
  const int K = in->K, Kp = in->Kp;
  if (!all_finite(V, (size_t)K * K) || !all_finite(Vinv, (size_t)K * K) || !all_finite(lambda_re, K))
    return set_error(EPOCH_ERR_ARG, "eigensystem %d has non-finite entries", s);
  if (lambda_im) {
    if (!all_finite(lambda_im, K)) return set_error(EPOCH_ERR_ARG, "lambda_im has non-finite entries");
    for (int j = 0; j < K; ++j) {
      if (lambda_im[j] > 0) {
        if (j + 1 >= K || lambda_im[j + 1] != -lambda_im[j] || lambda_re[j + 1] != lambda_re[j])
          return set_error(EPOCH_ERR_ARG, "complex pair at column %d is not followed by its conjugate", j);
        ++j;
      } else if (lambda_im[j] < 0) {
        return set_error(EPOCH_ERR_ARG, "negative imaginary part at column %d without its pair", j);
      }
    }
  }
  if (Q && !all_finite(Q, (size_t)K * K)) return set_error(EPOCH_ERR_ARG, "Q has non-finite entries");
  const size_t KK = (size_t)Kp * Kp, S = in->S;
  double* hV = in->h_V.data() + s * KK;
  double* hVi = in->h_Vinv.data() + s * KK;
  double* hr = in->h_lre.data() + (size_t)s * Kp;
  double* hi = in->h_lim.data() + (size_t)s * Kp;
  std::fill(hV, hV + KK, 0.0);
  std::fill(hVi, hVi + KK, 0.0);
  std::fill(hr, hr + Kp, 0.0);
  std::fill(hi, hi + Kp, 0.0);
  // Device column order: complex pairs first, so that every pair occupies an
  // (even, odd) column couple, then the real eigenvalues.  Permuting the
  // columns of V, the rows of V^-1 and the eigenvalues together leaves
  // V diag(.) V^-1 unchanged.
  std::vector<int> order;
  order.reserve(K);
  for (int j = 0; j < K; ++j)
    if (lambda_im && lambda_im[j] > 0) {
      order.push_back(j);
      order.push_back(j + 1);
    }
  for (int j = 0; j < K; ++j)
    if (!lambda_im || lambda_im[j] == 0) order.push_back(j);
  for (int i = 0; i < K; ++i) {
    for (int q = 0; q < K; ++q) {
      hV[i * Kp + q] = V[i * K + order[q]];
      hVi[q * Kp + i] = Vinv[order[q] * K + i];
    }
  }
  for (int q = 0; q < K; ++q) {
    hr[q] = lambda_re[order[q]];
    hi[q] = lambda_im ? lambda_im[order[q]] : 0.0;
  }
  in->any_complex = false;
  for (double x : in->h_lim)
    if (x != 0.0) in->any_complex = true;
  {
    double nv = 0.0, ni = 0.0;
    for (int i = 0; i < K; ++i) {
      double rv = 0.0, ri = 0.0;
      for (int j = 0; j < K; ++j) {
        rv += std::fabs(V[i * K + j]);
        ri += std::fabs(Vinv[i * K + j]);
      }
      nv = std::max(nv, rv);
      ni = std::max(ni, ri);
    }
    in->cond[s] = nv * ni;
    // a new eigensystem changes the factors of process s only (Eq. 6-7), unless the
    // arithmetic of every reconstruction changes with it
    if (choose_eig_precision(in) || !in->have_eig[s]) mark_dirty_all(in);
    else mark_dirty_process(in, s);
  }
  // this process's slices in double and in the compute type, and the transposed
  // copies (rows of V^T and V^-T feed the adjoint chain), staged in pinned host
  // memory and copied without waiting
  const size_t R = in->real_size;
  const size_t need = (2 * KK + 2 * Kp) * (8 + R) + 2 * KK * (8 + R) + (size_t)K * K * 8 + 16 * 16;
  EPOCH_TRY(stage_reserve(in, need));
  EigStage st{in};
  auto slice = [&](DevBuf& buf, bool as_float) {
    const size_t es = as_float ? sizeof(float) : sizeof(double);
    char* base = static_cast<char*>(buf.ptr);
    const double* src[4] = {hV, hVi, hr, hi};
    const size_t off[4] = {s * KK, S * KK + s * KK, 2 * S * KK + (size_t)s * Kp, 2 * S * KK + S * Kp + (size_t)s * Kp};
    const size_t cnt[4] = {KK, KK, (size_t)Kp, (size_t)Kp};
    for (int k = 0; k < 4; ++k) {
      if (as_float)
        st.put<float>(base + off[k] * es, src[k], cnt[k]);
      else
        st.put<double>(base + off[k] * es, src[k], cnt[k]);
    }
  };
  slice(in->eig64, false);
  slice(in->eigT, !in->fp64);
  {
    std::vector<double> tV(KK), tVi(KK);
    for (int i = 0; i < Kp; ++i)
      for (int j = 0; j < Kp; ++j) {
        tV[(size_t)j * Kp + i] = hV[(size_t)i * Kp + j];
        tVi[(size_t)j * Kp + i] = hVi[(size_t)i * Kp + j];
      }
    char* b64 = static_cast<char*>(in->eig64T.ptr);
    st.put<double>(b64 + s * KK * sizeof(double), tV.data(), KK);
    st.put<double>(b64 + (S * KK + s * KK) * sizeof(double), tVi.data(), KK);
    char* bT = static_cast<char*>(in->eigTT.ptr);
    if (in->fp64) {
      st.put<double>(bT + s * KK * 8, tV.data(), KK);
      st.put<double>(bT + (S * KK + s * KK) * 8, tVi.data(), KK);
    } else {
      st.put<float>(bT + s * KK * 4, tV.data(), KK);
      st.put<float>(bT + (S * KK + s * KK) * 4, tVi.data(), KK);
    }
  }
  double* dQ = static_cast<double*>(in->check.ptr);
  if (Q) st.put<double>(dQ, Q, (size_t)K * K);
  if (st.rc) {  // copies enqueued before the failure may still read the staging buffer
    (void)hipStreamSynchronize(in->stream);
    return st.rc;
  }
  EPOCH_TRY(hip_check(hipEventRecord(in->stage_event, in->stream), "eigensystem upload event"));
  in->stage_pending = true;
  in->have_eig[s] = 1;
  invalidate_downstream(in);
  int ret = EPOCH_OK;
  if (Q) {
    double* dout = dQ + (size_t)Kp * Kp;
    EPOCH_TRY(launch_eigen_check(in, s, dQ, dout));
    double res = 0.0;
    EPOCH_TRY(download(in, &res, dout, sizeof(res)));
    if (residual_out) *residual_out = res;
    if (!(res <= 1e-8)) {
      set_error(EPOCH_WARN_EIGEN_RESIDUAL, "eigensystem %d reconstruction residual %.3g", s, res);
      ret = EPOCH_WARN_EIGEN_RESIDUAL;
    }
  } else if (residual_out) {
    *residual_out = NAN;
  }
  return ret;
}

namespace {
// Work items of the matrix-core chain kernels (P stage, dlogL/dQ chain): one per
// node, longest segment chain first; and the same with every chain of at least
// chain_split_min segments cut into J parts of about max(4, chain_split_min / 2)
// segments (at most kChainMaxParts), which run in parallel and are combined
// afterwards.
int build_chain_items(EpochInstance* in, const std::vector<int32_t>& off) {  // off: the tree's segment offsets
  const int n = in->n_nodes;
  std::vector<int32_t> order(n);
  for (int v = 0; v < n; ++v) order[v] = v;
  std::stable_sort(order.begin(), order.end(),
                   [&](int32_t a, int32_t b) { return off[a + 1] - off[a] > off[b + 1] - off[b]; });
  std::vector<int4> whole, split, info;
  int max_tail = 0;
  const int part_len = std::max(4, in->chain_split_min / 2);
  for (int v : order) {
    const int m = off[v + 1] - off[v];
    whole.push_back(make_int4(v, 0, m, 0));
    const int J = std::min(kChainMaxParts, (m + part_len - 1) / part_len);
    if (in->chain_split_min > 0 && m >= in->chain_split_min && J >= 2) {
      // J parts [j m / J, (j + 1) m / J); info word: kind 1 | part << 2 | parts << 5 | slot << 9
      const int slot = (int)info.size();
      for (int p = 0; p < J; ++p)
        split.push_back(make_int4(v, p * m / J, (p + 1) * m / J, 1 | (p << 2) | (J << 5) | (slot << 9)));
      info.push_back(make_int4(v, m, J, slot));
      max_tail = std::max(max_tail, m - m / J);
    } else {
      split.push_back(make_int4(v, 0, m, 0));
    }
  }
  std::stable_sort(split.begin(), split.end(), [](const int4& a, const int4& b) { return a.z - a.y > b.z - b.y; });
  in->n_chain_split_items = (int)split.size();
  in->n_chain_splits = (int)info.size();
  in->chain_max_tail = max_tail;
  std::vector<int4> all(whole);
  all.insert(all.end(), split.begin(), split.end());
  all.insert(all.end(), info.begin(), info.end());
  int rc = ensure(in->chain_items, all.size() * sizeof(int4));
  if (!rc && !info.empty())
    rc = ensure(in->chain_scratch,
                info.size() * in->C * kChainMaxParts * 5 * (size_t)in->Kp * in->Kp * sizeof(double));
  if (!rc) rc = upload(in, in->chain_items.ptr, all.data(), all.size() * sizeof(int4));
  return rc;
}
}  // namespace

int set_tree_epochs(EpochInstance* in, const int32_t* parent, const double* height, const double* branch_rate,
                    int32_t n_intervals, const double* boundaries, const int32_t* interval_process) {
  if (!in) return set_error(EPOCH_ERR_ARG, "NULL instance");
  if (n_intervals > in->cfg.max_intervals)
    return set_error(EPOCH_ERR_ARG, "n_intervals %d exceeds max_intervals %d", n_intervals, in->cfg.max_intervals);
  TreePlan plan;
  std::string err;
  if (plan_tree(in->N, parent, height, branch_rate, n_intervals, boundaries, interval_process, in->S, plan, err))
    return set_error(EPOCH_ERR_ARG, "set_tree_epochs: %s", err.c_str());
  const size_t n = in->n_nodes, nseg = plan.seg_process.size(), Nm1 = in->N - 1;
  // int32 block: parent, left, right [n], level_nodes [N-1], seg_offset [n+1], seg_process [nseg]
  std::vector<int32_t> hi;
  hi.reserve(3 * n + Nm1 + n + 1 + nseg);
  hi.insert(hi.end(), plan.parent.begin(), plan.parent.end());
  hi.insert(hi.end(), plan.left.begin(), plan.left.end());
  hi.insert(hi.end(), plan.right.begin(), plan.right.end());
  hi.insert(hi.end(), plan.level_nodes.begin(), plan.level_nodes.end());
  hi.insert(hi.end(), plan.seg_offset.begin(), plan.seg_offset.end());
  hi.insert(hi.end(), plan.seg_process.begin(), plan.seg_process.end());
  std::vector<double> hd;
  hd.reserve(2 * n + 2 * nseg);
  hd.insert(hd.end(), plan.rate.begin(), plan.rate.end());
  hd.insert(hd.end(), plan.tau.begin(), plan.tau.end());
  hd.insert(hd.end(), plan.seg_time.begin(), plan.seg_time.end());
  hd.insert(hd.end(), plan.seg_frac.begin(), plan.seg_frac.end());
  EPOCH_TRY(ensure(in->tree_i, hi.size() * sizeof(int32_t)));
  EPOCH_TRY(ensure(in->tree_d, hd.size() * sizeof(double)));
  EPOCH_TRY(upload(in, in->tree_i.ptr, hi.data(), hi.size() * sizeof(int32_t)));
  EPOCH_TRY(upload(in, in->tree_d.ptr, hd.data(), hd.size() * sizeof(double)));
  int32_t* bi = static_cast<int32_t*>(in->tree_i.ptr);
  in->d_parent = bi;
  in->d_left = bi + n;
  in->d_right = bi + 2 * n;
  in->d_level_nodes = bi + 3 * n;
  in->d_seg_offset = bi + 3 * n + Nm1;
  in->d_seg_process = in->d_seg_offset + n + 1;
  EPOCH_TRY(build_chain_items(in, plan.seg_offset));  // in->plan still holds the previous tree here
  double* bd = static_cast<double*>(in->tree_d.ptr);
  in->d_rate = bd;
  in->d_tau = bd + n;
  in->d_seg_time = bd + 2 * n;
  in->d_seg_frac = bd + 2 * n + nseg;
  if (in->cfg.flags & EPOCH_GRAD_Q) {
    const size_t KK = (size_t)in->Kp * in->Kp, C = in->C;
    // prefix products may be formed in double even for FP32 instances (eig_fp64)
    EPOCH_TRY(ensure(in->qscratch, std::max<size_t>(1, nseg) * C * KK * sizeof(double)));
    std::vector<int32_t> off(in->S + 1, 0), items;
    for (size_t g = 0; g < nseg; ++g) off[plan.seg_process[g] + 1] += (int32_t)C;
    int max_items = 1;
    for (int s = 0; s < in->S; ++s) max_items = std::max(max_items, off[s + 1]);
    for (int s = 0; s < in->S; ++s) off[s + 1] += off[s];
    in->q_chunks = (max_items + in->q_chunk_items - 1) / in->q_chunk_items;
    // generic form: per-segment complex terms + per-process sums; matrix-core form:
    // per-segment real adjoints + chunk partials + per-process sums (complex)
    const size_t S2 = (size_t)in->S * KK * 2;
    const size_t generic_doubles = nseg * C * KK * 2 + S2;
    const size_t mfma_doubles = nseg * C * KK + S2 * in->q_chunks + S2;
    EPOCH_TRY(ensure(in->qseg, std::max(generic_doubles, mfma_doubles) * sizeof(double)));
    // tau of each segment term, then e^{tau lambda} of each eigenvalue (complex)
    EPOCH_TRY(ensure(in->qtau, std::max<size_t>(1, nseg * C) * (1 + 2 * (size_t)in->Kp) * sizeof(double)));
    items.assign(off[in->S], 0);
    std::vector<int32_t> fill(off.begin(), off.end());
    for (size_t g = 0; g < nseg; ++g)
      for (size_t c = 0; c < C; ++c) items[fill[plan.seg_process[g]]++] = (int32_t)(g * C + c);
    std::vector<int32_t> all(off);
    all.insert(all.end(), items.begin(), items.end());
    EPOCH_TRY(ensure(in->seglist, all.size() * sizeof(int32_t)));
    EPOCH_TRY(upload(in, in->seglist.ptr, all.data(), all.size() * sizeof(int32_t)));
  }
  in->plan = std::move(plan);
  if (in->cfg.flags & EPOCH_GRAD_TIME) EPOCH_TRY(tgrad_prepare(in));
  in->dirty.assign(in->n_nodes, 0);
  mark_dirty_all(in);
  in->have_tree = true;
  in->tree_generation++;
  invalidate_downstream(in);
  const int rc = fastpath_tree_changed(in);
  if (rc) in->have_tree = false;  // no evaluation on a half-prepared schedule
  return rc;
}

int update_transition_matrices(EpochInstance* in) {
  if (!in) return set_error(EPOCH_ERR_ARG, "NULL instance");
  if (!in->have_tree) return set_error(EPOCH_ERR_STATE, "set_tree_epochs has not been called");
  if (!in->have_cats) return set_error(EPOCH_ERR_STATE, "epoch_set_categories has not been called");
  for (int s = 0; s < in->S; ++s)
    if (!in->have_eig[s]) return set_error(EPOCH_ERR_STATE, "eigensystem %d has not been set", s);
  EPOCH_TRY(fastpath_pstage(in));
  in->P_valid = true;
  in->partials_valid = false;
  in->logL_valid = false;
  return EPOCH_OK;
}

int update_partials(EpochInstance* in) {
  if (!in) return set_error(EPOCH_ERR_ARG, "NULL instance");
  if (!in->P_valid) return set_error(EPOCH_ERR_STATE, "update_transition_matrices has not been called");
  if (!in->have_tips) return set_error(EPOCH_ERR_STATE, "epoch_set_tip_states has not been called");
  EPOCH_TRY(fastpath_post(in));
  in->partials_valid = true;
  in->logL_valid = false;
  return EPOCH_OK;
}

// The state after a log-likelihood reached the host: -inf (a pattern's
// likelihood is zero in the working precision) is a warning that leaves the
// state queryable but without gradients; NaN or +inf is an error.
static int classify_logL(EpochInstance* in, double v) {
  in->logL_underflow = false;
  if (std::isnan(v) || v == std::numeric_limits<double>::infinity()) {
    in->logL_valid = false;
    return set_error(EPOCH_ERR_NUMERIC, "log-likelihood is not finite (%g)", v);
  }
  in->logL_valid = true;
  if (v == -std::numeric_limits<double>::infinity()) {
    in->logL_underflow = true;
    return set_error(EPOCH_WARN_UNDERFLOW, "a pattern's likelihood is zero in the working precision (logL = -inf)");
  }
  return EPOCH_OK;
}

int root_log_likelihood(EpochInstance* in, double* logL, double* site_logL) {
  if (!in || !logL) return set_error(EPOCH_ERR_ARG, "instance and logL must not be NULL");
  if (!in->partials_valid) return set_error(EPOCH_ERR_STATE, "update_partials has not been called");
  if (!in->have_weights) return set_error(EPOCH_ERR_STATE, "epoch_set_pattern_weights has not been called");
  if (!in->have_pi) return set_error(EPOCH_ERR_STATE, "epoch_set_root_frequencies has not been called");
  EPOCH_TRY(fastpath_root(in));
  EPOCH_TRY(download(in, logL, in->result.ptr, sizeof(double)));
  if (site_logL) EPOCH_TRY(download(in, site_logL, in->site.ptr, (size_t)in->P * sizeof(double)));
  return classify_logL(in, *logL);
}

int log_likelihood_gradient(EpochInstance* in, double* d_branch, double* d_Q) {
  if (!in) return set_error(EPOCH_ERR_ARG, "NULL instance");
  if (d_branch && !(in->cfg.flags & EPOCH_GRAD_BRANCH))
    return set_error(EPOCH_ERR_STATE, "instance created without EPOCH_GRAD_BRANCH");
  if (d_Q && !(in->cfg.flags & EPOCH_GRAD_Q))
    return set_error(EPOCH_ERR_STATE, "instance created without EPOCH_GRAD_Q");
  if (!in->logL_valid) return set_error(EPOCH_ERR_STATE, "root_log_likelihood has not been called for this state");
  if (in->logL_underflow) return set_error(EPOCH_ERR_NUMERIC, "the log-likelihood of this state is -inf: no gradient");
  if (!d_branch && !d_Q) return EPOCH_OK;
  EPOCH_TRY(fastpath_gradient(in, d_Q != nullptr));
  if (d_branch) EPOCH_TRY(download(in, d_branch, in->dbranch.ptr, (size_t)in->n_nodes * sizeof(double)));
  if (d_Q) EPOCH_TRY(download(in, d_Q, in->dQ.ptr, (size_t)in->S * in->K * in->K * sizeof(double)));
  return EPOCH_OK;
}

int epoch_time_gradient(EpochInstance* in, double* d_height, double* d_boundary) {
  if (!in) return set_error(EPOCH_ERR_ARG, "NULL instance");
  if (!(in->cfg.flags & EPOCH_GRAD_TIME)) return set_error(EPOCH_ERR_STATE, "instance created without EPOCH_GRAD_TIME");
  if (!in->logL_valid) return set_error(EPOCH_ERR_STATE, "root_log_likelihood has not been called for this state");
  if (in->logL_underflow) return set_error(EPOCH_ERR_NUMERIC, "the log-likelihood of this state is -inf: no gradient");
  if (!d_height && !d_boundary) return EPOCH_OK;
  if (in->G_gen != in->eval_gen) EPOCH_TRY(fastpath_gradient(in, false));  // the branch adjoints of this state
  double *dh = nullptr, *db = nullptr;
  EPOCH_TRY(launch_time_gradient(in, &dh, &db));
  if (d_height) EPOCH_TRY(download(in, d_height, dh, (size_t)in->n_nodes * sizeof(double)));
  if (d_boundary && in->tg_n_bound > 0)
    EPOCH_TRY(download(in, d_boundary, db, (size_t)in->tg_n_bound * sizeof(double)));
  return EPOCH_OK;
}

int epoch_evaluate(EpochInstance* in, uint32_t what, double* logL, double* site_logL, double* d_branch,
                   double* d_Q) {
  if (!in || !logL) return set_error(EPOCH_ERR_ARG, "instance and logL must not be NULL");
  if (what & ~(EPOCH_EVAL_LOGL | EPOCH_EVAL_GRAD_BRANCH | EPOCH_EVAL_GRAD_Q))
    return set_error(EPOCH_ERR_ARG, "unknown evaluation flags");
  const bool gb = (what & EPOCH_EVAL_GRAD_BRANCH) != 0, gq = (what & EPOCH_EVAL_GRAD_Q) != 0;
  if (gb && !d_branch) return set_error(EPOCH_ERR_ARG, "d_branch must not be NULL with EPOCH_EVAL_GRAD_BRANCH");
  if (gq && !d_Q) return set_error(EPOCH_ERR_ARG, "d_Q must not be NULL with EPOCH_EVAL_GRAD_Q");
  if (gb && !(in->cfg.flags & EPOCH_GRAD_BRANCH))
    return set_error(EPOCH_ERR_STATE, "instance created without EPOCH_GRAD_BRANCH");
  if (gq && !(in->cfg.flags & EPOCH_GRAD_Q)) return set_error(EPOCH_ERR_STATE, "instance created without EPOCH_GRAD_Q");
  if (!in->have_tree) return set_error(EPOCH_ERR_STATE, "set_tree_epochs has not been called");
  if (!in->have_cats) return set_error(EPOCH_ERR_STATE, "epoch_set_categories has not been called");
  for (int s = 0; s < in->S; ++s)
    if (!in->have_eig[s]) return set_error(EPOCH_ERR_STATE, "eigensystem %d has not been set", s);
  if (!in->have_tips) return set_error(EPOCH_ERR_STATE, "epoch_set_tip_states has not been called");
  if (!in->have_weights) return set_error(EPOCH_ERR_STATE, "epoch_set_pattern_weights has not been called");
  if (!in->have_pi) return set_error(EPOCH_ERR_STATE, "epoch_set_root_frequencies has not been called");
  in->P_valid = in->partials_valid = in->logL_valid = false;
  EPOCH_TRY(fastpath_pstage(in));
  EPOCH_TRY(fastpath_post(in));
  EPOCH_TRY(fastpath_root(in));
  if (gb || gq) EPOCH_TRY(fastpath_gradient(in, gq));
  EPOCH_TRY(hip_check(hipMemcpyAsync(logL, in->result.ptr, sizeof(double), hipMemcpyDeviceToHost, in->stream),
                      "logL download"));
  if (site_logL)
    EPOCH_TRY(hip_check(hipMemcpyAsync(site_logL, in->site.ptr, (size_t)in->P * sizeof(double),
                                       hipMemcpyDeviceToHost, in->stream), "site download"));
  if (gb)
    EPOCH_TRY(hip_check(hipMemcpyAsync(d_branch, in->dbranch.ptr, (size_t)in->n_nodes * sizeof(double),
                                       hipMemcpyDeviceToHost, in->stream), "gradient download"));
  if (gq)
    EPOCH_TRY(hip_check(hipMemcpyAsync(d_Q, in->dQ.ptr, (size_t)in->S * in->K * in->K * sizeof(double),
                                       hipMemcpyDeviceToHost, in->stream), "gradient download"));
  EPOCH_TRY(hip_check(hipStreamSynchronize(in->stream), "evaluation sync"));
  in->P_valid = in->partials_valid = true;
  const int rc = classify_logL(in, *logL);
  if (rc == EPOCH_WARN_UNDERFLOW) {  // the gradient pass divided by zero site likelihoods
    if (gb) std::fill(d_branch, d_branch + in->n_nodes, std::numeric_limits<double>::quiet_NaN());
    if (gq) std::fill(d_Q, d_Q + (size_t)in->S * in->K * in->K, std::numeric_limits<double>::quiet_NaN());
  }
  return rc;
}

int epoch_get_kernel_path(EpochInstance* in, int32_t* out) {
  if (!in || !out) return set_error(EPOCH_ERR_ARG, "NULL argument");
  *out = in->path;
  return EPOCH_OK;
}

int epoch_get_transition_matrices(EpochInstance* in, double* out) {
  if (!in || !out) return set_error(EPOCH_ERR_ARG, "NULL argument");
  if (!in->P_valid) return set_error(EPOCH_ERR_STATE, "update_transition_matrices has not been called");
  const size_t n = in->n_nodes, C = in->C, Kp = in->Kp, K = in->K, KK = Kp * Kp;
  std::vector<char> raw(n * C * KK * in->real_size);
  EPOCH_TRY(download(in, raw.data(), in->Pm.ptr, raw.size()));
  for (size_t v = 0; v < n; ++v)
    for (size_t c = 0; c < C; ++c)
      for (size_t i = 0; i < K; ++i)
        for (size_t j = 0; j < K; ++j) {
          const size_t src = (v * C + c) * KK + i * Kp + j;
          double x = in->fp64 ? reinterpret_cast<double*>(raw.data())[src] : reinterpret_cast<float*>(raw.data())[src];
          if ((int)v == in->plan.root) x = 0.0;
          out[((v * C + c) * K + i) * K + j] = x;
        }
  return EPOCH_OK;
}

int epoch_plan_segments(int32_t n_tips, const int32_t* parent, const double* height, int32_t n_intervals,
                        const double* boundaries, const int32_t* interval_process, int32_t n_processes,
                        int32_t capacity, int32_t* seg_offset, int32_t* seg_process, double* seg_time,
                        int32_t* n_segments) {
  g_error.clear();
  if (!seg_offset || !n_segments) return set_error(EPOCH_ERR_ARG, "NULL output");
  TreePlan plan;
  std::string err;
  if (plan_tree(n_tips, parent, height, nullptr, n_intervals, boundaries, interval_process, n_processes, plan, err))
    return set_error(EPOCH_ERR_ARG, "%s", err.c_str());
  const int nseg = (int)plan.seg_process.size();
  *n_segments = nseg;
  std::copy(plan.seg_offset.begin(), plan.seg_offset.end(), seg_offset);
  if (nseg > capacity) return set_error(EPOCH_ERR_ARG, "capacity %d < %d segments", capacity, nseg);
  std::copy(plan.seg_process.begin(), plan.seg_process.end(), seg_process);
  std::copy(plan.seg_time.begin(), plan.seg_time.end(), seg_time);
  return EPOCH_OK;
}

int epoch_workspace_bytes(const EpochConfig* cfg, int64_t* out) {
  g_error.clear();
  if (!cfg || !out) return set_error(EPOCH_ERR_ARG, "cfg and out must not be NULL");
  if (cfg->n_tips < 2 || cfg->n_patterns < 1 || cfg->n_states < 2 || cfg->n_states > 64 || cfg->n_categories < 1 ||
      cfg->n_categories > kMaxCategories || (cfg->precision != EPOCH_FP32 && cfg->precision != EPOCH_FP64))
    return set_error(EPOCH_ERR_ARG, "invalid configuration");
  *out = (int64_t)workspace_total(*cfg, padded_states(*cfg));
  return EPOCH_OK;
}

int epoch_set_option(EpochInstance* in, int32_t key, int64_t value) {
  if (!in) return set_error(EPOCH_ERR_ARG, "NULL instance");
  // options change launch shapes and may reallocate schedules and work lists:
  // a batch holding this instance captures its graph again
  in->option_generation++;
  mark_dirty_all(in);
  switch (key) {
    case EPOCH_OPT_INCREMENTAL:
      if (value != 0 && value != 1) return set_error(EPOCH_ERR_ARG, "EPOCH_OPT_INCREMENTAL takes 0 or 1");
      in->inc_enable = (int)value;
      return EPOCH_OK;
    case EPOCH_OPT_TREE_WALK:
      if (value < -1 || value > 1) return set_error(EPOCH_ERR_ARG, "EPOCH_OPT_TREE_WALK takes -1, 0 or 1");
      if (in->budget > 0 && in->path == 1 && value != 1)
        return set_error(EPOCH_ERR_ARG, "an HBM budget needs the tree walk");
      in->walk_enable = (int)value;
      break;
    case EPOCH_OPT_WALK_RECOMPUTE:
      if (value < 2 || value > in->N) return set_error(EPOCH_ERR_ARG, "EPOCH_OPT_WALK_RECOMPUTE takes 2..N");
      if (in->budget > 0 && in->path == 1)
        return set_error(EPOCH_ERR_ARG, "under an HBM budget the budget sets the recomputation");
      in->walk_recompute = (int)value;
      break;
    case EPOCH_OPT_WALK_BLOCKS:
      if (value < 0 || value > (1 << 30)) return set_error(EPOCH_ERR_ARG, "EPOCH_OPT_WALK_BLOCKS out of range");
      in->walk_blocks = (int)value;
      return EPOCH_OK;
    case EPOCH_OPT_WALK_TILES:
      if (value != 1 && value != 2) return set_error(EPOCH_ERR_ARG, "EPOCH_OPT_WALK_TILES takes 1 or 2");
      in->walk_nt = (int)value;
      break;
    case EPOCH_OPT_LEVEL_MIN_TILES:
      if (value < 1 || value > 64) return set_error(EPOCH_ERR_ARG, "EPOCH_OPT_LEVEL_MIN_TILES takes 1..64");
      in->nuc_rmin = (int)value;
      if (int rc = fastpath_init(in)) return rc;
      break;
    case EPOCH_OPT_CHAIN_SPLIT:
      if (value < 0 || value > (1 << 30)) return set_error(EPOCH_ERR_ARG, "EPOCH_OPT_CHAIN_SPLIT out of range");
      in->chain_split_min = (int)value;
      // the parts' scratch (prefixes, suffixes) belongs to the P stage that formed it: evaluate again
      in->P_valid = in->partials_valid = in->logL_valid = false;
      in->pstage_split = false;
      if (in->have_tree) {
        if (int rc = build_chain_items(in, in->plan.seg_offset)) return rc;
      }
      return EPOCH_OK;
    case EPOCH_OPT_TARGET_BLOCKS:
      if (value < 1 || value > (1 << 30)) return set_error(EPOCH_ERR_ARG, "EPOCH_OPT_TARGET_BLOCKS out of range");
      in->codon_target_blocks = (int)value;
      break;
    case EPOCH_OPT_EIGEN_PRECISION:
      if (value < 0 || value > 2) return set_error(EPOCH_ERR_ARG, "EPOCH_OPT_EIGEN_PRECISION takes 0, 1 or 2");
      in->eig_mode = (int)value;
      choose_eig_precision(in);
      in->P_valid = in->partials_valid = in->logL_valid = false;
      in->pstage_split = false;
      return EPOCH_OK;
    case EPOCH_OPT_SPLIT_BLOCKS:
      if (value < 0 || value > (1 << 30)) return set_error(EPOCH_ERR_ARG, "EPOCH_OPT_SPLIT_BLOCKS out of range");
      in->codon_split_blocks = (int)value;
      break;
    default:
      return set_error(EPOCH_ERR_ARG, "unknown option %d", key);
  }
  in->partials_valid = in->logL_valid = false;
  if (!in->have_tree) return EPOCH_OK;
  const int rc = fastpath_tree_changed(in);
  if (rc) in->have_tree = false;
  return rc;
}

int epoch_plan_walk(int32_t n_tips, const int32_t* parent, const double* height, int32_t recompute_tips,
                    int32_t capacity, int32_t* ops, int32_t* counts) {
  g_error.clear();
  if (!counts || (capacity > 0 && !ops)) return set_error(EPOCH_ERR_ARG, "NULL output");
  if (recompute_tips < 2) return set_error(EPOCH_ERR_ARG, "recompute_tips must be >= 2");
  TreePlan plan;
  std::string err;
  const int32_t phi = 0;
  if (plan_tree(n_tips, parent, height, nullptr, 1, nullptr, &phi, 1, plan, err))
    return set_error(EPOCH_ERR_ARG, "%s", err.c_str());
  WalkProgram w;
  const int rc = build_walk_programs(plan, recompute_tips, w);
  counts[0] = (int32_t)(w.post.size() / 4);
  counts[1] = (int32_t)(w.pre.size() / 4);
  counts[2] = w.post_slots;
  counts[3] = w.pre_slots;
  if (rc) return set_error(EPOCH_ERR_ARG, "tree needs more than %d stack slots", kWalkMaxSlots);
  const int n_ops = counts[0] + counts[1];
  if (n_ops > capacity) return set_error(EPOCH_ERR_ARG, "capacity %d < %d operations", capacity, n_ops);
  std::copy(w.post.begin(), w.post.end(), ops);
  std::copy(w.pre.begin(), w.pre.end(), ops + w.post.size());
  return EPOCH_OK;
}

}  // extern "C"
