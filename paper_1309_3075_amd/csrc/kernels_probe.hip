// Attainable-bandwidth probes: plain copy, read-only and write-only streams over
// library-allocated buffers, timed with HIP events.  They give the measured
// ceiling that the likelihood kernels' HBM throughput is compared with.
#include <hip/hip_runtime.h>

#include <algorithm>

#include "../../include/epochlik.h"
#include "device_common.h"
#include "instance.h"

namespace epochlik {
namespace {

typedef float vf4 __attribute__((ext_vector_type(4)));

// The element range of one block: CHUNK = each block streams its own contiguous
// part of the buffer (many concurrent streams); otherwise the whole grid sweeps
// the buffer together (element i at grid stride).  Writes are non-temporal, so
// the streamed output does not evict what is still to be read.  On MI355X the
// write and copy rates depend on this shape (2 GiB: grid-stride writes from
// 4,096 blocks 3.9 TB/s, block-contiguous 5.5 TB/s), so the probes time several
// shapes and report the best.
struct Range {
  size_t begin, end, step;
};
template <bool CHUNK>
__device__ inline Range block_range(size_t n) {
  if constexpr (CHUNK) {
    const size_t per = (n + gridDim.x - 1) / gridDim.x;
    const size_t b = (size_t)blockIdx.x * per;
    return {b + threadIdx.x, b + per < n ? b + per : n, 256};
  } else {
    return {(size_t)blockIdx.x * 256 + threadIdx.x, n, (size_t)gridDim.x * 256};
  }
}

// Each thread keeps four 16-byte loads in flight before it stores.
template <bool CHUNK>
__global__ __launch_bounds__(256) void probe_copy(const vf4* __restrict__ src, vf4* __restrict__ dst, size_t n) {
  const Range r = block_range<CHUNK>(n);
  size_t i = r.begin;
  for (; i + 3 * r.step < r.end; i += 4 * r.step) {
    const vf4 a = src[i], b = src[i + r.step], c = src[i + 2 * r.step], d = src[i + 3 * r.step];
    __builtin_nontemporal_store(a, dst + i);
    __builtin_nontemporal_store(b, dst + i + r.step);
    __builtin_nontemporal_store(c, dst + i + 2 * r.step);
    __builtin_nontemporal_store(d, dst + i + 3 * r.step);
  }
  for (; i < r.end; i += r.step) __builtin_nontemporal_store(src[i], dst + i);
}

template <bool CHUNK>
__global__ __launch_bounds__(256) void probe_read(const vf4* __restrict__ src, float* __restrict__ out, size_t n) {
  const Range r = block_range<CHUNK>(n);
  float acc = 0.f;
  for (size_t i = r.begin; i < r.end; i += r.step) {
    const vf4 v = src[i];
    acc += (v.x + v.y) + (v.z + v.w);
  }
  if (acc == 123.456f) out[0] = acc;  // keeps the loads live; never true for the zero-filled input
}

template <bool CHUNK>
__global__ __launch_bounds__(256) void probe_write(vf4* __restrict__ dst, size_t n) {
  const vf4 v = {0.f, 1.f, 2.f, 3.f};
  const Range r = block_range<CHUNK>(n);
  for (size_t i = r.begin; i < r.end; i += r.step) __builtin_nontemporal_store(v, dst + i);
}

}  // namespace
}  // namespace epochlik

using namespace epochlik;

extern "C" int epoch_bandwidth_probe(int64_t bytes, int32_t kind, int32_t iters, double* gbs) {
  if (bytes < (1 << 20) || bytes > ((int64_t)64 << 30) || kind < 0 || kind > 2 || iters < 1 || !gbs)
    return set_error(EPOCH_ERR_ARG, "probe: bytes in [1 MiB, 64 GiB], kind 0..2, iters >= 1, gbs required");
  const size_t n = (size_t)bytes / 16;
  void *a = nullptr, *b = nullptr;
  if (hipMalloc(&a, n * 16) != hipSuccess) return set_error(EPOCH_ERR_OOM, "probe: hipMalloc failed");
  if (kind == 0 && hipMalloc(&b, n * 16) != hipSuccess) {
    (void)hipFree(a);
    return set_error(EPOCH_ERR_OOM, "probe: hipMalloc failed");
  }
  int rc = hip_check(hipMemset(a, 0, n * 16), "probe memset");
  hipEvent_t e0 = nullptr, e1 = nullptr;
  if (!rc) rc = hip_check(hipEventCreate(&e0), "probe event");
  if (!rc) rc = hip_check(hipEventCreate(&e1), "probe event");
  // launch shapes tried: grid-stride and block-contiguous, at 1,024 .. 65,536 blocks
  auto launch = [&](int grid, bool chunk) {
    if (kind == 0)
      hipLaunchKernelGGL(chunk ? probe_copy<true> : probe_copy<false>, dim3(grid), dim3(256), 0, nullptr,
                         (const vf4*)a, (vf4*)b, n);
    else if (kind == 1)
      hipLaunchKernelGGL(chunk ? probe_read<true> : probe_read<false>, dim3(grid), dim3(256), 0, nullptr,
                         (const vf4*)a, (float*)a, n);
    else
      hipLaunchKernelGGL(chunk ? probe_write<true> : probe_write<false>, dim3(grid), dim3(256), 0, nullptr, (vf4*)a,
                         n);
  };
  double best = 0.0;
  for (int grid : {1024, 4096, 16384, 65536})
    for (bool chunk : {false, true}) {
      if (rc) break;
      launch(grid, chunk);  // warm-up
      rc = hip_check(hipEventRecord(e0, nullptr), "probe record");
      for (int k = 0; k < iters && !rc; ++k) launch(grid, chunk);
      if (!rc) rc = hip_check(hipEventRecord(e1, nullptr), "probe record");
      if (!rc) rc = hip_check(hipEventSynchronize(e1), "probe sync");
      float ms = 0.f;
      if (!rc) rc = hip_check(hipEventElapsedTime(&ms, e0, e1), "probe elapsed");
      if (!rc) {
        const double moved = (double)n * 16 * (kind == 0 ? 2.0 : 1.0) * iters;
        best = std::max(best, moved / (ms * 1e-3) / 1e9);
      }
    }
  if (!rc) *gbs = best;
  if (e0) (void)hipEventDestroy(e0);
  if (e1) (void)hipEventDestroy(e1);
  (void)hipFree(a);
  if (b) (void)hipFree(b);
  return rc;
}
