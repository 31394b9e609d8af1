// Attainable-bandwidth probes: plain copy, read-only and write-only streams over
// library-allocated buffers, timed with HIP events.  They give the measured
// ceiling that the likelihood kernels' HBM throughput is compared with.
#include <hip/hip_runtime.h>

#include "../../include/epochlik.h"
#include "device_common.h"
#include "instance.h"

namespace epochlik {
namespace {

typedef float vf4 __attribute__((ext_vector_type(4)));

// Each thread keeps four 16-byte loads in flight before it stores; stores are
// non-temporal, so the streamed output does not evict what is still to be read.
__global__ __launch_bounds__(256) void probe_copy(const vf4* __restrict__ src, vf4* __restrict__ dst, size_t n) {
  const size_t stride = (size_t)gridDim.x * 256;
  size_t i = blockIdx.x * 256ull + threadIdx.x;
  for (; i + 3 * stride < n; i += 4 * stride) {
    const vf4 a = src[i], b = src[i + stride], c = src[i + 2 * stride], d = src[i + 3 * stride];
    __builtin_nontemporal_store(a, dst + i);
    __builtin_nontemporal_store(b, dst + i + stride);
    __builtin_nontemporal_store(c, dst + i + 2 * stride);
    __builtin_nontemporal_store(d, dst + i + 3 * stride);
  }
  for (; i < n; i += stride) __builtin_nontemporal_store(src[i], dst + i);
}

__global__ __launch_bounds__(256) void probe_read(const vf4* __restrict__ src, float* __restrict__ out, size_t n) {
  float acc = 0.f;
  for (size_t i = blockIdx.x * 256ull + threadIdx.x; i < n; i += (size_t)gridDim.x * 256) {
    const vf4 v = src[i];
    acc += (v.x + v.y) + (v.z + v.w);
  }
  if (acc == 123.456f) out[0] = acc;  // keeps the loads live; never true for the zero-filled input
}

__global__ __launch_bounds__(256) void probe_write(vf4* __restrict__ dst, size_t n) {
  const vf4 v = {0.f, 1.f, 2.f, 3.f};
  for (size_t i = blockIdx.x * 256ull + threadIdx.x; i < n; i += (size_t)gridDim.x * 256)
    __builtin_nontemporal_store(v, dst + i);
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
  hipEvent_t e0, e1;
  if (!rc) rc = hip_check(hipEventCreate(&e0), "probe event");
  if (!rc) rc = hip_check(hipEventCreate(&e1), "probe event");
  const int grid = 256 * 16;
  auto launch = [&]() {
    if (kind == 0)
      hipLaunchKernelGGL(probe_copy, dim3(grid), dim3(256), 0, nullptr, (const vf4*)a, (vf4*)b, n);
    else if (kind == 1)
      hipLaunchKernelGGL(probe_read, dim3(grid), dim3(256), 0, nullptr, (const vf4*)a, (float*)a, n);
    else
      hipLaunchKernelGGL(probe_write, dim3(grid), dim3(256), 0, nullptr, (vf4*)a, n);
  };
  if (!rc) {
    launch();  // warm-up
    rc = hip_check(hipEventRecord(e0, nullptr), "probe record");
    for (int k = 0; k < iters && !rc; ++k) launch();
    if (!rc) rc = hip_check(hipEventRecord(e1, nullptr), "probe record");
    if (!rc) rc = hip_check(hipEventSynchronize(e1), "probe sync");
    float ms = 0.f;
    if (!rc) rc = hip_check(hipEventElapsedTime(&ms, e0, e1), "probe elapsed");
    if (!rc) {
      const double moved = (double)n * 16 * (kind == 0 ? 2.0 : 1.0) * iters;
      *gbs = moved / (ms * 1e-3) / 1e9;
    }
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
  }
  (void)hipFree(a);
  if (b) (void)hipFree(b);
  return rc;
}
