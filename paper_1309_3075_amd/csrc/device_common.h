// Device helpers shared by the HIP kernels of the library.
#pragma once
#include <hip/hip_runtime.h>
#include <cstdint>

namespace epochlik {

constexpr int kMaxCategories = 8;
constexpr int kBlock = 256;
constexpr double kLn2 = 0.69314718055994530942;

// Power-of-two rescaling: returns e such that m * 2^-e lies in [0.5, 1) for m > 0
// (0 when m == 0 or not finite).  Exact for any rounding mode.
__device__ inline int scale_exponent(float m) {
  if (!(m > 0.0f) || !isfinite(m)) return 0;
  int e;
  frexpf(m, &e);
  return e;
}
__device__ inline int scale_exponent(double m) {
  if (!(m > 0.0) || !isfinite(m)) return 0;
  int e;
  frexp(m, &e);
  return e;
}
__device__ inline float scale_by_pow2(float x, int e) { return ldexpf(x, -e); }
__device__ inline double scale_by_pow2(double x, int e) { return ldexp(x, -e); }

__device__ inline float dev_exp(float x) { return expf(x); }
__device__ inline double dev_exp(double x) { return exp(x); }
__device__ inline float dev_expm1(float x) { return expm1f(x); }
__device__ inline double dev_expm1(double x) { return expm1(x); }
__device__ inline float dev_cos(float x) { return cosf(x); }
__device__ inline double dev_cos(double x) { return cos(x); }
__device__ inline float dev_sin(float x) { return sinf(x); }
__device__ inline double dev_sin(double x) { return sin(x); }

// Reductions within groups of W consecutive lanes of a 64-wide wavefront.
template <int W, typename T>
__device__ inline T group_max(T v) {
#pragma unroll
  for (int o = W / 2; o > 0; o >>= 1) {
    T u = __shfl_xor(v, o, W);
    v = u > v ? u : v;
  }
  return v;
}
template <int W, typename T>
__device__ inline T group_sum(T v) {
#pragma unroll
  for (int o = W / 2; o > 0; o >>= 1) v += __shfl_xor(v, o, W);
  return v;
}

// Deterministic block-wide sum of doubles (fixed tree order), result on thread 0.
template <int NT>
__device__ inline double block_sum(double v, double* smem) {
  const int t = threadIdx.x;
  smem[t] = v;
  __syncthreads();
#pragma unroll
  for (int s = NT / 2; s > 0; s >>= 1) {
    if (t < s) smem[t] += smem[t + s];
    __syncthreads();
  }
  double r = smem[0];
  __syncthreads();
  return r;
}

}  // namespace epochlik
