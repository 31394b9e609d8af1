// Matrix-core helpers for the chain kernels (products of K x K matrices kept
// as transposed 16-row stripes in accumulator registers).
#pragma once
#include <hip/hip_runtime.h>

namespace epochlik {

typedef float f32x4 __attribute__((ext_vector_type(4)));
typedef double f64x4 __attribute__((ext_vector_type(4)));

template <typename T>
struct Mfma;
// Both instructions take A[m][k] from lane m + 16 k and B[k][n] from lane
// n + 16 k.  The FP32 one returns D[m][n] in lane n + 16 (m / 4), register
// m % 4; the FP64 one in lane n + 16 (m % 4), register m / 4.  a_row(n) is the
// row of the 16-column block that lane n's A operand carries, chosen so that
// register v of lane (g, n) always ends up holding row 4 g + v.
template <>
struct Mfma<float> {
  using acc = f32x4;
  __device__ static inline acc mma(float a, float b, acc c) {
    return __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c, 0, 0, 0);
  }
  __device__ static inline int a_row(int n) { return n; }
};
template <>
struct Mfma<double> {
  using acc = f64x4;
  __device__ static inline acc mma(double a, double b, acc c) {
    return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0);
  }
  __device__ static inline int a_row(int n) { return 4 * (n & 3) + (n >> 2); }
};

template <typename T>
struct ColCoef {
  T ms, mo, dms, dmo;  // (E - I) and dE/dl acting on column j with its partner j ^ 1
};

template <typename T, typename TO>
__device__ inline void store4(TO* dst, const typename Mfma<T>::acc& x);
template <>
__device__ inline void store4<float, float>(float* dst, const f32x4& x) {
  *reinterpret_cast<f32x4*>(dst) = x;
}
template <>
__device__ inline void store4<double, double>(double* dst, const f64x4& x) {
  reinterpret_cast<double2*>(dst)[0] = make_double2(x[0], x[1]);
  reinterpret_cast<double2*>(dst)[1] = make_double2(x[2], x[3]);
}
template <>
__device__ inline void store4<double, float>(float* dst, const f64x4& x) {
  *reinterpret_cast<float4*>(dst) = make_float4(float(x[0]), float(x[1]), float(x[2]), float(x[3]));
}

// Orders the LDS accesses of one wavefront (a write, then reads by other lanes).
__device__ inline void wave_lds_sync() {
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
  __builtin_amdgcn_wave_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

}  // namespace epochlik
