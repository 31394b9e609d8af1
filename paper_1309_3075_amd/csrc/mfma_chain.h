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

// out[b] (+)= (in[b] M) for NB stripes held transposed (see the chain kernels):
// the A operand of k-step (t, q) is row 16 t + 4 g + q of the Kp x Kp matrix M
// at column 16 mt + arow.  The 4 NT operands of tile t + 1 are loaded while the
// MFMAs of tile t run, so a step waits on memory about once instead of once per
// instruction.
// Operands of k-step tile t of a stripe product by M (see stripe_gemm).
template <typename T, int NT>
__device__ inline void stripe_load(const T* __restrict__ M, int t, int g, int arow, T (&a)[4][NT]) {
  constexpr int Kp = 16 * NT;
#pragma unroll
  for (int q = 0; q < 4; ++q)
#pragma unroll
    for (int mt = 0; mt < NT; ++mt) a[q][mt] = M[(16 * t + 4 * g + q) * Kp + 16 * mt + arow];
}

// stripe_gemm with the operands of tile 0 already in a[0] (loaded earlier by
// stripe_load, so that their latency overlaps other work).
template <typename T, int NT, int NB>
__device__ inline void stripe_gemm_from(const T* __restrict__ M, int g, int arow, T (&a)[2][4][NT],
                                        const typename Mfma<T>::acc (&in)[NB][NT],
                                        typename Mfma<T>::acc (&out)[NB][NT]) {
#pragma unroll
  for (int t = 0; t < NT; ++t) {
    if (t + 1 < NT) stripe_load<T, NT>(M, t + 1, g, arow, a[(t + 1) & 1]);
#pragma unroll
    for (int q = 0; q < 4; ++q)
#pragma unroll
      for (int mt = 0; mt < NT; ++mt)
#pragma unroll
        for (int b = 0; b < NB; ++b) out[b][mt] = Mfma<T>::mma(a[t & 1][q][mt], in[b][t][q], out[b][mt]);
  }
}

template <typename T, int NT, int NB>
__device__ inline void stripe_gemm(const T* __restrict__ M, int g, int arow,
                                   const typename Mfma<T>::acc (&in)[NB][NT],
                                   typename Mfma<T>::acc (&out)[NB][NT]) {
  T a[2][4][NT];
  stripe_load<T, NT>(M, 0, g, arow, a[0]);
  stripe_gemm_from<T, NT, NB>(M, g, arow, a, in, out);
}

// Orders the LDS accesses of one wavefront (a write, then reads by other lanes).
__device__ inline void wave_lds_sync() {
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
  __builtin_amdgcn_wave_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

}  // namespace epochlik
