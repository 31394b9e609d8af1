// Four-state helpers shared by the level kernels and the tree-walk kernels:
// 4-vectors and 4x4 matrices held in registers, and reductions over the CP
// adjacent lanes that hold the categories of one pattern.
#pragma once
#include <hip/hip_runtime.h>
#include <cstdint>

namespace epochlik {
namespace nuc {

template <typename T>
struct alignas(4 * sizeof(T)) V4 {
  T v[4];
};

// Store of a pattern's 4-vector that no other block of the launch reads.  In
// FP32 a non-temporal vector store, so the streamed output does not displace
// the launch's inputs from L2 (C2: 1.7 % faster); in FP64 the plain store
// measured faster.
template <typename T>
__device__ inline void store_streaming(V4<T>* dst, const V4<T>& x) {
  if constexpr (sizeof(T) == 4) {
    typedef T vec4 __attribute__((ext_vector_type(4)));
    __builtin_nontemporal_store(vec4{x.v[0], x.v[1], x.v[2], x.v[3]}, reinterpret_cast<vec4*>(dst));
  } else {
    *dst = x;
  }
}

template <typename T>
struct M4 {
  T m[16];
};

// Tip states of the 4-state kernels are state sets: bit i set = state i
// possible (text after Eq. 4: a tip is a 0/1 indicator of the (partially)
// observed state; one state, an ambiguity set, or all four when missing).
template <typename T>
__device__ inline V4<T> onehot(int mask) {
  V4<T> r;
#pragma unroll
  for (int i = 0; i < 4; ++i) r.v[i] = ((mask >> i) & 1) ? T(1) : T(0);
  return r;
}

template <typename T>
__device__ inline V4<T> matvec(const M4<T>& M, const V4<T>& x) {
  V4<T> y;
#pragma unroll
  for (int i = 0; i < 4; ++i) {
    T s = M.m[4 * i] * x.v[0];
#pragma unroll
    for (int j = 1; j < 4; ++j) s += M.m[4 * i + j] * x.v[j];
    y.v[i] = s;
  }
  return y;
}

template <typename T>
__device__ inline V4<T> matvec_t(const M4<T>& M, const V4<T>& x) {
  V4<T> y;
#pragma unroll
  for (int j = 0; j < 4; ++j) {
    T s = M.m[j] * x.v[0];
#pragma unroll
    for (int i = 1; i < 4; ++i) s += M.m[4 * i + j] * x.v[i];
    y.v[j] = s;
  }
  return y;
}

template <typename T>
__device__ inline T max4(const V4<T>& x) {
  T a = x.v[0] > x.v[1] ? x.v[0] : x.v[1];
  T b = x.v[2] > x.v[3] ? x.v[2] : x.v[3];
  return a > b ? a : b;
}

template <typename T>
__device__ inline M4<T> load_matrix(const T* __restrict__ p) {
  M4<T> M;
  const V4<T>* q = reinterpret_cast<const V4<T>*>(p);
#pragma unroll
  for (int r = 0; r < 4; ++r) {
    const V4<T> row = q[r];
#pragma unroll
    for (int j = 0; j < 4; ++j) M.m[4 * r + j] = row.v[j];
  }
  return M;
}

// Lane exchange inside groups of CP adjacent lanes.  Offsets 1 and 2 use DPP
// quad permutations (no LDS traffic); offset 4 (CP = 8 only) uses ds_bpermute.
template <int OFF>
__device__ inline float xor_lanes(float v) {
  if constexpr (OFF == 1)
    return __int_as_float(__builtin_amdgcn_mov_dpp(__float_as_int(v), 0xB1, 0xF, 0xF, false));
  else if constexpr (OFF == 2)
    return __int_as_float(__builtin_amdgcn_mov_dpp(__float_as_int(v), 0x4E, 0xF, 0xF, false));
  else
    return __shfl_xor(v, OFF, 64);
}
template <int OFF>
__device__ inline double xor_lanes(double v) {
  if constexpr (OFF == 1 || OFF == 2) {
    const long long b = __double_as_longlong(v);
    const int ctrl = OFF == 1 ? 0xB1 : 0x4E;
    const int l = __builtin_amdgcn_mov_dpp((int)(b & 0xffffffffLL), ctrl, 0xF, 0xF, false);
    const int h = __builtin_amdgcn_mov_dpp((int)(b >> 32), ctrl, 0xF, 0xF, false);
    return __longlong_as_double(((long long)h << 32) | (unsigned int)l);
  } else {
    return __shfl_xor(v, OFF, 64);
  }
}

template <int CP, typename T>
__device__ inline T group_max_cp(T v) {
  if constexpr (CP >= 2) { const T u = xor_lanes<1>(v); v = u > v ? u : v; }
  if constexpr (CP >= 4) { const T u = xor_lanes<2>(v); v = u > v ? u : v; }
  if constexpr (CP >= 8) { const T u = xor_lanes<4>(v); v = u > v ? u : v; }
  return v;
}
template <int CP, typename T>
__device__ inline T group_sum_cp(T v) {
  if constexpr (CP >= 2) v += xor_lanes<1>(v);
  if constexpr (CP >= 4) v += xor_lanes<2>(v);
  if constexpr (CP >= 8) v += xor_lanes<4>(v);
  return v;
}

}  // namespace nuc
}  // namespace epochlik
