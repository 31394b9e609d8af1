// Specialised 4-state (nucleotide) kernels, FP32 or FP64.
//
// Layout (shared with the generic kernels): partials [slot][c][P][4] with
// slot = node - N; transition matrices [node][c][4][4] row-major.
//
// A block covers one internal node and 64 patterns; wavefront c of the block
// handles rate category c, so the 4x4 matrices it multiplies by are uniform
// across the wavefront and live in scalar registers.  The categories of a
// pattern share one power-of-two scale factor; they agree on it through LDS.
//   nuc_post_level : Felsenstein pruning for one tree level (Eq. 4), with the
//                    cumulative scale exponent of each node's subtree.
//   nuc_root       : root sum over pi and categories (text after Eq. 4), FP64.
//   nuc_pre_level  : outside vectors of one level plus the per-branch
//                    accumulation of dlogL/dP over R pattern tiles, reduced
//                    across the wavefront with a reduce-scatter butterfly.
#include <hip/hip_runtime.h>

#include "device_common.h"
#include "instance.h"

namespace epochlik {

namespace {

template <typename T>
struct alignas(4 * sizeof(T)) V4 {
  T v[4];
};

template <typename T>
__device__ inline V4<T> onehot(int st) {
  V4<T> r;
#pragma unroll
  for (int i = 0; i < 4; ++i) r.v[i] = (st >= 4 || st == i) ? T(1) : T(0);
  return r;
}

// y = M x with M row-major 4x4 at a wavefront-uniform address
template <typename T>
__device__ inline V4<T> matvec(const T* __restrict__ M, const V4<T>& x) {
  V4<T> y;
#pragma unroll
  for (int i = 0; i < 4; ++i) {
    T s = M[4 * i] * x.v[0];
#pragma unroll
    for (int j = 1; j < 4; ++j) s += M[4 * i + j] * x.v[j];
    y.v[i] = s;
  }
  return y;
}

// y = M^T x
template <typename T>
__device__ inline V4<T> matvec_t(const T* __restrict__ M, const V4<T>& x) {
  V4<T> y;
#pragma unroll
  for (int j = 0; j < 4; ++j) {
    T s = M[j] * x.v[0];
#pragma unroll
    for (int i = 1; i < 4; ++i) s += M[4 * i + j] * x.v[i];
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
__device__ inline V4<T> load_child(int child, int N, int c, int C, int P, int pc, const uint8_t* __restrict__ tips,
                                   const V4<T>* __restrict__ part) {
  if (child < N) return onehot<T>(tips[(size_t)child * P + pc]);
  return part[((size_t)(child - N) * C + c) * P + pc];
}

__device__ inline int wave_uniform(int x) { return __builtin_amdgcn_readfirstlane(x); }

// ---------------------------------------------------------------------------
template <typename T, int C>
__global__ __launch_bounds__(C * 64) void nuc_post_level_kernel(
    const int32_t* __restrict__ nodes, const int32_t* __restrict__ left, const int32_t* __restrict__ right,
    const T* __restrict__ Pm, const uint8_t* __restrict__ tips, V4<T>* __restrict__ part,
    int32_t* __restrict__ scale_cum, int N, int P) {
  __shared__ T smax[C][64];
  const int c = wave_uniform(threadIdx.x >> 6);
  const int lane = threadIdx.x & 63;
  const int u = nodes[blockIdx.y];
  const int a = left[u], b = right[u];
  const int p = blockIdx.x * 64 + lane;
  const bool pok = p < P;
  const int pc = pok ? p : P - 1;
  const V4<T> xa = load_child<T>(a, N, c, C, P, pc, tips, part);
  const V4<T> xb = load_child<T>(b, N, c, C, P, pc, tips, part);
  const V4<T> va = matvec(Pm + ((size_t)a * C + c) * 16, xa);
  const V4<T> vb = matvec(Pm + ((size_t)b * C + c) * 16, xb);
  V4<T> x;
#pragma unroll
  for (int i = 0; i < 4; ++i) x.v[i] = va.v[i] * vb.v[i];
  T m = max4(x);
  if constexpr (C > 1) {
    smax[c][lane] = m;
    __syncthreads();
#pragma unroll
    for (int k = 0; k < C; ++k) m = smax[k][lane] > m ? smax[k][lane] : m;
  }
  const int e = scale_exponent(m);
#pragma unroll
  for (int i = 0; i < 4; ++i) x.v[i] = scale_by_pow2(x.v[i], e);
  if (pok) {
    part[((size_t)(u - N) * C + c) * P + p] = x;
    if (c == 0) {
      int s = e;
      if (a >= N) s += scale_cum[(size_t)(a - N) * P + p];
      if (b >= N) s += scale_cum[(size_t)(b - N) * P + p];
      scale_cum[(size_t)(u - N) * P + p] = s;
    }
  }
}

// ---------------------------------------------------------------------------
template <typename T, int C>
__global__ __launch_bounds__(C * 64) void nuc_root_kernel(
    const V4<T>* __restrict__ rootp, const int32_t* __restrict__ scale_root, const double* __restrict__ pi,
    const double* __restrict__ cat, const double* __restrict__ weights, double* __restrict__ site,
    double* __restrict__ block_out, int P) {
  __shared__ double sl[C][64];
  const int c = wave_uniform(threadIdx.x >> 6);
  const int lane = threadIdx.x & 63;
  const int p = blockIdx.x * 64 + lane;
  const bool pok = p < P;
  const int pc = pok ? p : P - 1;
  const V4<T> x = rootp[(size_t)c * P + pc];
  double l = 0.0;
#pragma unroll
  for (int i = 0; i < 4; ++i) l += pi[i] * (double)x.v[i];
  sl[c][lane] = cat[kMaxCategories + c] * l;
  __syncthreads();
  if (c == 0) {
    double L = 0.0;
#pragma unroll
    for (int k = 0; k < C; ++k) L += sl[k][lane];
    double contrib = 0.0;
    if (pok) {
      const double s = log(L) + (double)scale_root[p] * kLn2;
      site[p] = s;
      contrib = weights[p] * s;
    }
    // wavefront sum in a fixed order
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) contrib += __shfl_xor(contrib, o, 64);
    if (lane == 0) block_out[blockIdx.x] = contrib;
  }
}

// ---------------------------------------------------------------------------
// Reduce-scatter of 16 values over the 64 lanes: afterwards lane l holds the
// wavefront total of element (l >> 2) & 15 (replicated on 4 lanes).
template <typename T>
__device__ inline T butterfly16(T (&v)[16], int lane) {
  T w8[8];
  {
    const bool hi = lane & 32;
#pragma unroll
    for (int j = 0; j < 8; ++j) {
      const T keep = hi ? v[8 + j] : v[j];
      const T give = hi ? v[j] : v[8 + j];
      w8[j] = keep + __shfl_xor(give, 32, 64);
    }
  }
  T w4[4];
  {
    const bool hi = lane & 16;
#pragma unroll
    for (int j = 0; j < 4; ++j) {
      const T keep = hi ? w8[4 + j] : w8[j];
      const T give = hi ? w8[j] : w8[4 + j];
      w4[j] = keep + __shfl_xor(give, 16, 64);
    }
  }
  T w2[2];
  {
    const bool hi = lane & 8;
#pragma unroll
    for (int j = 0; j < 2; ++j) {
      const T keep = hi ? w4[2 + j] : w4[j];
      const T give = hi ? w4[j] : w4[2 + j];
      w2[j] = keep + __shfl_xor(give, 8, 64);
    }
  }
  T w1;
  {
    const bool hi = lane & 4;
    const T keep = hi ? w2[1] : w2[0];
    const T give = hi ? w2[0] : w2[1];
    w1 = keep + __shfl_xor(give, 4, 64);
  }
  w1 += __shfl_xor(w1, 2, 64);
  w1 += __shfl_xor(w1, 1, 64);
  return w1;
}

template <typename T, int C, int R>
__global__ __launch_bounds__(C * 64) void nuc_pre_level_kernel(
    const int32_t* __restrict__ nodes, const int32_t* __restrict__ left, const int32_t* __restrict__ right,
    const T* __restrict__ Pm, const uint8_t* __restrict__ tips, const V4<T>* __restrict__ part,
    V4<T>* __restrict__ pre, const double* __restrict__ pi, const double* __restrict__ cat,
    const T* __restrict__ weights, int root, int N, int P, int n_nodes, double* __restrict__ Gpart) {
  __shared__ T sx[2][C][64];
  __shared__ T sm[2][C][2][64];
  const int c = wave_uniform(threadIdx.x >> 6);
  const int lane = threadIdx.x & 63;
  const int u = nodes[blockIdx.y];
  const int a = left[u], b = right[u];
  const T* Pa = Pm + ((size_t)a * C + c) * 16;
  const T* Pb = Pm + ((size_t)b * C + c) * 16;
  const T wc = T(cat[kMaxCategories + c]);
  V4<T> qroot;
#pragma unroll
  for (int i = 0; i < 4; ++i) qroot.v[i] = T(pi[i]);
  T ga[16], gb[16];
#pragma unroll
  for (int k = 0; k < 16; ++k) {
    ga[k] = 0;
    gb[k] = 0;
  }
  int buf = 0;
  for (int r = 0; r < R; ++r) {
    const int tile = blockIdx.x * R + r;
    if (tile * 64 >= P) break;  // uniform across the block
    const int p = tile * 64 + lane;
    const bool pok = p < P;
    const int pc = pok ? p : P - 1;
    const V4<T> q = (u == root) ? qroot : pre[((size_t)(u - N) * C + c) * P + pc];
    const V4<T> xa = load_child<T>(a, N, c, C, P, pc, tips, part);
    const V4<T> xb = load_child<T>(b, N, c, C, P, pc, tips, part);
    const V4<T> sa = matvec(Pa, xa);
    const V4<T> sb = matvec(Pb, xb);
    T l = 0;
#pragma unroll
    for (int i = 0; i < 4; ++i) l += q.v[i] * sa.v[i] * sb.v[i];
    l *= wc;
    if constexpr (C > 1) {
      sx[buf][c][lane] = l;
      __syncthreads();
      l = 0;
#pragma unroll
      for (int k = 0; k < C; ++k) l += sx[buf][k][lane];
    }
    const T coef = (pok && l > T(0)) ? weights[p] / l : T(0);
    const T f = coef * wc;
    V4<T> ta, tb;
#pragma unroll
    for (int i = 0; i < 4; ++i) {
      ta.v[i] = q.v[i] * sb.v[i];
      tb.v[i] = q.v[i] * sa.v[i];
    }
#pragma unroll
    for (int i = 0; i < 4; ++i) {
      const T fa = f * ta.v[i], fb = f * tb.v[i];
#pragma unroll
      for (int j = 0; j < 4; ++j) {
        ga[4 * i + j] += fa * xa.v[j];
        gb[4 * i + j] += fb * xb.v[j];
      }
    }
    V4<T> qa = matvec_t(Pa, ta);
    V4<T> qb = matvec_t(Pb, tb);
    T ma = max4(qa), mb = max4(qb);
    if constexpr (C > 1) {
      sm[buf][c][0][lane] = ma;
      sm[buf][c][1][lane] = mb;
      __syncthreads();
#pragma unroll
      for (int k = 0; k < C; ++k) {
        ma = sm[buf][k][0][lane] > ma ? sm[buf][k][0][lane] : ma;
        mb = sm[buf][k][1][lane] > mb ? sm[buf][k][1][lane] : mb;
      }
    }
    buf ^= 1;
    const int ea = scale_exponent(ma), eb = scale_exponent(mb);
    if (pok) {
      if (a >= N) {
#pragma unroll
        for (int i = 0; i < 4; ++i) qa.v[i] = scale_by_pow2(qa.v[i], ea);
        pre[((size_t)(a - N) * C + c) * P + p] = qa;
      }
      if (b >= N) {
#pragma unroll
        for (int i = 0; i < 4; ++i) qb.v[i] = scale_by_pow2(qb.v[i], eb);
        pre[((size_t)(b - N) * C + c) * P + p] = qb;
      }
    }
  }
  const T ra = butterfly16(ga, lane);
  const T rb = butterfly16(gb, lane);
  if ((lane & 3) == 0) {
    const int e = (lane >> 2) & 15;
    const size_t nG = (size_t)C * 16;
    Gpart[((size_t)blockIdx.x * n_nodes + a) * nG + c * 16 + e] = (double)ra;
    Gpart[((size_t)blockIdx.x * n_nodes + b) * nG + c * 16 + e] = (double)rb;
  }
}

template <typename T, int C>
int nuc_post_dispatch_c(EpochInstance* in) {
  const auto& pl = in->plan;
  const int tiles = (in->P + 63) / 64;
  const T* Pm = static_cast<const T*>(in->Pm.ptr);
  const uint8_t* tips = static_cast<const uint8_t*>(in->tips.ptr);
  V4<T>* part = static_cast<V4<T>*>(in->partials.ptr);
  int32_t* sc = static_cast<int32_t*>(in->scales.ptr);
  for (int l = 1; l <= pl.n_levels; ++l) {
    const int n_l = pl.level_offset[l + 1] - pl.level_offset[l];
    if (!n_l) continue;
    hipLaunchKernelGGL((nuc_post_level_kernel<T, C>), dim3(tiles, n_l), dim3(C * 64), 0, in->stream,
                       in->d_level_nodes + pl.level_offset[l], in->d_left, in->d_right, Pm, tips, part, sc,
                       in->N, in->P);
  }
  return hip_check(hipGetLastError(), "nuc_post_level launch");
}

template <typename T, int C>
int nuc_root_dispatch_c(EpochInstance* in) {
  const auto& pl = in->plan;
  const int tiles = (in->P + 63) / 64;
  const V4<T>* part = static_cast<const V4<T>*>(in->partials.ptr);
  const int32_t* sc = static_cast<const int32_t*>(in->scales.ptr);
  const size_t slot = pl.root - in->N;
  hipLaunchKernelGGL((nuc_root_kernel<T, C>), dim3(tiles), dim3(C * 64), 0, in->stream,
                     part + slot * C * (size_t)in->P, sc + slot * (size_t)in->P,
                     static_cast<const double*>(in->pi.ptr), static_cast<const double*>(in->cat.ptr),
                     static_cast<const double*>(in->weights.ptr), static_cast<double*>(in->site.ptr),
                     static_cast<double*>(in->blocksum.ptr), in->P);
  return hip_check(hipGetLastError(), "nuc_root launch");
}

template <typename T, int C>
int nuc_pre_dispatch_c(EpochInstance* in, int R) {
  const auto& pl = in->plan;
  const int tiles = (in->P + 63) / 64;
  const int chunks = (tiles + R - 1) / R;
  const T* Pm = static_cast<const T*>(in->Pm.ptr);
  const uint8_t* tips = static_cast<const uint8_t*>(in->tips.ptr);
  const V4<T>* part = static_cast<const V4<T>*>(in->partials.ptr);
  V4<T>* pre = static_cast<V4<T>*>(in->pre.ptr);
  const T* w = static_cast<const T*>(in->weightsT.ptr);
  for (int l = pl.n_levels; l >= 1; --l) {
    const int n_l = pl.level_offset[l + 1] - pl.level_offset[l];
    if (!n_l) continue;
#define EPOCH_NUC_PRE(RR)                                                                                  \
  hipLaunchKernelGGL((nuc_pre_level_kernel<T, C, RR>), dim3(chunks, n_l), dim3(C * 64), 0, in->stream,        \
                     in->d_level_nodes + pl.level_offset[l], in->d_left, in->d_right, Pm, tips, part, pre,      \
                     static_cast<const double*>(in->pi.ptr), static_cast<const double*>(in->cat.ptr), w,       \
                     pl.root, in->N, in->P, in->n_nodes, static_cast<double*>(in->Gpart.ptr))
    switch (R) {
      case 1: EPOCH_NUC_PRE(1); break;
      case 2: EPOCH_NUC_PRE(2); break;
      case 4: EPOCH_NUC_PRE(4); break;
      case 8: EPOCH_NUC_PRE(8); break;
      default: EPOCH_NUC_PRE(16); break;
    }
#undef EPOCH_NUC_PRE
  }
  return hip_check(hipGetLastError(), "nuc_pre_level launch");
}

template <typename T>
int nuc_post_dispatch(EpochInstance* in) {
  switch (in->C) {
    case 1: return nuc_post_dispatch_c<T, 1>(in);
    case 2: return nuc_post_dispatch_c<T, 2>(in);
    case 3: return nuc_post_dispatch_c<T, 3>(in);
    case 4: return nuc_post_dispatch_c<T, 4>(in);
    case 5: return nuc_post_dispatch_c<T, 5>(in);
    case 6: return nuc_post_dispatch_c<T, 6>(in);
    case 7: return nuc_post_dispatch_c<T, 7>(in);
    default: return nuc_post_dispatch_c<T, 8>(in);
  }
}

template <typename T>
int nuc_root_dispatch(EpochInstance* in) {
  switch (in->C) {
    case 1: return nuc_root_dispatch_c<T, 1>(in);
    case 2: return nuc_root_dispatch_c<T, 2>(in);
    case 3: return nuc_root_dispatch_c<T, 3>(in);
    case 4: return nuc_root_dispatch_c<T, 4>(in);
    case 5: return nuc_root_dispatch_c<T, 5>(in);
    case 6: return nuc_root_dispatch_c<T, 6>(in);
    case 7: return nuc_root_dispatch_c<T, 7>(in);
    default: return nuc_root_dispatch_c<T, 8>(in);
  }
}

template <typename T>
int nuc_pre_dispatch(EpochInstance* in, int R) {
  switch (in->C) {
    case 1: return nuc_pre_dispatch_c<T, 1>(in, R);
    case 2: return nuc_pre_dispatch_c<T, 2>(in, R);
    case 3: return nuc_pre_dispatch_c<T, 3>(in, R);
    case 4: return nuc_pre_dispatch_c<T, 4>(in, R);
    case 5: return nuc_pre_dispatch_c<T, 5>(in, R);
    case 6: return nuc_pre_dispatch_c<T, 6>(in, R);
    case 7: return nuc_pre_dispatch_c<T, 7>(in, R);
    default: return nuc_pre_dispatch_c<T, 8>(in, R);
  }
}

}  // namespace

int launch_nuc_post(EpochInstance* in) {
  return in->fp64 ? nuc_post_dispatch<double>(in) : nuc_post_dispatch<float>(in);
}

int launch_nuc_root(EpochInstance* in) {
  int rc = in->fp64 ? nuc_root_dispatch<double>(in) : nuc_root_dispatch<float>(in);
  if (rc) return rc;
  return launch_final_sum(in, (in->P + 63) / 64);
}

int launch_nuc_pre_grad(EpochInstance* in, int R) {
  return in->fp64 ? nuc_pre_dispatch<double>(in, R) : nuc_pre_dispatch<float>(in, R);
}

int nuc_chunks(int P, int R) { return ((P + 63) / 64 + R - 1) / R; }

}  // namespace epochlik
