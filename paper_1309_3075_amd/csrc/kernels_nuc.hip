// Specialised 4-state (nucleotide) kernels, FP32 or FP64.
//
// Layout (shared with the generic kernels): partials and outside vectors
// [slot][c][P][4] with slot = node - N; transition matrices [node][c][4][4]
// row-major; cumulative scale exponents [slot][P].
//
// Lane mapping: lane = (pattern, category) with the CP (power of two >= C)
// categories of a pattern in adjacent lanes, so the per-pattern scale factor
// (shared by all categories) and the category sums are in-group shuffles:
// no LDS and no barriers on the hot path.  Each lane keeps its category's
// two 4x4 matrices in registers for the whole node.  A wavefront walks R
// consecutive tiles of 64/CP patterns and loads tile r+1 while computing
// tile r.
//   nuc_post_level : Felsenstein pruning for one tree level (Eq. 4) with the
//                    cumulative power-of-two scale of every node's subtree.
//   nuc_root       : root sum over pi and categories (text after Eq. 4), FP64.
//   nuc_pre_level  : outside vectors of one level plus the accumulation of
//                    dlogL/dP for the two child branches of each node.
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
struct M4 {
  T m[16];
};

template <typename T>
__device__ inline V4<T> onehot(int st) {
  V4<T> r;
#pragma unroll
  for (int i = 0; i < 4; ++i) r.v[i] = (st >= 4 || st == i) ? T(1) : T(0);
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

// Child vector for one (pattern, category): tip indicator or stored partial.
template <typename T>
__device__ inline V4<T> load_child(int child, int N, int c, int P, int pc, const uint8_t* __restrict__ tips,
                                   const V4<T>* __restrict__ part, int C) {
  if (child < N) return onehot<T>(tips[(size_t)child * P + pc]);
  return part[((size_t)(child - N) * C + c) * P + pc];
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

// Sum of 16 values over the lanes of a wavefront that share a category
// (lanes differing in bits log2(CP)..5), as a reduce-scatter: halving steps
// over lane bits 5, 4, 3, 2 (as far as they are pattern bits), then plain sums
// over the remaining pattern bits.  On return lane l holds the total of element
// (l >> 2) & 15 in out[0] when CP <= 4, and of elements 2 * ((l >> 3) & 7) +
// {0, 1} in out[0..1] when CP == 8.
template <int CP, typename T>
__device__ inline void reduce16(const T (&v)[16], int lane, T (&out)[2]) {
  constexpr int LOG_CP = CP == 1 ? 0 : (CP == 2 ? 1 : (CP == 4 ? 2 : 3));
  constexpr int PB = 6 - LOG_CP;          // pattern bits of the lane index
  constexpr int HALVE = PB < 4 ? PB : 4;  // halving steps
  T buf[16];
#pragma unroll
  for (int k = 0; k < 16; ++k) buf[k] = v[k];
  int n = 16;
#pragma unroll
  for (int s = 0; s < HALVE; ++s) {
    const int bit = 5 - s;  // highest pattern bit first
    const bool hi = (lane >> bit) & 1;
    n >>= 1;
#pragma unroll
    for (int j = 0; j < 8; ++j) {
      if (j < n) {
        const T keep = hi ? buf[n + j] : buf[j];
        const T give = hi ? buf[j] : buf[n + j];
        buf[j] = keep + __shfl_xor(give, 1 << bit, 64);
      }
    }
  }
#pragma unroll
  for (int s = HALVE; s < PB; ++s) {
    const int bit = 5 - s;
    buf[0] += __shfl_xor(buf[0], 1 << bit, 64);
  }
  out[0] = buf[0];
  out[1] = (CP == 8) ? buf[1] : T(0);
}

// Raw per-lane data of one child for one tile: the tip state byte, or the
// stored partial (and its cumulative scale for the post-order pass).  The
// conversion of a tip state to its indicator vector happens at use, so loads
// prefetched for the next tile stay in flight.
template <typename T, bool TIP>
struct ChildBuf;
template <typename T>
struct ChildBuf<T, true> {
  int st;
};
template <typename T>
struct ChildBuf<T, false> {
  V4<T> x;
  int sc;
};

template <typename T, bool TIP, bool SCALE>
__device__ inline void fetch_child(ChildBuf<T, TIP>& cb, int child, int N, int c, int C, int P, int pc,
                                   const uint8_t* __restrict__ tips, const V4<T>* __restrict__ part,
                                   const int32_t* __restrict__ scale_in) {
  if constexpr (TIP) {
    cb.st = tips[(size_t)child * P + pc];
  } else {
    cb.x = part[((size_t)(child - N) * C + c) * P + pc];
    if constexpr (SCALE) cb.sc = scale_in[(size_t)(child - N) * P + pc];
  }
}

template <typename T, bool TIP>
__device__ inline V4<T> child_vec(const ChildBuf<T, TIP>& cb) {
  if constexpr (TIP)
    return onehot<T>(cb.st);
  else
    return cb.x;
}

template <typename T, bool TIP>
__device__ inline int child_scale(const ChildBuf<T, TIP>& cb) {
  if constexpr (TIP)
    return 0;
  else
    return cb.sc;
}

// ---------------------------------------------------------------------------
template <typename T, int CP, bool TA, bool TB>
__device__ inline void post_tiles(int u, int a, int b, int N, int P, int C, int c, int cl, bool cat_ok,
                                  int first, int R, const M4<T>& Pa, const M4<T>& Pb,
                                  const uint8_t* __restrict__ tips, const V4<T>* __restrict__ part_in,
                                  V4<T>* __restrict__ part_out, const int32_t* __restrict__ scale_in,
                                  int32_t* __restrict__ scale_out) {
  constexpr int TPW = 64 / CP;
  const int pbase = first + (int)(threadIdx.x & 63) / CP;
  ChildBuf<T, TA> ca;
  ChildBuf<T, TB> cb;
  {
    const int pc = pbase < P ? pbase : P - 1;
    fetch_child<T, TA, true>(ca, a, N, c, C, P, pc, tips, part_in, scale_in);
    fetch_child<T, TB, true>(cb, b, N, c, C, P, pc, tips, part_in, scale_in);
  }
  for (int r = 0; r < R; ++r) {
    if (first + r * TPW >= P) break;  // uniform
    const int p = pbase + r * TPW;
    ChildBuf<T, TA> na = ca;
    ChildBuf<T, TB> nb = cb;
    if (r + 1 < R) {
      const int pn = p + TPW;
      const int pc = pn < P ? pn : P - 1;
      fetch_child<T, TA, true>(na, a, N, c, C, P, pc, tips, part_in, scale_in);
      fetch_child<T, TB, true>(nb, b, N, c, C, P, pc, tips, part_in, scale_in);
    }
    const V4<T> va = matvec(Pa, child_vec(ca));
    const V4<T> vb = matvec(Pb, child_vec(cb));
    V4<T> x;
#pragma unroll
    for (int i = 0; i < 4; ++i) x.v[i] = va.v[i] * vb.v[i];
    T m = cat_ok ? max4(x) : T(0);
    m = group_max_cp<CP>(m);
    const int e = scale_exponent(m);
#pragma unroll
    for (int i = 0; i < 4; ++i) x.v[i] = scale_by_pow2(x.v[i], e);
    if (p < P && cat_ok) {
      part_out[((size_t)(u - N) * C + c) * P + p] = x;
      if (cl == 0) scale_out[(size_t)(u - N) * P + p] = e + child_scale(ca) + child_scale(cb);
    }
    ca = na;
    cb = nb;
  }
}

template <typename T, int CP>
__global__ __launch_bounds__(256) void nuc_post_level_kernel(
    const int32_t* __restrict__ nodes, const int32_t* __restrict__ left, const int32_t* __restrict__ right,
    const T* __restrict__ Pm, const uint8_t* __restrict__ tips, const V4<T>* __restrict__ part_in,
    V4<T>* __restrict__ part_out, const int32_t* __restrict__ scale_in, int32_t* __restrict__ scale_out,
    int N, int P, int C, int R) {
  constexpr int TPW = 64 / CP;  // patterns per wavefront tile
  const int lane = threadIdx.x & 63;
  const int wave = threadIdx.x >> 6;
  const int cl = lane & (CP - 1);
  const bool cat_ok = cl < C;
  const int c = cat_ok ? cl : 0;
  const int u = nodes[blockIdx.y];
  const int a = left[u], b = right[u];
  const int first = (blockIdx.x * 4 + wave) * R * TPW;  // first pattern of the wavefront
  if (first >= P) return;                                // uniform across the wavefront
  const M4<T> Pa = load_matrix(Pm + ((size_t)a * C + c) * 16);
  const M4<T> Pb = load_matrix(Pm + ((size_t)b * C + c) * 16);
  const bool ta = a < N, tb = b < N;  // uniform
  if (ta && tb)
    post_tiles<T, CP, true, true>(u, a, b, N, P, C, c, cl, cat_ok, first, R, Pa, Pb, tips, part_in, part_out, scale_in, scale_out);
  else if (ta)
    post_tiles<T, CP, true, false>(u, a, b, N, P, C, c, cl, cat_ok, first, R, Pa, Pb, tips, part_in, part_out, scale_in, scale_out);
  else if (tb)
    post_tiles<T, CP, false, true>(u, a, b, N, P, C, c, cl, cat_ok, first, R, Pa, Pb, tips, part_in, part_out, scale_in, scale_out);
  else
    post_tiles<T, CP, false, false>(u, a, b, N, P, C, c, cl, cat_ok, first, R, Pa, Pb, tips, part_in, part_out, scale_in, scale_out);
}

// ---------------------------------------------------------------------------
template <typename T, int CP>
__global__ __launch_bounds__(256) void nuc_root_kernel(
    const V4<T>* __restrict__ rootp, const int32_t* __restrict__ scale_root, const double* __restrict__ pi,
    const double* __restrict__ cat, const double* __restrict__ weights, double* __restrict__ site,
    double* __restrict__ block_out, int P, int C) {
  __shared__ double sm[4];
  constexpr int TPW = 64 / CP;
  const int lane = threadIdx.x & 63;
  const int wave = threadIdx.x >> 6;
  const int cl = lane & (CP - 1);
  const bool cat_ok = cl < C;
  const int c = cat_ok ? cl : 0;
  const int p = (blockIdx.x * 4 + wave) * TPW + lane / CP;
  const int pc = p < P ? p : P - 1;
  const V4<T> x = rootp[(size_t)c * P + pc];
  double l = 0.0;
#pragma unroll
  for (int i = 0; i < 4; ++i) l += pi[i] * (double)x.v[i];
  l = cat_ok ? cat[kMaxCategories + c] * l : 0.0;
  const double L = group_sum_cp<CP>(l);
  double contrib = 0.0;
  if (p < P && cl == 0) {
    const double s = log(L) + (double)scale_root[p] * kLn2;
    site[p] = s;
    contrib = weights[p] * s;
  }
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) contrib += __shfl_xor(contrib, o, 64);
  if (lane == 0) sm[wave] = contrib;
  __syncthreads();
  if (threadIdx.x == 0) block_out[blockIdx.x] = ((sm[0] + sm[1]) + sm[2]) + sm[3];
}

// ---------------------------------------------------------------------------
template <typename T, int CP, bool TA, bool TB, bool ROOT>
__device__ inline void pre_tiles(int u, int a, int b, int N, int P, int C, int c, bool cat_ok, int first,
                                 int R, const M4<T>& Pa, const M4<T>& Pb, T wc, const V4<T>& qroot,
                                 const uint8_t* __restrict__ tips, const V4<T>* __restrict__ part,
                                 const V4<T>* __restrict__ pre_in, V4<T>* __restrict__ pre_out,
                                 const T* __restrict__ weights, T (&ga)[16], T (&gb)[16]) {
  constexpr int TPW = 64 / CP;
  const int pbase = first + (int)(threadIdx.x & 63) / CP;
  ChildBuf<T, TA> ca;
  ChildBuf<T, TB> cb;
  V4<T> q = qroot;
  T w;
  {
    const int pc = pbase < P ? pbase : P - 1;
    if constexpr (!ROOT) q = pre_in[((size_t)(u - N) * C + c) * P + pc];
    fetch_child<T, TA, false>(ca, a, N, c, C, P, pc, tips, part, nullptr);
    fetch_child<T, TB, false>(cb, b, N, c, C, P, pc, tips, part, nullptr);
    w = weights[pc];
  }
  for (int r = 0; r < R; ++r) {
    if (first + r * TPW >= P) break;  // uniform
    const int p = pbase + r * TPW;
    ChildBuf<T, TA> na = ca;
    ChildBuf<T, TB> nb = cb;
    V4<T> nq = q;
    T nw = w;
    if (r + 1 < R) {
      const int pn = p + TPW;
      const int pc = pn < P ? pn : P - 1;
      if constexpr (!ROOT) nq = pre_in[((size_t)(u - N) * C + c) * P + pc];
      fetch_child<T, TA, false>(na, a, N, c, C, P, pc, tips, part, nullptr);
      fetch_child<T, TB, false>(nb, b, N, c, C, P, pc, tips, part, nullptr);
      nw = weights[pc];
    }
    const V4<T> xa = child_vec(ca);
    const V4<T> xb = child_vec(cb);
    const V4<T> sa = matvec(Pa, xa);
    const V4<T> sb = matvec(Pb, xb);
    T l = 0;
#pragma unroll
    for (int i = 0; i < 4; ++i) l += q.v[i] * sa.v[i] * sb.v[i];
    l = group_sum_cp<CP>(l * wc);
    const T wt = (p < P && cat_ok) ? w : T(0);
    const T f = (l > T(0) ? wt / l : T(0)) * wc;
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
    if constexpr (!TA) {
      V4<T> qa = matvec_t(Pa, ta);
      const T ma = group_max_cp<CP>(cat_ok ? max4(qa) : T(0));
      const int ea = scale_exponent(ma);
#pragma unroll
      for (int i = 0; i < 4; ++i) qa.v[i] = scale_by_pow2(qa.v[i], ea);
      if (p < P && cat_ok) pre_out[((size_t)(a - N) * C + c) * P + p] = qa;
    }
    if constexpr (!TB) {
      V4<T> qb = matvec_t(Pb, tb);
      const T mb = group_max_cp<CP>(cat_ok ? max4(qb) : T(0));
      const int eb = scale_exponent(mb);
#pragma unroll
      for (int i = 0; i < 4; ++i) qb.v[i] = scale_by_pow2(qb.v[i], eb);
      if (p < P && cat_ok) pre_out[((size_t)(b - N) * C + c) * P + p] = qb;
    }
    ca = na;
    cb = nb;
    q = nq;
    w = nw;
  }
}

template <typename T, int CP, bool ROOT>
__device__ inline void pre_dispatch_kind(int u, int a, int b, int N, int P, int C, int c, bool cat_ok, int first,
                                         int R, const M4<T>& Pa, const M4<T>& Pb, T wc, const V4<T>& qroot,
                                         const uint8_t* __restrict__ tips, const V4<T>* __restrict__ part,
                                         const V4<T>* __restrict__ pre_in, V4<T>* __restrict__ pre_out,
                                         const T* __restrict__ weights, T (&ga)[16], T (&gb)[16]) {
  const bool ta = a < N, tb = b < N;  // uniform
  if (ta && tb)
    pre_tiles<T, CP, true, true, ROOT>(u, a, b, N, P, C, c, cat_ok, first, R, Pa, Pb, wc, qroot, tips, part, pre_in, pre_out, weights, ga, gb);
  else if (ta)
    pre_tiles<T, CP, true, false, ROOT>(u, a, b, N, P, C, c, cat_ok, first, R, Pa, Pb, wc, qroot, tips, part, pre_in, pre_out, weights, ga, gb);
  else if (tb)
    pre_tiles<T, CP, false, true, ROOT>(u, a, b, N, P, C, c, cat_ok, first, R, Pa, Pb, wc, qroot, tips, part, pre_in, pre_out, weights, ga, gb);
  else
    pre_tiles<T, CP, false, false, ROOT>(u, a, b, N, P, C, c, cat_ok, first, R, Pa, Pb, wc, qroot, tips, part, pre_in, pre_out, weights, ga, gb);
}

template <typename T, int CP>
__global__ __launch_bounds__(256) void nuc_pre_level_kernel(
    const int32_t* __restrict__ nodes, const int32_t* __restrict__ left, const int32_t* __restrict__ right,
    const T* __restrict__ Pm, const uint8_t* __restrict__ tips, const V4<T>* __restrict__ part,
    const V4<T>* __restrict__ pre_in, V4<T>* __restrict__ pre_out, const double* __restrict__ pi,
    const double* __restrict__ cat, const T* __restrict__ weights, int root, int N, int P, int C, int R,
    int n_slots, double* __restrict__ Gpart) {
  constexpr int TPW = 64 / CP;
  __shared__ T sG[4][2][CP][16];
  const int lane = threadIdx.x & 63;
  const int wave = threadIdx.x >> 6;
  const int cl = lane & (CP - 1);
  const bool cat_ok = cl < C;
  const int c = cat_ok ? cl : 0;
  const int u = nodes[blockIdx.y];
  const int a = left[u], b = right[u];
  T ga[16], gb[16];
#pragma unroll
  for (int k = 0; k < 16; ++k) {
    ga[k] = 0;
    gb[k] = 0;
  }
  const int first = (blockIdx.x * 4 + wave) * R * TPW;
  if (first < P) {  // uniform across the wavefront
    const M4<T> Pa = load_matrix(Pm + ((size_t)a * C + c) * 16);
    const M4<T> Pb = load_matrix(Pm + ((size_t)b * C + c) * 16);
    const T wc = cat_ok ? T(cat[kMaxCategories + c]) : T(0);
    V4<T> qroot;
#pragma unroll
    for (int i = 0; i < 4; ++i) qroot.v[i] = T(pi[i]);
    if (u == root)
      pre_dispatch_kind<T, CP, true>(u, a, b, N, P, C, c, cat_ok, first, R, Pa, Pb, wc, qroot, tips, part, pre_in, pre_out, weights, ga, gb);
    else
      pre_dispatch_kind<T, CP, false>(u, a, b, N, P, C, c, cat_ok, first, R, Pa, Pb, wc, qroot, tips, part, pre_in, pre_out, weights, ga, gb);
  }
  // wavefront reduce-scatter, then the four wavefronts of the block in order
  T ra[2], rb[2];
  reduce16<CP>(ga, lane, ra);
  reduce16<CP>(gb, lane, rb);
  if constexpr (CP == 8) {
    const int e0 = 2 * ((lane >> 3) & 7);
    sG[wave][0][cl][e0] = ra[0];
    sG[wave][0][cl][e0 + 1] = ra[1];
    sG[wave][1][cl][e0] = rb[0];
    sG[wave][1][cl][e0 + 1] = rb[1];
  } else {
    // the halving steps run over lane bits 5..2, so lane l holds element
    // (l >> 2) & 15; lane bits below 2 that are pattern bits were summed and
    // replicate it: only the lane with those bits clear stores
    const int e = (lane >> 2) & 15;
    if ((lane & 3 & ~(CP - 1)) == 0) {
      sG[wave][0][cl][e] = ra[0];
      sG[wave][1][cl][e] = rb[0];
    }
  }
  __syncthreads();
  if (threadIdx.x < 2 * CP * 16) {
    const int side = threadIdx.x / (CP * 16);
    const int rem = threadIdx.x % (CP * 16);
    const int cc = rem / 16, e = rem % 16;
    if (cc < C) {
      const T s = ((sG[0][side][cc][e] + sG[1][side][cc][e]) + sG[2][side][cc][e]) + sG[3][side][cc][e];
      const int v = side == 0 ? a : b;
      Gpart[((size_t)v * n_slots + blockIdx.x) * ((size_t)C * 16) + cc * 16 + e] = (double)s;
    }
  }
}

int cp_of(int C) { return C <= 1 ? 1 : (C <= 2 ? 2 : (C <= 4 ? 4 : 8)); }

// tiles per wavefront for a level with n_l nodes: enough wavefronts to fill the chip
int tiles_per_wave(int tiles, int n_l, int r_min, int r_max) {
  const long target_waves = 8192;
  const long waves_per_node = (target_waves + n_l - 1) / n_l;
  long R = (tiles + waves_per_node - 1) / waves_per_node;
  if (R < r_min) R = r_min;
  if (R > r_max) R = r_max;
  return (int)R;
}

template <typename T, int CP>
int post_dispatch_cp(EpochInstance* in) {
  const auto& pl = in->plan;
  constexpr int TPW = 64 / CP;
  const int tiles = (in->P + TPW - 1) / TPW;
  const T* Pm = static_cast<const T*>(in->Pm.ptr);
  const uint8_t* tips = static_cast<const uint8_t*>(in->tips.ptr);
  V4<T>* part = static_cast<V4<T>*>(in->partials.ptr);
  int32_t* sc = static_cast<int32_t*>(in->scales.ptr);
  for (int l = 1; l <= pl.n_levels; ++l) {
    const int n_l = pl.level_offset[l + 1] - pl.level_offset[l];
    if (!n_l) continue;
    const int R = tiles_per_wave(tiles, n_l, 1, 16);
    const int blocks = (tiles + 4 * R - 1) / (4 * R);
    hipLaunchKernelGGL((nuc_post_level_kernel<T, CP>), dim3(blocks, n_l), dim3(256), 0, in->stream,
                       in->d_level_nodes + pl.level_offset[l], in->d_left, in->d_right, Pm, tips, part, part,
                       sc, sc, in->N, in->P, in->C, R);
  }
  return hip_check(hipGetLastError(), "nuc_post_level launch");
}

template <typename T, int CP>
int root_dispatch_cp(EpochInstance* in) {
  const auto& pl = in->plan;
  constexpr int TPW = 64 / CP;
  const int blocks = (in->P + 4 * TPW - 1) / (4 * TPW);
  const V4<T>* part = static_cast<const V4<T>*>(in->partials.ptr);
  const int32_t* sc = static_cast<const int32_t*>(in->scales.ptr);
  const size_t slot = pl.root - in->N;
  hipLaunchKernelGGL((nuc_root_kernel<T, CP>), dim3(blocks), dim3(256), 0, in->stream,
                     part + slot * in->C * (size_t)in->P, sc + slot * (size_t)in->P,
                     static_cast<const double*>(in->pi.ptr), static_cast<const double*>(in->cat.ptr),
                     static_cast<const double*>(in->weights.ptr), static_cast<double*>(in->site.ptr),
                     static_cast<double*>(in->blocksum.ptr), in->P, in->C);
  int rc = hip_check(hipGetLastError(), "nuc_root launch");
  if (rc) return rc;
  return launch_final_sum(in, blocks);
}

int pre_blocks(const EpochInstance* in, int n_l) {
  const int TPW = 64 / cp_of(in->C);
  const int tiles = (in->P + TPW - 1) / TPW;
  const int R = tiles_per_wave(tiles, n_l, in->nuc_rmin, 64);
  return (tiles + 4 * R - 1) / (4 * R);
}

template <typename T, int CP>
int pre_dispatch_cp(EpochInstance* in) {
  const auto& pl = in->plan;
  constexpr int TPW = 64 / CP;
  const int tiles = (in->P + TPW - 1) / TPW;
  const T* Pm = static_cast<const T*>(in->Pm.ptr);
  const uint8_t* tips = static_cast<const uint8_t*>(in->tips.ptr);
  const V4<T>* part = static_cast<const V4<T>*>(in->partials.ptr);
  V4<T>* pre = static_cast<V4<T>*>(in->pre.ptr);
  const T* w = static_cast<const T*>(in->weightsT.ptr);
  for (int l = pl.n_levels; l >= 1; --l) {
    const int n_l = pl.level_offset[l + 1] - pl.level_offset[l];
    if (!n_l) continue;
    const int R = tiles_per_wave(tiles, n_l, in->nuc_rmin, 64);
    const int blocks = pre_blocks(in, n_l);
    hipLaunchKernelGGL((nuc_pre_level_kernel<T, CP>), dim3(blocks, n_l), dim3(256), 0, in->stream,
                       in->d_level_nodes + pl.level_offset[l], in->d_left, in->d_right, Pm, tips, part, pre, pre,
                       static_cast<const double*>(in->pi.ptr), static_cast<const double*>(in->cat.ptr), w,
                       pl.root, in->N, in->P, in->C, R, in->nuc_slots, static_cast<double*>(in->Gpart.ptr));
  }
  return hip_check(hipGetLastError(), "nuc_pre_level launch");
}

}  // namespace

// Partial-sum slots per branch of the 4-state gradient: the block count of a
// level launched with the smallest tile count per wavefront.
int nuc_slots(int P, int C, int rmin) {
  const int TPW = 64 / cp_of(C);
  const int tiles = (P + TPW - 1) / TPW;
  return (tiles + 4 * rmin - 1) / (4 * rmin);
}

// Number of partial-sum slots each branch receives from the gradient pass
// (the block count of its parent's level), host [n_nodes].
void nuc_slots_per_node(const EpochInstance* in, std::vector<int32_t>& out) {
  const auto& pl = in->plan;
  out.assign(in->n_nodes, 0);
  for (int l = 1; l <= pl.n_levels; ++l) {
    const int n_l = pl.level_offset[l + 1] - pl.level_offset[l];
    if (!n_l) continue;
    const int blocks = pre_blocks(in, n_l);
    for (int k = pl.level_offset[l]; k < pl.level_offset[l + 1]; ++k) {
      const int u = pl.level_nodes[k];
      out[pl.left[u]] = blocks;
      out[pl.right[u]] = blocks;
    }
  }
}

int launch_nuc_post(EpochInstance* in) {
  switch (cp_of(in->C)) {
    case 1: return in->fp64 ? post_dispatch_cp<double, 1>(in) : post_dispatch_cp<float, 1>(in);
    case 2: return in->fp64 ? post_dispatch_cp<double, 2>(in) : post_dispatch_cp<float, 2>(in);
    case 4: return in->fp64 ? post_dispatch_cp<double, 4>(in) : post_dispatch_cp<float, 4>(in);
    default: return in->fp64 ? post_dispatch_cp<double, 8>(in) : post_dispatch_cp<float, 8>(in);
  }
}

int launch_nuc_root(EpochInstance* in) {
  switch (cp_of(in->C)) {
    case 1: return in->fp64 ? root_dispatch_cp<double, 1>(in) : root_dispatch_cp<float, 1>(in);
    case 2: return in->fp64 ? root_dispatch_cp<double, 2>(in) : root_dispatch_cp<float, 2>(in);
    case 4: return in->fp64 ? root_dispatch_cp<double, 4>(in) : root_dispatch_cp<float, 4>(in);
    default: return in->fp64 ? root_dispatch_cp<double, 8>(in) : root_dispatch_cp<float, 8>(in);
  }
}

int launch_nuc_pre_grad(EpochInstance* in) {
  switch (cp_of(in->C)) {
    case 1: return in->fp64 ? pre_dispatch_cp<double, 1>(in) : pre_dispatch_cp<float, 1>(in);
    case 2: return in->fp64 ? pre_dispatch_cp<double, 2>(in) : pre_dispatch_cp<float, 2>(in);
    case 4: return in->fp64 ? pre_dispatch_cp<double, 4>(in) : pre_dispatch_cp<float, 4>(in);
    default: return in->fp64 ? pre_dispatch_cp<double, 8>(in) : pre_dispatch_cp<float, 8>(in);
  }
}

}  // namespace epochlik
