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
#include "nuc_common.h"

namespace epochlik {

namespace {
using namespace nuc;

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

// Child kinds: a tip (state byte), an internal node whose partial is stored, or
// a cherry (an internal node whose two children are tips).  Cherries are never
// stored: their partial is the product of two tip lookups, recomputed by the
// parent in both passes from the cherry's tip states and transposed tip
// matrices staged in LDS (row 4 holds the row sums used for missing data).
enum ChildKind { kTip = 0, kInternal = 1, kCherry = 2 };

template <typename T, int KIND>
struct ChildBuf;
template <typename T>
struct ChildBuf<T, kTip> {
  int st;
};
template <typename T>
struct ChildBuf<T, kInternal> {
  V4<T> x;
  int sc;
};
template <typename T>
struct ChildBuf<T, kCherry> {
  int st1, st2;
};

template <typename T>
struct NucCtx {
  int N, P, C, c, cl;
  bool cat_ok;
  const uint8_t* __restrict__ tips;
  const V4<T>* __restrict__ part;
  const int32_t* __restrict__ scale_in;
  const int32_t* __restrict__ left;
  const int32_t* __restrict__ right;
  const V4<T>* sTip;  // LDS [4 slots][8 categories][5 rows]
};

template <typename T, int KIND, bool SCALE>
__device__ inline void fetch_child(ChildBuf<T, KIND>& cb, const NucCtx<T>& x, int child, int pc) {
  if constexpr (KIND == kTip) {
    cb.st = x.tips[(size_t)child * x.P + pc];
  } else if constexpr (KIND == kInternal) {
    cb.x = x.part[((size_t)(child - x.N) * x.C + x.c) * x.P + pc];
    if constexpr (SCALE) cb.sc = x.scale_in[(size_t)(child - x.N) * x.P + pc];
  } else {
    cb.st1 = x.tips[(size_t)x.left[child] * x.P + pc];
    cb.st2 = x.tips[(size_t)x.right[child] * x.P + pc];
  }
}

// Child vector; for a cherry the raw product of its two tip lookups (slots s0, s0+1).
template <typename T, int KIND>
__device__ inline V4<T> child_vec(const ChildBuf<T, KIND>& cb, const NucCtx<T>& x, int s0) {
  if constexpr (KIND == kTip) {
    return onehot<T>(cb.st);
  } else if constexpr (KIND == kInternal) {
    return cb.x;
  } else {
    const V4<T> u = x.sTip[(s0 * 8 + x.c) * 16 + cb.st1];
    const V4<T> w = x.sTip[((s0 + 1) * 8 + x.c) * 16 + cb.st2];
    V4<T> r;
#pragma unroll
    for (int i = 0; i < 4; ++i) r.v[i] = u.v[i] * w.v[i];
    return r;
  }
}

// Post-order only: a cherry's partial is rescaled exactly like a stored one
// (power of two shared by the categories of the pattern); returns its exponent.
template <int CP, typename T, int KIND>
__device__ inline int child_normalise(V4<T>& v, const ChildBuf<T, KIND>& cb, bool cat_ok) {
  if constexpr (KIND == kTip) {
    return 0;
  } else if constexpr (KIND == kInternal) {
    return cb.sc;
  } else {
    const T m = group_max_cp<CP>(cat_ok ? max4(v) : T(0));
    const int e = scale_exponent(m);
#pragma unroll
    for (int i = 0; i < 4; ++i) v.v[i] = scale_by_pow2(v.v[i], e);
    return e;
  }
}

// Stage the tip lookups of cherry children: for every state set j (1..15),
// column j = sum over the states in j of column P[:, state], so a tip lookup is
// one LDS read for an observed, ambiguous or missing state alike.  Slots 0-1
// for child a, 2-3 for child b.  Called by every thread of the block before a
// barrier.
template <typename T>
__device__ inline void stage_cherry_tips(V4<T>* sTip, const T* __restrict__ Pm, const int32_t* __restrict__ left,
                                         const int32_t* __restrict__ right, int N, int C, int a, int b, bool ca,
                                         bool cb) {
  for (int t = threadIdx.x; t < 4 * C * 16; t += blockDim.x) {
    const int slot = t / (C * 16), c = (t / 16) % C, j = t % 16;
    const int owner = slot < 2 ? a : b;
    if (!(slot < 2 ? ca : cb)) continue;
    const int tip = (slot & 1) ? right[owner] : left[owner];
    const T* M = Pm + ((size_t)tip * C + c) * 16;
    V4<T> col;
#pragma unroll
    for (int i = 0; i < 4; ++i) {
      const T m0 = (j & 1) ? M[4 * i] : T(0), m1 = (j & 2) ? M[4 * i + 1] : T(0);
      const T m2 = (j & 4) ? M[4 * i + 2] : T(0), m3 = (j & 8) ? M[4 * i + 3] : T(0);
      col.v[i] = (m0 + m1) + (m2 + m3);
    }
    sTip[(slot * 8 + c) * 16 + j] = col;
  }
}

template <typename T>
__device__ inline int kind_of(int v, int N, const int32_t* __restrict__ left, const int32_t* __restrict__ right) {
  if (v < N) return kTip;
  return (left[v] < N && right[v] < N) ? kCherry : kInternal;
}

// ---------------------------------------------------------------------------
template <typename T, int CP, int KA, int KB>
__device__ inline void post_tiles(const NucCtx<T>& x, int u, int a, int b, int first, int R, const M4<T>& Pa,
                                  const M4<T>& Pb, V4<T>* __restrict__ part_out, int32_t* __restrict__ scale_out) {
  constexpr int TPW = 64 / CP;
  const int N = x.N, P = x.P, C = x.C, c = x.c;
  const int pbase = first + (int)(threadIdx.x & 63) / CP;
  ChildBuf<T, KA> ca;
  ChildBuf<T, KB> cb;
  {
    const int pc = pbase < P ? pbase : P - 1;
    fetch_child<T, KA, true>(ca, x, a, pc);
    fetch_child<T, KB, true>(cb, x, b, pc);
  }
  for (int r = 0; r < R; ++r) {
    if (first + r * TPW >= P) break;  // uniform
    const int p = pbase + r * TPW;
    ChildBuf<T, KA> na = ca;
    ChildBuf<T, KB> nb = cb;
    if (r + 1 < R) {
      const int pn = p + TPW;
      const int pc = pn < P ? pn : P - 1;
      fetch_child<T, KA, true>(na, x, a, pc);
      fetch_child<T, KB, true>(nb, x, b, pc);
    }
    V4<T> xa = child_vec<T, KA>(ca, x, 0);
    V4<T> xb = child_vec<T, KB>(cb, x, 2);
    const int sa = child_normalise<CP, T, KA>(xa, ca, x.cat_ok);
    const int sb = child_normalise<CP, T, KB>(xb, cb, x.cat_ok);
    const V4<T> va = matvec(Pa, xa);
    const V4<T> vb = matvec(Pb, xb);
    V4<T> y;
#pragma unroll
    for (int i = 0; i < 4; ++i) y.v[i] = va.v[i] * vb.v[i];
    T m = x.cat_ok ? max4(y) : T(0);
    m = group_max_cp<CP>(m);
    const int e = scale_exponent(m);
#pragma unroll
    for (int i = 0; i < 4; ++i) y.v[i] = scale_by_pow2(y.v[i], e);
    if (p < P && x.cat_ok) {
      store_streaming(&part_out[((size_t)(u - N) * C + c) * P + p], y);
      if (x.cl == 0) scale_out[(size_t)(u - N) * P + p] = e + sa + sb;
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
  __shared__ V4<T> sTip[4 * 8 * 16];
  const int lane = threadIdx.x & 63;
  const int wave = threadIdx.x >> 6;
  const int cl = lane & (CP - 1);
  const bool cat_ok = cl < C;
  const int c = cat_ok ? cl : 0;
  const int u = nodes[blockIdx.y];
  int a = left[u], b = right[u];
  int ka = kind_of<T>(a, N, left, right), kb = kind_of<T>(b, N, left, right);
  if (ka > kb) {  // canonical order: the smaller kind first (the product is symmetric)
    const int t = a; a = b; b = t;
    const int k = ka; ka = kb; kb = k;
  }
  stage_cherry_tips<T>(sTip, Pm, left, right, N, C, a, b, ka == kCherry, kb == kCherry);
  __syncthreads();
  const int first = (blockIdx.x * 4 + wave) * R * TPW;  // first pattern of the wavefront
  if (first >= P) return;                                // uniform across the wavefront (after the barrier)
  const M4<T> Pa = load_matrix(Pm + ((size_t)a * C + c) * 16);
  const M4<T> Pb = load_matrix(Pm + ((size_t)b * C + c) * 16);
  const NucCtx<T> x{N, P, C, c, cl, cat_ok, tips, part_in, scale_in, left, right, sTip};
#define EPOCH_POST_CASE(A, B) \
  if (ka == A && kb == B) return post_tiles<T, CP, A, B>(x, u, a, b, first, R, Pa, Pb, part_out, scale_out)
  EPOCH_POST_CASE(kTip, kTip);
  EPOCH_POST_CASE(kTip, kInternal);
  EPOCH_POST_CASE(kTip, kCherry);
  EPOCH_POST_CASE(kInternal, kInternal);
  EPOCH_POST_CASE(kInternal, kCherry);
  EPOCH_POST_CASE(kCherry, kCherry);
#undef EPOCH_POST_CASE
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
// Outer product of a cherry's tip branches.  At the cherry's parent the cherry's
// outside vector q_c = P_c^T t_c is already in registers (unscaled: it shares the
// scale of t_c and of the pattern likelihood l behind f), so the dlogL/dP of the
// cherry's two tip branches is formed there, and q_c is never stored: its tip
// children get f (q_c o S_other) (x) onehot(state).
template <typename T>
__device__ inline void cherry_tip_grads(const V4<T>& qc, const V4<T>& s1, const V4<T>& s2, int st1, int st2, T f,
                                        T (&g1)[16], T (&g2)[16]) {
  const V4<T> o1 = onehot<T>(st1), o2 = onehot<T>(st2);
#pragma unroll
  for (int i = 0; i < 4; ++i) {
    const T f1 = f * qc.v[i] * s2.v[i], f2 = f * qc.v[i] * s1.v[i];
#pragma unroll
    for (int j = 0; j < 4; ++j) {
      g1[4 * i + j] += f1 * o1.v[j];
      g2[4 * i + j] += f2 * o2.v[j];
    }
  }
}

// NX: cherry children of the node (0, 1 = the second child after the canonical
// order, 2 = both); gx holds their tip branches' accumulators, 2 per cherry.
template <typename T, int CP, int KA, int KB, bool ROOT, int NX>
__device__ inline void pre_tiles(const NucCtx<T>& x, int u, int a, int b, int first, int R, const M4<T>& Pa,
                                 const M4<T>& Pb, T wc, const V4<T>& qroot, const V4<T>* __restrict__ pre_in,
                                 V4<T>* __restrict__ pre_out, const T* __restrict__ weights, T (&ga)[16],
                                 T (&gb)[16], T (&gx)[2 * NX + (NX == 0)][16]) {
  constexpr int TPW = 64 / CP;
  const int N = x.N, P = x.P, C = x.C, c = x.c;
  const bool cat_ok = x.cat_ok;
  const int pbase = first + (int)(threadIdx.x & 63) / CP;
  ChildBuf<T, KA> ca;
  ChildBuf<T, KB> cb;
  V4<T> q = qroot;
  T w;
  {
    const int pc = pbase < P ? pbase : P - 1;
    if constexpr (!ROOT) q = pre_in[((size_t)(u - N) * C + c) * P + pc];
    fetch_child<T, KA, false>(ca, x, a, pc);
    fetch_child<T, KB, false>(cb, x, b, pc);
    w = weights[pc];
  }
  for (int r = 0; r < R; ++r) {
    if (first + r * TPW >= P) break;  // uniform
    const int p = pbase + r * TPW;
    ChildBuf<T, KA> na = ca;
    ChildBuf<T, KB> nb = cb;
    V4<T> nq = q;
    T nw = w;
    if (r + 1 < R) {
      const int pn = p + TPW;
      const int pc = pn < P ? pn : P - 1;
      if constexpr (!ROOT) nq = pre_in[((size_t)(u - N) * C + c) * P + pc];
      fetch_child<T, KA, false>(na, x, a, pc);
      fetch_child<T, KB, false>(nb, x, b, pc);
      nw = weights[pc];
    }
    // a cherry's recomputed partial is left unscaled: its scale cancels in the ratios
    const V4<T> xa = child_vec<T, KA>(ca, x, 0);
    const V4<T> xb = child_vec<T, KB>(cb, x, 2);
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
    if constexpr (NX == 2 && KA == kCherry) {
      const V4<T> qa = matvec_t(Pa, ta);
      cherry_tip_grads<T>(qa, x.sTip[(0 * 8 + c) * 16 + ca.st1], x.sTip[(1 * 8 + c) * 16 + ca.st2], ca.st1, ca.st2,
                          f, gx[0], gx[1]);
    } else if constexpr (KA != kTip) {
      V4<T> qa = matvec_t(Pa, ta);
      const T ma = group_max_cp<CP>(cat_ok ? max4(qa) : T(0));
      const int ea = scale_exponent(ma);
#pragma unroll
      for (int i = 0; i < 4; ++i) qa.v[i] = scale_by_pow2(qa.v[i], ea);
      if (p < P && cat_ok) store_streaming(&pre_out[((size_t)(a - N) * C + c) * P + p], qa);
    }
    if constexpr (NX >= 1 && KB == kCherry) {
      constexpr int h = NX == 2 ? 2 : 0;
      const V4<T> qb = matvec_t(Pb, tb);
      cherry_tip_grads<T>(qb, x.sTip[(2 * 8 + c) * 16 + cb.st1], x.sTip[(3 * 8 + c) * 16 + cb.st2], cb.st1, cb.st2,
                          f, gx[h], gx[h + 1]);
    } else if constexpr (KB != kTip) {
      V4<T> qb = matvec_t(Pb, tb);
      const T mb = group_max_cp<CP>(cat_ok ? max4(qb) : T(0));
      const int eb = scale_exponent(mb);
#pragma unroll
      for (int i = 0; i < 4; ++i) qb.v[i] = scale_by_pow2(qb.v[i], eb);
      if (p < P && cat_ok) store_streaming(&pre_out[((size_t)(b - N) * C + c) * P + p], qb);
    }
    ca = na;
    cb = nb;
    q = nq;
    w = nw;
  }
}

template <typename T, int CP, bool ROOT, int NX>
__device__ inline void pre_dispatch_kind(const NucCtx<T>& x, int ka, int kb, int u, int a, int b, int first, int R,
                                         const M4<T>& Pa, const M4<T>& Pb, T wc, const V4<T>& qroot,
                                         const V4<T>* __restrict__ pre_in, V4<T>* __restrict__ pre_out,
                                         const T* __restrict__ weights, T (&ga)[16], T (&gb)[16],
                                         T (&gx)[2 * NX + (NX == 0)][16]) {
#define EPOCH_PRE_CASE(A, B)                                                                                  \
  if (ka == A && kb == B)                                                                                     \
    return pre_tiles<T, CP, A, B, ROOT, NX>(x, u, a, b, first, R, Pa, Pb, wc, qroot, pre_in, pre_out, weights, \
                                            ga, gb, gx)
  if constexpr (NX == 2) {
    EPOCH_PRE_CASE(kCherry, kCherry);
  } else if constexpr (NX == 1) {
    EPOCH_PRE_CASE(kTip, kCherry);
    EPOCH_PRE_CASE(kInternal, kCherry);
  } else {
    EPOCH_PRE_CASE(kTip, kTip);
    EPOCH_PRE_CASE(kTip, kInternal);
    EPOCH_PRE_CASE(kInternal, kInternal);
  }
#undef EPOCH_PRE_CASE
}

// NX: every node of the launch has exactly NX cherry children, whose tip
// branches' dlogL/dP is formed here (see cherry_tip_grads).
template <typename T, int CP, int NX>
__global__ __launch_bounds__(256) void nuc_pre_level_kernel(
    const int32_t* __restrict__ nodes, const int32_t* __restrict__ left, const int32_t* __restrict__ right,
    const T* __restrict__ Pm, const uint8_t* __restrict__ tips, const V4<T>* __restrict__ part,
    const V4<T>* __restrict__ pre_in, V4<T>* __restrict__ pre_out, const double* __restrict__ pi,
    const double* __restrict__ cat, const T* __restrict__ weights, int root, int N, int P, int C, int R,
    int n_slots, double* __restrict__ Gpart) {
  constexpr int TPW = 64 / CP;
  constexpr int NG = 2 + 2 * NX;  // branches receiving dlogL/dP from this block
  __shared__ T sG[4][NG][CP][16];
  __shared__ V4<T> sTip[4 * 8 * 16];
  const int lane = threadIdx.x & 63;
  const int wave = threadIdx.x >> 6;
  const int cl = lane & (CP - 1);
  const bool cat_ok = cl < C;
  const int c = cat_ok ? cl : 0;
  const int u = nodes[blockIdx.y];
  int a = left[u], b = right[u];
  int ka = kind_of<T>(a, N, left, right), kb = kind_of<T>(b, N, left, right);
  if (ka > kb) {  // canonical order; each child's gradient still goes to its own branch
    const int t = a; a = b; b = t;
    const int k = ka; ka = kb; kb = k;
  }
  stage_cherry_tips<T>(sTip, Pm, left, right, N, C, a, b, ka == kCherry, kb == kCherry);
  __syncthreads();
  T ga[16], gb[16];
  T gx[2 * NX + (NX == 0)][16];
#pragma unroll
  for (int k = 0; k < 16; ++k) {
    ga[k] = 0;
    gb[k] = 0;
#pragma unroll
    for (int h = 0; h < 2 * NX + (NX == 0); ++h) gx[h][k] = 0;
  }
  const int first = (blockIdx.x * 4 + wave) * R * TPW;
  if (first < P) {  // uniform across the wavefront
    const M4<T> Pa = load_matrix(Pm + ((size_t)a * C + c) * 16);
    const M4<T> Pb = load_matrix(Pm + ((size_t)b * C + c) * 16);
    const T wc = cat_ok ? T(cat[kMaxCategories + c]) : T(0);
    V4<T> qroot;
#pragma unroll
    for (int i = 0; i < 4; ++i) qroot.v[i] = T(pi[i]);
    const NucCtx<T> x{N, P, C, c, cl, cat_ok, tips, part, nullptr, left, right, sTip};
    if (u == root)
      pre_dispatch_kind<T, CP, true, NX>(x, ka, kb, u, a, b, first, R, Pa, Pb, wc, qroot, pre_in, pre_out, weights,
                                         ga, gb, gx);
    else
      pre_dispatch_kind<T, CP, false, NX>(x, ka, kb, u, a, b, first, R, Pa, Pb, wc, qroot, pre_in, pre_out, weights,
                                          ga, gb, gx);
  }
  // wavefront reduce-scatter, then the four wavefronts of the block in order
  auto scatter = [&](T (&g)[16], int side) {
    T rg[2];
    reduce16<CP>(g, lane, rg);
    if constexpr (CP == 8) {
      const int e0 = 2 * ((lane >> 3) & 7);
      sG[wave][side][cl][e0] = rg[0];
      sG[wave][side][cl][e0 + 1] = rg[1];
    } else {
      // the halving steps run over lane bits 5..2, so lane l holds element
      // (l >> 2) & 15; lane bits below 2 that are pattern bits were summed and
      // replicate it: only the lane with those bits clear stores
      const int e = (lane >> 2) & 15;
      if ((lane & 3 & ~(CP - 1)) == 0) sG[wave][side][cl][e] = rg[0];
    }
  };
  scatter(ga, 0);
  scatter(gb, 1);
#pragma unroll
  for (int h = 0; h < 2 * NX; ++h) scatter(gx[h], 2 + h);
  __syncthreads();
  for (int t = threadIdx.x; t < NG * CP * 16; t += 256) {
    const int side = t / (CP * 16);
    const int rem = t % (CP * 16);
    const int cc = rem / 16, e = rem % 16;
    int v = side == 0 ? a : b;
    if (side >= 2) {  // tip children of the cherry children (b's when NX == 1)
      const int owner = (NX == 2 && side < 4) ? a : b;
      v = (side & 1) ? right[owner] : left[owner];
    }
    if (cc < C) {
      const T s = ((sG[0][side][cc][e] + sG[1][side][cc][e]) + sG[2][side][cc][e]) + sG[3][side][cc][e];
      Gpart[((size_t)v * n_slots + blockIdx.x) * ((size_t)C * 16) + cc * 16 + e] = (double)s;
    }
  }
}

int cp_of(int C) { return C <= 1 ? 1 : (C <= 2 ? 2 : (C <= 4 ? 4 : 8)); }

// Wavefronts per level launch that the tile count per wavefront aims for.  C2
// in FP32: 348.6 evals/s with 8,192 for both passes, 355.9 with 32,768 for the
// post-order and 16,384 for the pre-order launches; in FP64 (twice the bytes
// per tile) those gave 165 evals/s against 171 with 8,192.
constexpr long post_target_waves(bool fp64) { return fp64 ? 8192 : 32768; }
constexpr long pre_target_waves(bool fp64) { return fp64 ? 8192 : 16384; }

// tiles per wavefront for a launch over n_l nodes: about target_waves wavefronts
int tiles_per_wave(int tiles, int n_l, int r_min, int r_max, long target_waves) {
  const long waves_per_node = (target_waves + n_l - 1) / n_l;
  long R = (tiles + waves_per_node - 1) / waves_per_node;
  if (R < r_min) R = r_min;
  if (R > r_max) R = r_max;
  return (int)R;
}

template <typename T, int CP>
int post_dispatch_cp(EpochInstance* in, const int32_t* d_nodes, const int32_t* level_off) {
  const auto& pl = in->plan;
  constexpr int TPW = 64 / CP;
  const int tiles = (in->P + TPW - 1) / TPW;
  const T* Pm = static_cast<const T*>(in->Pm.ptr);
  const uint8_t* tips = static_cast<const uint8_t*>(in->tips.ptr);
  V4<T>* part = static_cast<V4<T>*>(in->partials.ptr);
  int32_t* sc = static_cast<int32_t*>(in->scales.ptr);
  // level 1 holds exactly the cherries, which are recomputed by their parents;
  // it is launched only when the root itself is a cherry (two tips)
  for (int l = (pl.n_levels == 1 ? 1 : 2); l <= pl.n_levels; ++l) {
    const int n_l = level_off[l + 1] - level_off[l];
    if (!n_l) continue;
    const int R = tiles_per_wave(tiles, n_l, 1, 16, post_target_waves(sizeof(T) == 8));
    const int blocks = (tiles + 4 * R - 1) / (4 * R);
    hipLaunchKernelGGL((nuc_post_level_kernel<T, CP>), dim3(blocks, n_l), dim3(256), 0, in->stream,
                       d_nodes + level_off[l], in->d_left, in->d_right, Pm, tips, part, part,
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
  const size_t slot = in->root_slot;  // pl.root - N, or its compact slot under an HBM budget
  (void)pl;
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
  const int R = tiles_per_wave(tiles, n_l, in->nuc_rmin, 64, pre_target_waves(in->fp64));
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
  const int32_t* nodes = static_cast<const int32_t*>(in->nuc_nodes.ptr);
  // level 1 holds exactly the cherries, whose tip branches are handled by their
  // parents; it is launched only when the root itself is a cherry
  const int lowest = pl.n_levels == 1 ? 1 : 2;
  for (int l = pl.n_levels; l >= lowest; --l) {
    const int n_l = pl.level_offset[l + 1] - pl.level_offset[l];
    if (!n_l) continue;
    // nodes with two cherry children first, then one, then none; each group's
    // launch picks its own tiles per wavefront for its node count
    const int n2 = in->nuc_fuse[2 * l], n1 = in->nuc_fuse[2 * l + 1];
    const int32_t* lv = nodes + pl.level_offset[l];
#define EPOCH_PRE_LAUNCH(NXV, first_node, count)                                                              \
  if ((count) > 0)                                                                                           \
    hipLaunchKernelGGL((nuc_pre_level_kernel<T, CP, NXV>), dim3(pre_blocks(in, (count)), (count)), dim3(256), 0, \
                       in->stream, lv + (first_node), in->d_left, in->d_right, Pm, tips, part, pre, pre,      \
                       static_cast<const double*>(in->pi.ptr), static_cast<const double*>(in->cat.ptr), w,   \
                       pl.root, in->N, in->P, in->C, tiles_per_wave(tiles, (count), in->nuc_rmin, 64, pre_target_waves(sizeof(T) == 8)), \
                       in->nuc_slots, static_cast<double*>(in->Gpart.ptr))
    EPOCH_PRE_LAUNCH(2, 0, n2);
    EPOCH_PRE_LAUNCH(1, n2, n1);
    EPOCH_PRE_LAUNCH(0, n2 + n1, n_l - n2 - n1);
#undef EPOCH_PRE_LAUNCH
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

// Number of partial-sum slots each branch receives from the gradient pass, host
// [n_nodes]: the block count of the launch that forms its dlogL/dP (its parent's
// group within its level, or its grandparent's for the tip children of a
// cherry).  nodes / fuse: the pre-order launch order (nuc_pre_order_nodes).
void nuc_slots_per_node(const EpochInstance* in, const std::vector<int32_t>& nodes, const std::vector<int>& fuse,
                        std::vector<int32_t>& out) {
  const auto& pl = in->plan;
  const int N = in->N;
  out.assign(in->n_nodes, 0);
  const int lowest = pl.n_levels == 1 ? 1 : 2;
  for (int l = lowest; l <= pl.n_levels; ++l) {
    const int n_l = pl.level_offset[l + 1] - pl.level_offset[l];
    if (!n_l) continue;
    const int n2 = fuse[2 * l], n1 = fuse[2 * l + 1];
    for (int k = pl.level_offset[l]; k < pl.level_offset[l + 1]; ++k) {
      const int u = nodes[k];
      const int r = k - pl.level_offset[l];
      const int blocks = pre_blocks(in, r < n2 ? n2 : (r < n2 + n1 ? n1 : n_l - n2 - n1));
      for (int child : {pl.left[u], pl.right[u]}) {
        out[child] = blocks;
        if (l > 1 && child >= N && pl.left[child] < N && pl.right[child] < N) {
          out[pl.left[child]] = blocks;
          out[pl.right[child]] = blocks;
        }
      }
    }
  }
}

// Level order of the pre-order launches: within each level, the nodes with two
// cherry children, then those with one, then the rest (host [N-1]; fuse[2 l]
// and fuse[2 l + 1] count the first two groups of level l).
void nuc_pre_order_nodes(const EpochInstance* in, std::vector<int32_t>& nodes, std::vector<int>& fuse) {
  const auto& pl = in->plan;
  const int N = in->N;
  nodes.assign(pl.level_nodes.begin(), pl.level_nodes.end());
  fuse.assign(2 * (pl.n_levels + 2), 0);
  auto is_cherry = [&](int v) { return v >= N && pl.left[v] < N && pl.right[v] < N; };
  for (int l = 1; l <= pl.n_levels; ++l) {
    std::vector<int32_t> group[3];
    for (int k = pl.level_offset[l]; k < pl.level_offset[l + 1]; ++k) {
      const int u = pl.level_nodes[k];
      const int nc = l > 1 ? (int)is_cherry(pl.left[u]) + (int)is_cherry(pl.right[u]) : 0;
      group[2 - nc].push_back(u);
    }
    fuse[2 * l] = (int)group[0].size();
    fuse[2 * l + 1] = (int)group[1].size();
    auto dst = nodes.begin() + pl.level_offset[l];
    for (auto& gr : group) dst = std::copy(gr.begin(), gr.end(), dst);
  }
}

int launch_nuc_post(EpochInstance* in) {
  return launch_nuc_post_nodes(in, in->d_level_nodes, in->plan.level_offset.data());
}

// Level l's nodes are d_nodes[level_off[l] .. level_off[l + 1]): the plan's level lists, or a
// restricted list of the same layout (incremental re-evaluation).
int launch_nuc_post_nodes(EpochInstance* in, const int32_t* d_nodes, const int32_t* level_off) {
  switch (cp_of(in->C)) {
    case 1: return in->fp64 ? post_dispatch_cp<double, 1>(in, d_nodes, level_off) : post_dispatch_cp<float, 1>(in, d_nodes, level_off);
    case 2: return in->fp64 ? post_dispatch_cp<double, 2>(in, d_nodes, level_off) : post_dispatch_cp<float, 2>(in, d_nodes, level_off);
    case 4: return in->fp64 ? post_dispatch_cp<double, 4>(in, d_nodes, level_off) : post_dispatch_cp<float, 4>(in, d_nodes, level_off);
    default: return in->fp64 ? post_dispatch_cp<double, 8>(in, d_nodes, level_off) : post_dispatch_cp<float, 8>(in, d_nodes, level_off);
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
