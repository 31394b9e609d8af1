// Four-state pruning (Eq. 4) and its adjoint as one traversal of the whole tree
// per tile of patterns.
//
// Felsenstein's recursion never mixes patterns, so a wavefront can carry one
// tile of patterns (lane = (pattern, category), as in the level kernels)
// through every node of the tree without waiting for any other wavefront.
// The host turns the tree into a short program (build_walk_programs); every
// wavefront runs it for each of its tiles:
//   POST u: x_u = (P_a x_a) o (P_b x_b), rescaled per pattern by a power of
//           two whose exponent joins the pattern's running total;
//   PRE u:  from the outside vector q_u and the children's partials, the
//           pattern's share of dlogL/dl for the branches above a and b, and
//           the outside vectors q_a = P_a^T (q_u o P_b x_b) (likewise q_b) of
//           internal children.
// Vectors in flight sit in a per-wavefront stack in LDS; the host orders the
// children so that few slots are needed (about log2 N for balanced trees).
// HBM sees one write (post-order) and one read (pre-order) of the partials of
// the nodes the pre-order program reads; outside vectors never leave the chip,
// and small subtrees are recomputed from tip states instead of being stored.
// Tip children use precomputed columns of P and dP/dl (column 4 = row sums
// for a missing state), so a tip costs one 16-byte load instead of a 4x4
// product.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <vector>

#include "device_common.h"
#include "instance.h"
#include "nuc_common.h"

namespace epochlik {

namespace {
using namespace nuc;

constexpr size_t kWalkMaxLds = 64 * 1024;  // per block
// stand-in region: 64 read entries, 64 written entries, 64 written int32 (V4<double> size)
constexpr size_t kWalkDummyBytes = 192 * 32;

template <typename T>
struct WalkArgs {
  const int4* ops;
  int n_ops;
  const T* Pm;            // [n][C][4][4]
  const T* dPm;           // [n][C][4][4] (pre-order program only)
  const V4<T>* tcol;      // FP64 walk: [N][C][5] columns of the tip branches' P, then [N][C][5] of their dP/dl
  const T* PmT;           // FP32 walk: [n][C][4][4] transposed transition matrices
  const uint8_t* tips;    // [N][P]
  V4<T>* part;            // [N-1][C][P]
  int32_t* root_scales;   // [P]: each pattern's total exponent (the root's row of the scales)
  const int32_t* slot_of; // [n_nodes]: partial slot of each stored node, -1 otherwise
  const double* pi;       // [4]
  const double* cat;      // rates[8], weights[8]
  const T* weightsT;      // [P]
  T* dpart;               // [groups][n_nodes]: dlogL/dl shares of each group of tiles
  V4<T>* dummy;           // [128]: read (first 64) and write (last 64) stand-ins
  int N, P, C, n_tiles, slots, n_nodes, root, n_groups;
};

// LDS bytes of one wavefront: NT stacks of slots + 1 (the discard slot) entries of 64 lanes
template <typename T>
__host__ __device__ inline size_t walk_lds_per_wave(int slots, int nt) {
  return (size_t)nt * (slots + 1) * 64 * sizeof(nuc::V4<T>);
}

template <int CTRL>
__device__ inline float dpp_mov(float v) {
  return __int_as_float(__builtin_amdgcn_mov_dpp(__float_as_int(v), CTRL, 0xF, 0xF, false));
}
template <int CTRL>
__device__ inline double dpp_mov(double v) {
  const long long b = __double_as_longlong(v);
  const int l = __builtin_amdgcn_mov_dpp((int)(b & 0xffffffffLL), CTRL, 0xF, 0xF, false);
  const int h = __builtin_amdgcn_mov_dpp((int)(b >> 32), CTRL, 0xF, 0xF, false);
  return __longlong_as_double(((long long)h << 32) | (unsigned int)l);
}

// Sum over the 64 lanes in a fixed order; every lane receives the total.
template <typename T>
__device__ inline T wave_sum(T v) {
  v += dpp_mov<0xB1>(v);   // quad_perm [1,0,3,2]
  v += dpp_mov<0x4E>(v);   // quad_perm [2,3,0,1]
  v += dpp_mov<0x124>(v);  // row_ror:4
  v += dpp_mov<0x128>(v);  // row_ror:8
  v += __shfl_xor(v, 16, 64);
  v += __shfl_xor(v, 32, 64);
  return v;
}

template <typename T>
struct Fetch {
  V4<T> xa, xb;
  int sta, stb;
};

// One operation, read through the constant address space so that the uniform
// loads become scalar loads (they then never wait for vector memory).
struct Op {
  int info, a, b, u;
};
__device__ inline Op load_op(const int4* ops, int i) {
  const __attribute__((address_space(4))) int* q =
      (const __attribute__((address_space(4))) int*)(const void*)(ops + i);
  return Op{q[0], q[1], q[2], q[3]};
}

// Per-lane constants of a walk; NT tiles of patterns travel together.
template <typename T, int NT>
struct Lane {
  V4<T>* stk[NT];  // this lane's element of stack slot 0 of each tile (slot s at stk[t][64 s])
  const V4<T>* rdummy;  // a small cached region read in place of absent operands
  V4<T>* wdummy;        // a small region written in place of discarded results
  int c, cl, lane;
  int p[NT], pc[NT];
  bool cat_ok, valid[NT];
  T wc, wt[NT];
  V4<T> qroot;
  size_t tcol_d;
  size_t drow;  // row of dpart for this group of tiles
};

// Long-latency loads of an operation: tip states and stored partials.  Every
// load is issued whatever the operands' kinds (absent ones read a cached dummy
// region), so the loop holds no memory operation under a branch and the
// compiler can wait for exactly the loads each value needs.
template <typename T, int NT>
__device__ inline void fetch_op(const WalkArgs<T>& g, const Lane<T, NT>& L, const Op& op, Fetch<T> (&f)[NT]) {
  const int ka = (op.info >> 3) & 3, kb = (op.info >> 5) & 3;
  const int ta = op.a < g.N ? op.a : g.N - 1, tb = op.b < g.N ? op.b : g.N - 1;
  const size_t ra = ka == kWalkHbm ? (size_t)g.slot_of[op.a] * g.C + L.c : 0;
  const size_t rb = kb == kWalkHbm ? (size_t)g.slot_of[op.b] * g.C + L.c : 0;
#pragma unroll
  for (int t = 0; t < NT; ++t) {
    f[t].sta = g.tips[(size_t)ta * g.P + L.pc[t]];
    f[t].stb = g.tips[(size_t)tb * g.P + L.pc[t]];
    f[t].xa = *(ka == kWalkHbm ? g.part + ra * g.P + L.pc[t] : L.rdummy + L.lane);
    f[t].xb = *(kb == kWalkHbm ? g.part + rb * g.P + L.pc[t] : L.rdummy + L.lane);
  }
}

template <int CP, typename T>
__device__ inline int normalise(V4<T>& v, bool cat_ok) {
  const T m = group_max_cp<CP>(cat_ok ? max4(v) : T(0));
  const int e = scale_exponent(m);
#pragma unroll
  for (int i = 0; i < 4; ++i) v.v[i] = scale_by_pow2(v.v[i], e);
  return e;
}

// One operation of the program for NT tiles.  Order of memory operations: this
// operation's cached loads (matrices, tip columns), then the next operation's
// HBM loads, LDS reads, arithmetic, then every write.
template <typename T, int CP, bool PRE, int NT>
__device__ inline void walk_step(const WalkArgs<T>& g, const Lane<T, NT>& L, const Op& op,
                                 const Fetch<T> (&cur)[NT], bool has_next, const Op& nop, Fetch<T> (&nxt)[NT],
                                 int (&E)[NT]) {
  const int info = op.info, a = op.a, b = op.b, u = op.u;
  const int ka = (info >> 3) & 3, kb = (info >> 5) & 3;
  const int s_a = (info >> 8) & 63, s_b = (info >> 14) & 63, s_q = (info >> 20) & 63, s_qb = (info >> 26) & 63;
  const int c = L.c;
  const M4<T> Ma = load_matrix(g.Pm + ((size_t)a * g.C + c) * 16);
  const M4<T> Mb = load_matrix(g.Pm + ((size_t)b * g.C + c) * 16);
  M4<T> Da, Db;
  if constexpr (PRE) {
    Da = load_matrix(g.dPm + ((size_t)a * g.C + c) * 16);
    Db = load_matrix(g.dPm + ((size_t)b * g.C + c) * 16);
  }
  const size_t ta = (size_t)(a < g.N ? a : g.N - 1) * g.C + c, tb = (size_t)(b < g.N ? b : g.N - 1) * g.C + c;
  V4<T> ca[NT], cb[NT], dca[NT], dcb[NT];
#pragma unroll
  for (int t = 0; t < NT; ++t) {
    const size_t ka5 = ta * 16 + (cur[t].sta & 15), kb5 = tb * 16 + (cur[t].stb & 15);  // state-set columns
    ca[t] = g.tcol[ka5];
    cb[t] = g.tcol[kb5];
    if constexpr (PRE) {
      dca[t] = g.tcol[L.tcol_d + ka5];
      dcb[t] = g.tcol[L.tcol_d + kb5];
    }
  }
  __asm__ volatile("" ::: "memory");
  if (has_next) fetch_op(g, L, nop, nxt);

  V4<T> xa[NT], xb[NT], q[NT];
#pragma unroll
  for (int t = 0; t < NT; ++t) {
    const V4<T> sa = L.stk[t][s_a * 64], sb = L.stk[t][s_b * 64];
    xa[t] = ka == kWalkStack ? sa : cur[t].xa;
    xb[t] = kb == kWalkStack ? sb : cur[t].xb;
    if constexpr (PRE) q[t] = (info & kWalkRoot) ? L.qroot : L.stk[t][s_q * 64];
  }
  V4<T> Sa[NT], Sb[NT];
#pragma unroll
  for (int t = 0; t < NT; ++t) {
    Sa[t] = ka == kWalkTip ? ca[t] : matvec(Ma, xa[t]);
    Sb[t] = kb == kWalkTip ? cb[t] : matvec(Mb, xb[t]);
  }

  if (!(info & kWalkPre)) {
    V4<T> y[NT];
    int e[NT];
#pragma unroll
    for (int t = 0; t < NT; ++t) {
#pragma unroll
      for (int k = 0; k < 4; ++k) y[t].v[k] = Sa[t].v[k] * Sb[t].v[k];
      e[t] = normalise<CP>(y[t], L.cat_ok);
    }
#pragma unroll
    for (int t = 0; t < NT; ++t) {
      L.stk[t][s_q * 64] = y[t];  // the discard slot for the root
      if constexpr (!PRE) {
        E[t] += e[t];
        const bool st = (info & kWalkStore) && L.valid[t];
        *(st ? g.part + ((size_t)g.slot_of[u] * g.C + c) * g.P + L.p[t] : L.wdummy + L.lane) = y[t];
        int32_t* sp = ((info & kWalkRoot) && L.cl == 0 && L.valid[t]) ? g.root_scales + L.p[t]
                                                                       : reinterpret_cast<int32_t*>(L.wdummy + 64) + L.lane;
        *sp = E[t];
      }
    }
  } else if constexpr (PRE) {
    T ga = T(0), gb = T(0);
    V4<T> qa[NT], qb[NT];
#pragma unroll
    for (int t = 0; t < NT; ++t) {
      V4<T> Ua, Ub;
      Ua = ka == kWalkTip ? dca[t] : matvec(Da, xa[t]);
      Ub = kb == kWalkTip ? dcb[t] : matvec(Db, xb[t]);
      T l = T(0);
#pragma unroll
      for (int k = 0; k < 4; ++k) l += q[t].v[k] * Sa[t].v[k] * Sb[t].v[k];
      l = group_sum_cp<CP>(l * L.wc);
      const T f = (l > T(0) ? L.wt[t] / l : T(0)) * L.wc;
      V4<T> ta, tb;
      T ha = T(0), hb = T(0);
#pragma unroll
      for (int k = 0; k < 4; ++k) {
        ta.v[k] = q[t].v[k] * Sb[t].v[k];
        tb.v[k] = q[t].v[k] * Sa[t].v[k];
        ha += ta.v[k] * Ua.v[k];
        hb += tb.v[k] * Ub.v[k];
      }
      ga += ha * f;
      gb += hb * f;
      qa[t] = matvec_t(Ma, ta);
      qb[t] = matvec_t(Mb, tb);
      normalise<CP>(qa[t], L.cat_ok);
      normalise<CP>(qb[t], L.cat_ok);
    }
    ga = wave_sum(ga);
    gb = wave_sum(gb);
#pragma unroll
    for (int t = 0; t < NT; ++t) {  // outputs of tip children go to the discard slot
      L.stk[t][s_q * 64] = qa[t];
      L.stk[t][s_qb * 64] = qb[t];
    }
    if (L.lane == 0) {  // every branch is the child of exactly one PRE operation
      g.dpart[L.drow + a] = ga;
      g.dpart[L.drow + b] = gb;
    }
  }
}

// PRE = false: the post-order program (partials, root partial and exponents).
// PRE = true: the pre-order program (dlogL/dl shares per group of NT tiles).
template <typename T, int CP, bool PRE, int NT>
__global__ __launch_bounds__(256) void nuc_walk_kernel(const WalkArgs<T> g) {
  constexpr int TPW = 64 / CP;
  extern __shared__ __align__(16) unsigned char walk_lds[];
  const int lane = threadIdx.x & 63;
  const int wave = threadIdx.x >> 6;
  const int wpb = blockDim.x >> 6;
  Lane<T, NT> L;
  V4<T>* const wlds = reinterpret_cast<V4<T>*>(walk_lds) + (size_t)wave * NT * (g.slots + 1) * 64 + lane;
#pragma unroll
  for (int t = 0; t < NT; ++t) L.stk[t] = wlds + (size_t)t * (g.slots + 1) * 64;
  L.rdummy = g.dummy;
  L.wdummy = g.dummy + 64;
  L.lane = lane;
  L.cl = lane & (CP - 1);
  L.cat_ok = L.cl < g.C;
  L.c = L.cat_ok ? L.cl : 0;
  L.wc = L.cat_ok ? T(g.cat[kMaxCategories + L.c]) : T(0);
#pragma unroll
  for (int i = 0; i < 4; ++i) L.qroot.v[i] = T(g.pi[i]);
  L.tcol_d = (size_t)g.N * g.C * 16;  // offset of the dP/dl columns
  const int n = g.n_ops;
  const int n_groups = (g.n_tiles + NT - 1) / NT;

  for (int grp = blockIdx.x * wpb + wave; grp < n_groups; grp += gridDim.x * wpb) {
    L.drow = (size_t)grp * g.n_nodes;
#pragma unroll
    for (int t = 0; t < NT; ++t) {
      L.p[t] = (grp * NT + t) * TPW + lane / CP;
      L.valid[t] = L.p[t] < g.P && L.cat_ok;
      L.pc[t] = L.p[t] < g.P ? L.p[t] : g.P - 1;
      L.wt[t] = T(0);
      if constexpr (PRE) L.wt[t] = L.valid[t] ? g.weightsT[L.pc[t]] : T(0);
    }
    int E[NT];
#pragma unroll
    for (int t = 0; t < NT; ++t) E[t] = 0;
    // unrolled by two so that the two fetch buffers swap roles without copies
    Op o0 = load_op(g.ops, 0);
    Op o1 = load_op(g.ops, n > 1 ? 1 : 0);
    Fetch<T> f0[NT], f1[NT];
    fetch_op(g, L, o0, f0);
    for (int i = 0;;) {
      const Op o2 = load_op(g.ops, i + 2 < n ? i + 2 : 0);
      walk_step<T, CP, PRE, NT>(g, L, o0, f0, i + 1 < n, o1, f1, E);
      if (++i >= n) break;
      const Op o3 = load_op(g.ops, i + 2 < n ? i + 2 : 0);
      walk_step<T, CP, PRE, NT>(g, L, o1, f1, i + 1 < n, o2, f0, E);
      if (++i >= n) break;
      o0 = o2;
      o1 = o3;
    }
    if constexpr (PRE) {
      if (lane == 0) g.dpart[L.drow + g.root] = T(0);
    }
  }
}

// ---------------------------------------------------------------------------
// FP32 walk on matrix cores.  Lanes are category-major (lane = c * TPW +
// pattern), so every group of 4 consecutive lanes shares one category and the
// 4x4 products of the whole wavefront are 16 independent 4x4x1 matrix-core
// blocks: with lane 4b + i holding row i of M (A operand) and each lane its own
// vector component k (B operand), four accumulating instructions leave
// (M x)_i of every lane in its register i.  A lane thus loads one 16-byte row
// of each matrix instead of the whole matrix.
typedef float f4v __attribute__((ext_vector_type(4)));

__device__ inline f4v mv_mfma(const f4v& A, const V4<float>& x) {
  f4v d = {0.f, 0.f, 0.f, 0.f};
  d = __builtin_amdgcn_mfma_f32_4x4x1f32(A[0], x.v[0], d, 0, 0, 0);
  d = __builtin_amdgcn_mfma_f32_4x4x1f32(A[1], x.v[1], d, 0, 0, 0);
  d = __builtin_amdgcn_mfma_f32_4x4x1f32(A[2], x.v[2], d, 0, 0, 0);
  d = __builtin_amdgcn_mfma_f32_4x4x1f32(A[3], x.v[3], d, 0, 0, 0);
  return d;
}
__device__ inline V4<float> to_v4(const f4v& d) {
  V4<float> r;
  r.v[0] = d[0];
  r.v[1] = d[1];
  r.v[2] = d[2];
  r.v[3] = d[3];
  return r;
}
__device__ inline f4v load_row(const float* __restrict__ p) { return *reinterpret_cast<const f4v*>(p); }

// Reductions over the CP lanes of one pattern (lanes p, p + TPW, ...).  The
// gfx950 lane-swap instructions hand each lane the pair sum (or max) across
// lane bit 4 or 5 without going through LDS; bit 3 is a DPP row rotation.
template <bool MAX>
__device__ inline float pair_op(float a, float b) {
  return MAX ? fmaxf(a, b) : a + b;
}
template <int CP, bool MAX>
__device__ inline float cat_reduce(float v) {
  if constexpr (CP >= 8) v = pair_op<MAX>(v, dpp_mov<0x128>(v));  // row_ror:8 = lane ^ 8
  if constexpr (CP >= 4) {
    const auto s = __builtin_amdgcn_permlane16_swap(__float_as_uint(v), __float_as_uint(v), false, false);
    v = pair_op<MAX>(__uint_as_float(s[0]), __uint_as_float(s[1]));
  }
  if constexpr (CP >= 2) {
    const auto s = __builtin_amdgcn_permlane32_swap(__float_as_uint(v), __float_as_uint(v), false, false);
    v = pair_op<MAX>(__uint_as_float(s[0]), __uint_as_float(s[1]));
  }
  return v;
}
__device__ inline float wave_sum_cm(float v) {
  v += dpp_mov<0xB1>(v);
  v += dpp_mov<0x4E>(v);
  v += dpp_mov<0x124>(v);
  v += dpp_mov<0x128>(v);
  return cat_reduce<4, false>(v);
}
template <int CP>
__device__ inline int normalise_cm(V4<float>& v, bool cat_ok) {
  const float m = cat_reduce<CP, true>(cat_ok ? max4(v) : 0.f);
  const int e = scale_exponent(m);
#pragma unroll
  for (int i = 0; i < 4; ++i) v.v[i] = scale_by_pow2(v.v[i], e);
  return e;
}

// Raw buffer access: the base and size come from scalar registers and each
// lane adds a fixed byte offset.  An operand that is absent is read (or
// written) with bit 31 set in the lane offset; every buffer here is smaller
// than 2^31 bytes, so the hardware range check turns that into a zero (or a
// dropped store) without touching memory.  The scalar offset is always 0.
constexpr int kRsrcWord3 = 0x00020000;
__device__ inline __amdgpu_buffer_rsrc_t rsrc(const void* base, uint32_t bytes) {
  return __builtin_amdgcn_make_buffer_rsrc(const_cast<void*>(base), (short)0, (int)bytes, kRsrcWord3);
}
constexpr uint32_t kAbsent = 0x80000000u;
__device__ inline f4v bload16(__amdgpu_buffer_rsrc_t r, uint32_t voff) {
  return __builtin_bit_cast(f4v, __builtin_amdgcn_raw_buffer_load_b128(r, voff, 0, 0));
}
__device__ inline V4<float> bload_v4(__amdgpu_buffer_rsrc_t r, uint32_t voff) { return to_v4(bload16(r, voff)); }
__device__ inline void bstore_v4(const V4<float>& x, __amdgpu_buffer_rsrc_t r, uint32_t voff) {
  const f4v v = {x.v[0], x.v[1], x.v[2], x.v[3]};
  __builtin_amdgcn_raw_buffer_store_b128(__builtin_bit_cast(__attribute__((ext_vector_type(4))) unsigned, v), r,
                                         voff, 0, 0);
}

template <int NT>
struct LaneM {
  V4<float>* stk[NT];
  int c, lane;
  uint32_t voff_m;      // byte offset of this lane's matrix row: (c * 16 + 4 * (lane & 3)) * 4
  uint32_t voff_t[NT];  // tip state byte of this lane's pattern
  uint32_t voff_p[NT];  // partial of this lane (clamped pattern), bytes within a node's [C][P][4]
  uint32_t voff_s[NT];  // the same for stores; past the end for lanes without a pattern
  bool cat_ok, valid[NT];
  int p[NT];
  float wc, wt[NT];
  V4<float> qroot;
  uint32_t drow;        // byte offset of this group's row of dlogL/dl shares
};

struct FetchM {
  V4<float> xa, xb;
  int sta, stb;
};

// Tip indicator: one-hot for an observed state, all ones for a missing one.
__device__ inline V4<float> tip_vector(int mask) {  // the tip's state set as a 0/1 vector
  V4<float> x;
#pragma unroll
  for (int k = 0; k < 4; ++k) x.v[k] = ((mask >> k) & 1) ? 1.f : 0.f;
  return x;
}

template <int NT>
__device__ inline void fetch_op_m(const WalkArgs<float>& g, const LaneM<NT>& L, const Op& op, FetchM (&f)[NT]) {
  const int ka = (op.info >> 3) & 3, kb = (op.info >> 5) & 3;
  const uint32_t tb_bytes = (uint32_t)g.P, nb = (uint32_t)g.C * g.P * 16;
  const auto rta = rsrc(g.tips + (size_t)(ka == kWalkTip ? op.a : 0) * g.P, tb_bytes);
  const auto rtb = rsrc(g.tips + (size_t)(kb == kWalkTip ? op.b : 0) * g.P, tb_bytes);
  const auto rxa = rsrc(g.part + (size_t)(ka == kWalkHbm ? g.slot_of[op.a] : 0) * g.C * g.P, nb);
  const auto rxb = rsrc(g.part + (size_t)(kb == kWalkHbm ? g.slot_of[op.b] : 0) * g.C * g.P, nb);
  const uint32_t mta = ka == kWalkTip ? 0u : kAbsent, mtb = kb == kWalkTip ? 0u : kAbsent;
  const uint32_t mxa = ka == kWalkHbm ? 0u : kAbsent, mxb = kb == kWalkHbm ? 0u : kAbsent;
#pragma unroll
  for (int t = 0; t < NT; ++t) {
    f[t].sta = __builtin_amdgcn_raw_buffer_load_b8(rta, L.voff_t[t] | mta, 0, 0);
    f[t].stb = __builtin_amdgcn_raw_buffer_load_b8(rtb, L.voff_t[t] | mtb, 0, 0);
    f[t].xa = bload_v4(rxa, L.voff_p[t] | mxa);
    f[t].xb = bload_v4(rxb, L.voff_p[t] | mxb);
  }
}

template <int CP, bool PRE, int NT>
__device__ inline void walk_step_m(const WalkArgs<float>& g, const LaneM<NT>& L, const Op& op,
                                   const FetchM (&cur)[NT], bool has_next, const Op& nop, FetchM (&nxt)[NT],
                                   int (&E)[NT]) {
  const int info = op.info, a = op.a, b = op.b, u = op.u;
  const int ka = (info >> 3) & 3, kb = (info >> 5) & 3;
  const int s_a = (info >> 8) & 63, s_b = (info >> 14) & 63, s_q = (info >> 20) & 63, s_qb = (info >> 26) & 63;
  const uint32_t mb = (uint32_t)g.C * 64;
  const auto rPa = rsrc(g.Pm + (size_t)a * g.C * 16, mb), rPb = rsrc(g.Pm + (size_t)b * g.C * 16, mb);
  const f4v Ra = bload16(rPa, L.voff_m), Rb = bload16(rPb, L.voff_m);
  f4v Ca, Cb, DRa, DRb;
  if constexpr (PRE) {
    Ca = bload16(rsrc(g.PmT + (size_t)a * g.C * 16, mb), L.voff_m);
    Cb = bload16(rsrc(g.PmT + (size_t)b * g.C * 16, mb), L.voff_m);
    DRa = bload16(rsrc(g.dPm + (size_t)a * g.C * 16, mb), L.voff_m);
    DRb = bload16(rsrc(g.dPm + (size_t)b * g.C * 16, mb), L.voff_m);
  }
  __asm__ volatile("" ::: "memory");
  if (has_next) fetch_op_m(g, L, nop, nxt);

  V4<float> xa[NT], xb[NT], q[NT];
#pragma unroll
  for (int t = 0; t < NT; ++t) {
    const V4<float> sa = L.stk[t][s_a * 64], sb = L.stk[t][s_b * 64];
    xa[t] = ka == kWalkStack ? sa : (ka == kWalkTip ? tip_vector(cur[t].sta) : cur[t].xa);
    xb[t] = kb == kWalkStack ? sb : (kb == kWalkTip ? tip_vector(cur[t].stb) : cur[t].xb);
    if constexpr (PRE) q[t] = (info & kWalkRoot) ? L.qroot : L.stk[t][s_q * 64];
  }
  V4<float> Sa[NT], Sb[NT];
#pragma unroll
  for (int t = 0; t < NT; ++t) {
    Sa[t] = to_v4(mv_mfma(Ra, xa[t]));
    Sb[t] = to_v4(mv_mfma(Rb, xb[t]));
  }

  if (!(info & kWalkPre)) {
    const uint32_t nb = (uint32_t)g.C * g.P * 16;
    const int su = g.slot_of[u];  // -1 for a node the post-order program does not store
    const auto rS = rsrc(g.part + (size_t)(su < 0 ? 0 : su) * g.C * g.P, nb);
    const uint32_t mS = (!PRE && (info & kWalkStore)) ? 0u : kAbsent;
#pragma unroll
    for (int t = 0; t < NT; ++t) {
      V4<float> y;
#pragma unroll
      for (int k = 0; k < 4; ++k) y.v[k] = Sa[t].v[k] * Sb[t].v[k];
      const int e = normalise_cm<CP>(y, L.cat_ok);
      L.stk[t][s_q * 64] = y;  // the discard slot for the root
      if constexpr (!PRE) {
        E[t] += e;
        bstore_v4(y, rS, L.voff_s[t] | mS);
      }
    }
  } else if constexpr (PRE) {
    float ga = 0.f, gb = 0.f;
#pragma unroll
    for (int t = 0; t < NT; ++t) {
      const V4<float> Ua = to_v4(mv_mfma(DRa, xa[t])), Ub = to_v4(mv_mfma(DRb, xb[t]));
      float l = 0.f;
#pragma unroll
      for (int k = 0; k < 4; ++k) l += q[t].v[k] * Sa[t].v[k] * Sb[t].v[k];
      l = cat_reduce<CP, false>(l * L.wc);
      const float f = (l > 0.f ? L.wt[t] / l : 0.f) * L.wc;
      V4<float> ta, tb;
      float ha = 0.f, hb = 0.f;
#pragma unroll
      for (int k = 0; k < 4; ++k) {
        ta.v[k] = q[t].v[k] * Sb[t].v[k];
        tb.v[k] = q[t].v[k] * Sa[t].v[k];
        ha += ta.v[k] * Ua.v[k];
        hb += tb.v[k] * Ub.v[k];
      }
      ga += ha * f;
      gb += hb * f;
      V4<float> qa = to_v4(mv_mfma(Ca, ta)), qb = to_v4(mv_mfma(Cb, tb));
      normalise_cm<CP>(qa, L.cat_ok);
      normalise_cm<CP>(qb, L.cat_ok);
      L.stk[t][s_q * 64] = qa;  // q_u's (consumed) slot or the discard slot when a is a tip
      L.stk[t][s_qb * 64] = qb;
    }
    ga = wave_sum_cm(ga);
    gb = wave_sum_cm(gb);
    const auto rD = rsrc(g.dpart, (uint32_t)g.n_groups * g.n_nodes * 4);
    const uint32_t vD = L.lane == 0 ? L.drow : kAbsent;  // one lane writes, the others fall outside
    __builtin_amdgcn_raw_buffer_store_b32(__float_as_uint(ga), rD, vD + (uint32_t)a * 4, 0, 0);
    __builtin_amdgcn_raw_buffer_store_b32(__float_as_uint(gb), rD, vD + (uint32_t)b * 4, 0, 0);
  }
}

template <int CP, bool PRE, int NT>
__global__ __launch_bounds__(256) void nuc_walk_mfma_kernel(const WalkArgs<float> g) {
  constexpr int TPW = 64 / CP;
  extern __shared__ __align__(16) unsigned char walk_lds[];
  const int lane = threadIdx.x & 63;
  const int wave = threadIdx.x >> 6;
  const int wpb = blockDim.x >> 6;
  LaneM<NT> L;
  V4<float>* const wlds = reinterpret_cast<V4<float>*>(walk_lds) + (size_t)wave * NT * (g.slots + 1) * 64 + lane;
#pragma unroll
  for (int t = 0; t < NT; ++t) L.stk[t] = wlds + (size_t)t * (g.slots + 1) * 64;
  L.lane = lane;
  const int cl = lane / TPW;  // category-major lanes
  L.cat_ok = cl < g.C;
  L.c = L.cat_ok ? cl : 0;
  L.voff_m = (uint32_t)(L.c * 16 + 4 * (lane & 3)) * 4;
  L.wc = L.cat_ok ? float(g.cat[kMaxCategories + L.c]) : 0.f;
#pragma unroll
  for (int i = 0; i < 4; ++i) L.qroot.v[i] = float(g.pi[i]);
  const int n = g.n_ops;

  for (int grp = blockIdx.x * wpb + wave; grp < g.n_groups; grp += gridDim.x * wpb) {
    L.drow = (uint32_t)grp * g.n_nodes * 4;
#pragma unroll
    for (int t = 0; t < NT; ++t) {
      const int p = (grp * NT + t) * TPW + lane % TPW;
      const int pc = p < g.P ? p : g.P - 1;
      L.p[t] = p;
      L.valid[t] = p < g.P && L.cat_ok;
      L.voff_t[t] = (uint32_t)pc;
      L.voff_p[t] = ((uint32_t)L.c * g.P + pc) * 16;
      L.voff_s[t] = L.valid[t] ? ((uint32_t)L.c * g.P + p) * 16 : kAbsent;
      L.wt[t] = 0.f;
      if constexpr (PRE) L.wt[t] = L.valid[t] ? g.weightsT[pc] : 0.f;
    }
    int E[NT];
#pragma unroll
    for (int t = 0; t < NT; ++t) E[t] = 0;
    Op o0 = load_op(g.ops, 0);
    Op o1 = load_op(g.ops, n > 1 ? 1 : 0);
    FetchM f0[NT], f1[NT];
    fetch_op_m(g, L, o0, f0);
    for (int i = 0;;) {
      const Op o2 = load_op(g.ops, i + 2 < n ? i + 2 : 0);
      walk_step_m<CP, PRE, NT>(g, L, o0, f0, i + 1 < n, o1, f1, E);
      if (++i >= n) break;
      const Op o3 = load_op(g.ops, i + 2 < n ? i + 2 : 0);
      walk_step_m<CP, PRE, NT>(g, L, o1, f1, i + 1 < n, o2, f0, E);
      if (++i >= n) break;
      o0 = o2;
      o1 = o3;
    }
    if constexpr (PRE) {
      if (lane == 0) g.dpart[(size_t)grp * g.n_nodes + g.root] = 0.f;
    } else {  // the pattern's total exponent, with the root's partial
#pragma unroll
      for (int t = 0; t < NT; ++t)
        if (L.valid[t] && L.c == 0) g.root_scales[L.p[t]] = E[t];
    }
  }
}

// Transposed transition matrices (row i of PmT[v][c] = column i of Pm[v][c]).
__global__ __launch_bounds__(256) void walk_transpose_kernel(const float* __restrict__ Pm, int n_mats,
                                                             float* __restrict__ PmT) {
  const int t = blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= n_mats * 16) return;
  const int m = t / 16, i = (t / 4) % 4, j = t % 4;
  PmT[(size_t)m * 16 + 4 * i + j] = Pm[(size_t)m * 16 + 4 * j + i];
}

// Columns of P (and dP/dl) of every tip branch: tcol[m][v][c][j] for j < 4 is
// column j, j = 4 holds the row sums (a missing tip state).
template <typename T>
__global__ __launch_bounds__(256) void walk_tipcol_kernel(const T* __restrict__ Pm, const T* __restrict__ dPm, int N,
                                                          int C, V4<T>* __restrict__ tcol) {
  // column j (a state set, 1..15) = sum over its states of column P[:, state]
  const int per = N * C * 16;
  const int t = blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= (dPm ? 2 : 1) * per) return;
  const int m = t / per, r = t % per;
  const int v = r / (C * 16), c = (r / 16) % C, j = r % 16;
  const T* M = (m ? dPm : Pm) + ((size_t)v * C + c) * 16;
  V4<T> col;
#pragma unroll
  for (int i = 0; i < 4; ++i) {
    const T m0 = (j & 1) ? M[4 * i] : T(0), m1 = (j & 2) ? M[4 * i + 1] : T(0);
    const T m2 = (j & 4) ? M[4 * i + 2] : T(0), m3 = (j & 8) ? M[4 * i + 3] : T(0);
    col.v[i] = (m0 + m1) + (m2 + m3);
  }
  tcol[t] = col;
}

// dlogL/dl of every branch: fixed-order FP64 sums of its per-tile shares, first
// over strided row groups (grid.y), then over the groups.
constexpr int kWalkRowGroups = 32;
template <typename T>
__global__ __launch_bounds__(256) void walk_dbranch_rows_kernel(const T* __restrict__ dpart, int n_tiles, int n_nodes,
                                                                double* __restrict__ part2) {
  const int v = blockIdx.x * 256 + threadIdx.x;
  if (v >= n_nodes) return;
  double s = 0.0;
  for (int t = blockIdx.y; t < n_tiles; t += kWalkRowGroups) s += (double)dpart[(size_t)t * n_nodes + v];
  part2[(size_t)blockIdx.y * n_nodes + v] = s;
}
__global__ __launch_bounds__(256) void walk_dbranch_final_kernel(const double* __restrict__ part2, int n_nodes,
                                                                 double* __restrict__ dbranch) {
  const int v = blockIdx.x * 256 + threadIdx.x;
  if (v >= n_nodes) return;
  double s = 0.0;
  for (int r = 0; r < kWalkRowGroups; ++r) s += part2[(size_t)r * n_nodes + v];
  dbranch[v] = s;
}

int cp_walk(int C) { return C <= 1 ? 1 : (C <= 2 ? 2 : (C <= 4 ? 4 : 8)); }

// Tiles per wavefront (they share the matrix operands): walk_nt in FP32 (1 or
// 2), one in FP64.
int walk_nt_of(const EpochInstance* in) { return in->fp64 ? 1 : (in->walk_nt == 1 ? 1 : 2); }

template <typename T>
WalkArgs<T> walk_args(EpochInstance* in, bool pre) {
  WalkArgs<T> g{};
  const int4* ops = static_cast<const int4*>(in->walk_ops.ptr);
  g.ops = pre ? ops + in->walk.post.size() / 4 : ops;
  g.n_ops = (int)((pre ? in->walk.pre.size() : in->walk.post.size()) / 4);
  g.Pm = static_cast<const T*>(in->Pm.ptr);
  g.dPm = static_cast<const T*>(in->dPm.ptr);
  g.tcol = static_cast<const V4<T>*>(in->walk_tcol.ptr);
  g.PmT = static_cast<const T*>(in->walk_tcol.ptr);
  g.tips = static_cast<const uint8_t*>(in->tips.ptr);
  g.part = static_cast<V4<T>*>(in->partials.ptr);
  g.root_scales = static_cast<int32_t*>(in->scales.ptr) + (size_t)in->root_slot * in->P;
  g.slot_of = static_cast<const int32_t*>(in->walk_slots.ptr);
  g.pi = static_cast<const double*>(in->pi.ptr);
  g.cat = static_cast<const double*>(in->cat.ptr);
  g.weightsT = static_cast<const T*>(in->weightsT.ptr);
  g.dpart = static_cast<T*>(in->walk_dpart.ptr);
  g.dummy = static_cast<V4<T>*>(in->walk_dummy.ptr);
  g.N = in->N;
  g.P = in->P;
  g.C = in->C;
  g.n_tiles = walk_tiles(in);
  g.slots = std::max(1, pre ? in->walk.pre_slots : in->walk.post_slots);
  g.n_nodes = in->n_nodes;
  g.root = in->plan.root;
  g.n_groups = (g.n_tiles + walk_nt_of(in) - 1) / walk_nt_of(in);
  return g;
}


template <typename T, int CP, int NT>
int walk_launch(EpochInstance* in, bool pre) {
  const WalkArgs<T> g = walk_args<T>(in, pre);
  const size_t per_wave = walk_lds_per_wave<T>(g.slots, NT);
  int wpb = 4;  // wavefronts per block, each with its own stacks
  while (wpb > 1 && wpb * per_wave > kWalkMaxLds) wpb >>= 1;
  const size_t lds = wpb * per_wave;
  const int groups = (g.n_tiles + NT - 1) / NT;
  int blocks = (groups + wpb - 1) / wpb;
  if (in->walk_blocks > 0) blocks = std::min(blocks, in->walk_blocks);
  if constexpr (sizeof(T) == 4) {
    if (pre)
      hipLaunchKernelGGL((nuc_walk_mfma_kernel<CP, true, NT>), dim3(blocks), dim3(64 * wpb), lds, in->stream, g);
    else
      hipLaunchKernelGGL((nuc_walk_mfma_kernel<CP, false, NT>), dim3(blocks), dim3(64 * wpb), lds, in->stream, g);
  } else {
    if (pre)
      hipLaunchKernelGGL((nuc_walk_kernel<T, CP, true, NT>), dim3(blocks), dim3(64 * wpb), lds, in->stream, g);
    else
      hipLaunchKernelGGL((nuc_walk_kernel<T, CP, false, NT>), dim3(blocks), dim3(64 * wpb), lds, in->stream, g);
  }
  int rc = hip_check(hipGetLastError(), pre ? "nuc_walk pre-order launch" : "nuc_walk post-order launch");
  if (rc || !pre) return rc;
  double* part2 = reinterpret_cast<double*>(static_cast<char*>(in->walk_dpart.ptr) + walk_dpart_rows_bytes(in));
  const int nb = (in->n_nodes + 255) / 256;
  hipLaunchKernelGGL((walk_dbranch_rows_kernel<T>), dim3(nb, kWalkRowGroups), dim3(256), 0, in->stream, g.dpart,
                     groups, in->n_nodes, part2);
  hipLaunchKernelGGL(walk_dbranch_final_kernel, dim3(nb), dim3(256), 0, in->stream, part2, in->n_nodes,
                     static_cast<double*>(in->dbranch.ptr));
  return hip_check(hipGetLastError(), "walk_dbranch launch");
}

template <typename T, int CP>
int walk_launch_nt(EpochInstance* in, bool pre) {
  if constexpr (sizeof(T) == 4) {
    if (walk_nt_of(in) == 2) return walk_launch<T, CP, 2>(in, pre);
  }
  return walk_launch<T, CP, 1>(in, pre);
}

template <typename T>
int walk_dispatch(EpochInstance* in, bool pre) {
  switch (cp_walk(in->C)) {
    case 1: return walk_launch_nt<T, 1>(in, pre);
    case 2: return walk_launch_nt<T, 2>(in, pre);
    case 4: return walk_launch_nt<T, 4>(in, pre);
    default: return walk_launch_nt<T, 8>(in, pre);
  }
}

}  // namespace

int walk_tiles(const EpochInstance* in) {
  const int TPW = 64 / cp_walk(in->C);
  return (in->P + TPW - 1) / TPW;
}

size_t walk_tcol_bytes(const EpochInstance* in) {
  if (!in->fp64) return (size_t)in->n_nodes * in->C * 16 * sizeof(float);  // transposed P
  return (size_t)2 * in->N * in->C * 16 * 4 * sizeof(double);               // state-set columns of P and dP/dl
}

size_t walk_dpart_rows_bytes(const EpochInstance* in) {
  return ((size_t)walk_tiles(in) * in->n_nodes * in->real_size + 255) / 256 * 256;
}

bool walk_fits(const EpochInstance* in, int slots) {
  const size_t per_wave = in->fp64 ? walk_lds_per_wave<double>(std::max(1, slots), walk_nt_of(in))
                                   : walk_lds_per_wave<float>(std::max(1, slots), walk_nt_of(in));
  return per_wave <= kWalkMaxLds;
}

// Automatic choice: the walk where the level kernels cannot fill the chip (a
// launch per level, each with fewer 16-pattern tiles than there are SIMDs).
constexpr int kWalkAutoTiles = 1024;

// Bytes an HBM budget must hold for a walk that stores n_stored partials: the
// partials, the root's scale row and (with gradients) the rows of dlogL/dl shares.
size_t walk_budget_bytes(const EpochInstance* in, size_t n_stored) {
  const size_t V = (size_t)in->C * in->P * in->Kp * in->real_size;
  size_t b = n_stored * V + (size_t)in->P * sizeof(int32_t);
  if (in->cfg.flags & (EPOCH_GRAD_BRANCH | EPOCH_GRAD_Q))
    b += walk_dpart_rows_bytes(in) + (size_t)kWalkRowGroups * in->n_nodes * sizeof(double);
  return b;
}

// Under an HBM budget: the smallest recomputation threshold (tips per subtree)
// whose stored partials fit, or -1.
int walk_budget_threshold(const EpochInstance* in) {
  const auto& pl = in->plan;
  const int N = in->N, n = in->n_nodes;
  std::vector<int> tips(n, 1);
  for (int u : pl.post) tips[u] = tips[pl.left[u]] + tips[pl.right[u]];
  std::vector<int> sizes(tips.begin() + N, tips.end());
  std::sort(sizes.begin(), sizes.end());
  sizes.erase(std::unique(sizes.begin(), sizes.end()), sizes.end());
  for (int T : sizes) {  // nodes with more than T tips are stored, and the root always
    if (T < 2) continue;
    size_t stored = 1;
    for (int u = N; u < n; ++u) stored += (u != pl.root && tips[u] > T) ? 1 : 0;
    if (walk_budget_bytes(in, stored) <= (size_t)in->budget) return T;
  }
  return -1;
}

int walk_prepare(EpochInstance* in) {
  in->walk_ok = false;
  in->root_slot = in->plan.root - in->N;
  // the time gradient reads the branch adjoints G that only the level kernels form
  if (in->path != 1 || in->walk_enable == 0 || (in->cfg.flags & EPOCH_GRAD_TIME)) return EPOCH_OK;
  if (in->walk_enable < 0 && (in->fp64 || walk_tiles(in) > kWalkAutoTiles)) return EPOCH_OK;
  int rt = (in->cfg.flags & EPOCH_GRAD_Q) ? 2 : std::max(2, in->walk_recompute);
  if (in->budget > 0) {
    rt = walk_budget_threshold(in);
    if (rt < 0)
      return set_error(EPOCH_ERR_OOM, "hbm_budget_bytes %lld is below the %zu bytes the root's partial needs",
                       (long long)in->budget, walk_budget_bytes(in, 1));
  }
  bool built = !build_walk_programs(in->plan, rt, in->walk) && walk_fits(in, in->walk.post_slots);
  // When the pre-order program does not fit, the level kernels take the gradient from the
  // walk's stored partials; they recompute only cherries, so every larger subtree must be stored.
  const bool grad = (in->cfg.flags & (EPOCH_GRAD_BRANCH | EPOCH_GRAD_Q)) != 0;
  if (built && grad && in->budget == 0 && rt > 2 && !walk_fits(in, in->walk.pre_slots)) {
    rt = 2;
    built = !build_walk_programs(in->plan, rt, in->walk) && walk_fits(in, in->walk.post_slots);
  }
  if (!built) {
    if (in->budget > 0) return set_error(EPOCH_ERR_ARG, "the tree is too deep for the tree walk an HBM budget needs");
    return EPOCH_OK;  // too deep for the stack: level kernels
  }
  // partial slots: node - N without a budget (the level kernels' layout); under a
  // budget, compact slots for the stored nodes, the root first
  std::vector<int32_t> slot(in->n_nodes, -1);
  size_t n_stored = 0;
  if (in->budget > 0) {
    slot[in->plan.root] = (int32_t)n_stored++;
    for (int u = in->N; u < in->n_nodes; ++u)
      if (u != in->plan.root && in->walk.stored[u]) slot[u] = (int32_t)n_stored++;
    in->root_slot = 0;
  } else {
    for (int u = in->N; u < in->n_nodes; ++u) slot[u] = u - in->N;
  }
  if (!in->fp64) {    // the FP32 walk addresses each node's partials and the gradient rows as buffers below 2^31 bytes
    const size_t groups = ((size_t)walk_tiles(in) + walk_nt_of(in) - 1) / walk_nt_of(in);
    if ((size_t)in->C * in->P * 16 >= (size_t(1) << 31) || groups * in->n_nodes * 4 >= (size_t(1) << 31)) {
      if (in->budget > 0) return set_error(EPOCH_ERR_ARG, "too many patterns for the FP32 tree walk an HBM budget needs");
      return EPOCH_OK;
    }
  }
  std::vector<int32_t> ops(in->walk.post);
  ops.insert(ops.end(), in->walk.pre.begin(), in->walk.pre.end());
  int rc = ensure(in->walk_ops, ops.size() * sizeof(int32_t));
  if (!rc) rc = ensure(in->walk_tcol, walk_tcol_bytes(in));
  if (!rc) rc = ensure(in->walk_slots, slot.size() * sizeof(int32_t));
  if (!rc && in->budget > 0) {
    rc = ensure(in->partials, n_stored * (size_t)in->C * in->P * in->Kp * in->real_size);
    if (!rc) rc = ensure(in->scales, (size_t)in->P * sizeof(int32_t));
  }
  if (!rc)
    rc = hip_check(hipMemcpyAsync(in->walk_slots.ptr, slot.data(), slot.size() * sizeof(int32_t), hipMemcpyHostToDevice,
                                  in->stream), "walk slot upload");
  if (!rc && !in->walk_dummy.ptr) {
    rc = ensure(in->walk_dummy, kWalkDummyBytes);
    if (!rc) rc = hip_check(hipMemsetAsync(in->walk_dummy.ptr, 0, kWalkDummyBytes, in->stream), "walk dummy clear");
  }
  if (!rc && (in->cfg.flags & (EPOCH_GRAD_BRANCH | EPOCH_GRAD_Q)))
    rc = ensure(in->walk_dpart, walk_dpart_rows_bytes(in) + (size_t)kWalkRowGroups * in->n_nodes * sizeof(double));
  if (!rc)
    rc = hip_check(hipMemcpyAsync(in->walk_ops.ptr, ops.data(), ops.size() * sizeof(int32_t), hipMemcpyHostToDevice,
                                  in->stream), "walk program upload");
  if (!rc) rc = hip_check(hipStreamSynchronize(in->stream), "walk program sync");
  if (rc) return rc;
  in->walk_ok = true;
  in->walk_pre_ok = walk_fits(in, in->walk.pre_slots);
  if (in->budget > 0 && !in->walk_pre_ok && (in->cfg.flags & EPOCH_GRAD_BRANCH)) {
    in->walk_ok = false;
    return set_error(EPOCH_ERR_ARG, "the tree is too deep for the pre-order walk an HBM budget needs");
  }
  return EPOCH_OK;
}

int launch_walk_tipcol(EpochInstance* in) {
  if (!in->fp64) {
    const int n_mats = in->n_nodes * in->C;
    hipLaunchKernelGGL(walk_transpose_kernel, dim3((n_mats * 16 + 255) / 256), dim3(256), 0, in->stream,
                       static_cast<const float*>(in->Pm.ptr), n_mats, static_cast<float*>(in->walk_tcol.ptr));
    return hip_check(hipGetLastError(), "walk_transpose launch");
  }
  const bool grad = in->dPm.ptr != nullptr && (in->cfg.flags & (EPOCH_GRAD_BRANCH | EPOCH_GRAD_Q));
  const int n = (grad ? 2 : 1) * in->N * in->C * 16;
  const int blocks = (n + 255) / 256;
  if (in->fp64)
    hipLaunchKernelGGL((walk_tipcol_kernel<double>), dim3(blocks), dim3(256), 0, in->stream,
                       static_cast<const double*>(in->Pm.ptr), grad ? static_cast<const double*>(in->dPm.ptr) : nullptr,
                       in->N, in->C, static_cast<V4<double>*>(in->walk_tcol.ptr));
  else
    hipLaunchKernelGGL((walk_tipcol_kernel<float>), dim3(blocks), dim3(256), 0, in->stream,
                       static_cast<const float*>(in->Pm.ptr), grad ? static_cast<const float*>(in->dPm.ptr) : nullptr,
                       in->N, in->C, static_cast<V4<float>*>(in->walk_tcol.ptr));
  return hip_check(hipGetLastError(), "walk_tipcol launch");
}

int launch_walk_post(EpochInstance* in) { return in->fp64 ? walk_dispatch<double>(in, false) : walk_dispatch<float>(in, false); }

int launch_walk_pre_grad(EpochInstance* in) {
  return in->fp64 ? walk_dispatch<double>(in, true) : walk_dispatch<float>(in, true);
}

}  // namespace epochlik
