// Codon-sized (and amino-acid-sized) kernels on the matrix cores: FP32
// (v_mfma_f32_16x16x4f32) and FP64 (v_mfma_f64_16x16x4f64); an FP32 tip
// child's dlogL/dP also on v_mfma_f32_16x16x32_bf16, with the FP32 operand
// split exactly into three bf16 parts (grad_rows_tip_bf16).
//
// Applies to instances with 48 < K <= 64 (padded to KP = 64, NT = 4 tiles of
// 16 states) or 16 < K <= 32 (padded to KP = 32, NT = 2).  Each rate category
// is a problem of its own (a descriptor of its own): its partials / outside
// vectors [slot][P][KP] and scale exponents [slot][P] are the category's
// region of the instance's buffers, its transition matrices every C-th KP x KP
// row-major block of [node][category]; the root reduction combines the
// categories.
//
// MFMA operand mapping (16x16x4, wavefront of 64 lanes, g = lane / 16,
// r = lane % 16):  A[m][k]: m = r, k = g;  B[k][n]: k = g, n = r;
// D[m][n] (4 registers v): FP32 m = 4 g + v, FP64 m = 4 v + g; n = r.
//
// Work split.  A block takes one internal node and R tiles of 64 patterns;
// it stages the two child transition matrices in LDS (row sums in the
// padding column, so a missing tip state is one more column), and each of
// its four wavefronts then works alone on 16-pattern tiles: D-layout
// registers hold pattern drow(g, v), state 16 nt + r of each 16x16 block nt.
//   child vectors   S = L P^T     A = child partial rows (16-byte loads), B = P rows (LDS)
//   post-order      x = S_a o S_b, per-pattern power-of-two scale (row reduction by DPP)
//   dlogL/dP        G += sum_p (w_p / L_p) t_p L_p^T, contraction over the 16
//                   patterns: A = t (registers), B = child partials in the D layout
//   outside vector  q_c = t P_c    A = t through a wave-private LDS transpose, B = P (LDS)
// with t = q_u o S_sibling.  The four wavefronts' dlogL/dP partials are
// summed in LDS in a fixed order and written to one slot per block; a last
// kernel sums the slots of each branch in FP64.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <climits>
#include <cstring>

#include "device_common.h"
#include "instance.h"

#define EPOCH_GLOBAL __attribute__((address_space(1)))

namespace epochlik {

namespace {

typedef float f4 __attribute__((ext_vector_type(4)));
typedef double d4 __attribute__((ext_vector_type(4)));

// Padded state counts: NT tiles of 16 states, 64 (NT = 4) or 32 (NT = 2).  The
// namespace-level KP, KK, LDP are the 64-state values (the side-split kernel
// and the host); the kernels templated on NT declare their own.
template <int NT>
struct Dim {
  static constexpr int KP = 16 * NT;   // padded states
  static constexpr int KK = KP * KP;   // entries of a transition matrix
  static constexpr int LDP = KP + 4;   // LDS row stride (elements): the states, the row sum, padding
  static constexpr int NCT = NT * NT / 4;  // 16 x 16 tiles of dlogL/dP per wavefront in the gradient phase
};
constexpr int KP = Dim<4>::KP;
constexpr int KK = Dim<4>::KK;
constexpr int LDP = Dim<4>::LDP;
constexpr int TILE = 64;  // patterns per block tile
constexpr int WT = 16;    // patterns per wavefront tile
#define EPOCH_DIMS(NT)                     \
  constexpr int KP = Dim<NT>::KP;          \
  constexpr int KK = Dim<NT>::KK;          \
  constexpr int LDP = Dim<NT>::LDP;        \
  (void)KP;                                \
  (void)KK;                                \
  (void)LDP

// FP32 (v_mfma_f32_16x16x4f32) and FP64 (v_mfma_f64_16x16x4f64) forms of the
// kernels.  The A and B operands map alike; the four D registers of lane
// (g, r) are rows 4 g + v (FP32) or 4 v + g (FP64) of column r.
template <typename T>
struct Vec4;
template <>
struct Vec4<float> {
  typedef f4 type;
};
template <>
struct Vec4<double> {
  typedef d4 type;
};
template <typename T>
using v4 = typename Vec4<T>::type;

__device__ inline f4 mfma(float a, float b, f4 c) { return __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c, 0, 0, 0); }
__device__ inline d4 mfma(double a, double b, d4 c) { return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0); }
template <typename T>
__device__ constexpr int drow(int g, int v) {
  return sizeof(T) == 8 ? 4 * v + g : 4 * g + v;
}

template <typename T>
__device__ inline const EPOCH_GLOBAL T* gptr(const T* p) {
  return (const EPOCH_GLOBAL T*)p;
}
template <typename T>
__device__ inline EPOCH_GLOBAL T* gptr(T* p) {
  return (EPOCH_GLOBAL T*)p;
}

// Orders LDS accesses of one wavefront (write, then read by other lanes).
__device__ inline void wave_lds_sync() {
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
  __builtin_amdgcn_wave_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

// Stage a KP x KP row-major matrix into LDS with row stride LDP, in 16-byte
// pieces (256 threads, t = 0 .. 255).
template <int NT, typename T>
__device__ inline void stage_matrix(T* __restrict__ s, const T* __restrict__ g, int t) {
  EPOCH_DIMS(NT);
  constexpr int PER_ROW = KP * sizeof(T) / 16;  // 16-byte pieces per row
  const EPOCH_GLOBAL f4* src = gptr(reinterpret_cast<const f4*>(g));
  for (int e = t; e < KP * PER_ROW; e += 256) {
    const int row = e / PER_ROW, c = e % PER_ROW;
    *reinterpret_cast<f4*>(reinterpret_cast<char*>(s + row * LDP) + 16 * c) = src[e];
  }
}
template <int NT, typename T>
__device__ inline void stage_matrix(T* __restrict__ s, const T* __restrict__ g) {
  stage_matrix<NT>(s, g, threadIdx.x);
}
// Row sums over the first K columns into column KP (needs the staged matrix;
// 256 threads, t = 0 .. 255: TPR threads per row, CPT columns each).
template <int NT, typename T>
__device__ inline void stage_row_sums(T* __restrict__ s, int K, int t) {
  EPOCH_DIMS(NT);
  constexpr int TPR = 256 / KP, CPT = KP / TPR;
  const int row = t / TPR, q = t % TPR;
  T acc = 0;
#pragma unroll
  for (int j = 0; j < CPT; ++j) acc += (CPT * q + j < K) ? s[row * LDP + CPT * q + j] : T(0);
#pragma unroll
  for (int o = 1; o < TPR; o <<= 1) acc += __shfl_xor(acc, o, TPR);
  if (q == 0) s[row * LDP + KP] = acc;
}
template <int NT, typename T>
__device__ inline void stage_row_sums(T* __restrict__ s, int K) { stage_row_sums<NT>(s, K, threadIdx.x); }

// Row-max / row-sum over the 16 lanes of a DPP row (lanes sharing g).
__device__ inline float row16_max(float v) {
  v = fmaxf(v, __int_as_float(__builtin_amdgcn_mov_dpp(__float_as_int(v), 0x121, 0xF, 0xF, false)));  // row_ror:1
  v = fmaxf(v, __int_as_float(__builtin_amdgcn_mov_dpp(__float_as_int(v), 0x122, 0xF, 0xF, false)));  // row_ror:2
  v = fmaxf(v, __int_as_float(__builtin_amdgcn_mov_dpp(__float_as_int(v), 0x124, 0xF, 0xF, false)));  // row_ror:4
  v = fmaxf(v, __int_as_float(__builtin_amdgcn_mov_dpp(__float_as_int(v), 0x128, 0xF, 0xF, false)));  // row_ror:8
  return v;
}
__device__ inline float row16_sum(float v) {
  v += __int_as_float(__builtin_amdgcn_mov_dpp(__float_as_int(v), 0x121, 0xF, 0xF, false));
  v += __int_as_float(__builtin_amdgcn_mov_dpp(__float_as_int(v), 0x122, 0xF, 0xF, false));
  v += __int_as_float(__builtin_amdgcn_mov_dpp(__float_as_int(v), 0x124, 0xF, 0xF, false));
  v += __int_as_float(__builtin_amdgcn_mov_dpp(__float_as_int(v), 0x128, 0xF, 0xF, false));
  return v;
}
// The same for doubles, moving the two 32-bit halves.
template <int CTRL>
__device__ inline double dpp_double(double v) {
  const long long b = __double_as_longlong(v);
  const int lo = __builtin_amdgcn_mov_dpp((int)(b & 0xffffffffll), CTRL, 0xF, 0xF, false);
  const int hi = __builtin_amdgcn_mov_dpp((int)(b >> 32), CTRL, 0xF, 0xF, false);
  return __longlong_as_double(((long long)hi << 32) | (unsigned)lo);
}
__device__ inline double row16_max(double v) {
  v = fmax(v, dpp_double<0x121>(v));
  v = fmax(v, dpp_double<0x122>(v));
  v = fmax(v, dpp_double<0x124>(v));
  v = fmax(v, dpp_double<0x128>(v));
  return v;
}
__device__ inline double row16_sum(double v) {
  v += dpp_double<0x121>(v);
  v += dpp_double<0x122>(v);
  v += dpp_double<0x124>(v);
  v += dpp_double<0x128>(v);
  return v;
}

// Tip states of the patterns of D-layout rows v as LDS columns: an observed
// state is its column, a missing one column KP (the row sums), and the
// caller's ambiguity set a is KP + 1 + a (text after Eq. 4: tips are 0/1
// indicators of the possible states).
template <int NT, typename T>
__device__ inline void tip_columns(int (&col)[4], const uint8_t* __restrict__ tipst, int P, int p0, int K, int g) {
  EPOCH_DIMS(NT);
#pragma unroll
  for (int v = 0; v < 4; ++v) {
    const int st = gptr(tipst)[min(p0 + drow<T>(g, v), P - 1)];
    col[v] = st < K ? st : KP + (st - K);
  }
}
// Sum of row entries over an ambiguity set (rare: kept off the common path).
template <typename T>
__device__ __noinline__ T masked_row_sum(const T* __restrict__ row, uint64_t set) {
  T acc = 0;
  while (set) {
    const int j = __builtin_ctzll(set);
    acc += row[j];
    set &= set - 1;
  }
  return acc;
}
// Tip child: S = P[i][state_p] (or the sum of P[i][.] over the tip's state set).
// AMB: the problem has tips with ambiguity codes (a separate instantiation, so
// the common case keeps its registers).
template <int NT, bool AMB, typename T>
__device__ inline void tip_lookup(v4<T> (&S)[NT], const int (&col)[4], const T* __restrict__ sP, int r,
                                  const uint64_t* __restrict__ amb) {
  EPOCH_DIMS(NT);
#pragma unroll
  for (int nt = 0; nt < NT; ++nt)
#pragma unroll
    for (int v = 0; v < 4; ++v) S[nt][v] = sP[(16 * nt + r) * LDP + (AMB ? min(col[v], KP) : col[v])];
  if (AMB && max(max(col[0], col[1]), max(col[2], col[3])) > KP) {  // an ambiguity set
#pragma unroll
    for (int v = 0; v < 4; ++v)
      if (col[v] > KP)
        for (int nt = 0; nt < NT; ++nt) S[nt][v] = masked_row_sum(sP + (16 * nt + r) * LDP, amb[col[v] - KP - 1]);
  }
}

// D-layout load of a [P][KP] array: value at pattern p0 + drow(g, v), state 16 nt + r.
template <int NT, typename T>
__device__ inline void load_dlayout(v4<T> (&X)[NT], const T* __restrict__ base, int P, int p0, int g, int r) {
  EPOCH_DIMS(NT);
#pragma unroll
  for (int v = 0; v < 4; ++v) {
    const EPOCH_GLOBAL T* row = gptr(base + (size_t)min(p0 + drow<T>(g, v), P - 1) * KP) + r;
#pragma unroll
    for (int nt = 0; nt < NT; ++nt) X[nt][v] = row[16 * nt];
  }
}

__device__ inline float dmax(float a, float b) { return fmaxf(a, b); }
__device__ inline double dmax(double a, double b) { return fmax(a, b); }

// ---------------------------------------------------------------------------
// Root: one thread per pattern, in FP64; block partial sums of w_p log L_p per
// instance (blockIdx.y runs over descriptors; those of categories above 0 have
// nothing to do).  One category: L_p = sum_i pi_i x_root(p, i) 2^E_p.  Several
// (text after Eq. 4, rate categories): each category c has its own scale
// exponent E_c, so L_p = 2^Emax sum_c w_c l_c 2^(E_c - Emax) with
// l_c = sum_i pi_i x_c(p, i); the pre-order pass of category c then weighs
// pattern p by w_p w_c l_c 2^E_c / L_p (its posterior share), written to that
// category's weightsT.
template <typename T, int NT>
__global__ __launch_bounds__(256) void codon_root_kernel(const CodonProblem* __restrict__ probs) {
  EPOCH_DIMS(NT);
  __shared__ double sm[256];
  const CodonProblem& pr = probs[blockIdx.y];
  if (pr.cat_index != 0) return;  // uniform
  const int P = pr.P, K = pr.K;
  if ((int)blockIdx.x * 256 >= P) return;  // uniform
  const int p = blockIdx.x * 256 + threadIdx.x;
  const size_t slot = pr.root - pr.N;
  double contrib = 0.0;
  if (p < P) {
    double s;
    if (pr.n_cats == 1) {
      double L = 0.0;
      const T* x = reinterpret_cast<const T*>(pr.part) + (slot * P + p) * KP;
      for (int i = 0; i < K; ++i) L += pr.pi[i] * (double)x[i];
      s = log(L) + (double)pr.scales[slot * P + p] * kLn2;
    } else {
      double l[kMaxCategories];
      int e[kMaxCategories], emax = INT_MIN;
      for (int c = 0; c < pr.n_cats; ++c) {
        const CodonProblem& pc = probs[blockIdx.y + c];
        const T* x = reinterpret_cast<const T*>(pc.part) + (slot * P + p) * KP;
        double acc = 0.0;
        for (int i = 0; i < K; ++i) acc += pr.pi[i] * (double)x[i];
        l[c] = pr.cat[kMaxCategories + c] * acc;
        e[c] = pc.scales[slot * P + p];
        if (l[c] > 0.0) emax = max(emax, e[c]);
      }
      double L = 0.0;
      for (int c = 0; c < pr.n_cats; ++c) {
        l[c] = l[c] > 0.0 ? ldexp(l[c], e[c] - emax) : 0.0;
        L += l[c];
      }
      s = L > 0.0 ? log(L) + (double)emax * kLn2 : -INFINITY;
      for (int c = 0; c < pr.n_cats; ++c)
        reinterpret_cast<T*>(probs[blockIdx.y + c].weightsT)[p] = L > 0.0 ? (T)(pr.weights[p] * (l[c] / L)) : T(0);
    }
    pr.site[p] = s;
    contrib = pr.weights[p] * s;
  }
  const double tot = block_sum<256>(contrib, sm);
  if (threadIdx.x == 0) pr.blocksum[blockIdx.x] = tot;
}

// Ordered sum of each problem's block partial sums into its result[0].
__global__ __launch_bounds__(256) void codon_final_kernel(const CodonProblem* __restrict__ probs) {
  __shared__ double sm[256];
  const CodonProblem& pr = probs[blockIdx.x];
  if (pr.cat_index != 0) return;  // uniform
  const int nb = (pr.P + 255) / 256;
  double acc = 0.0;
  for (int k = threadIdx.x; k < nb; k += 256) acc += pr.blocksum[k];
  const double tot = block_sum<256>(acc, sm);
  if (threadIdx.x == 0) pr.result[0] = tot;
}

// ---------------------------------------------------------------------------
// Pre-order of one level fused with dlogL/dP of the two child branches.
//
// The block's four wavefronts walk its R tiles of 64 patterns together.  For
// each tile, wavefront w first works on patterns 16 w .. 16 w + 15: child
// vectors, q_u, the weights w_p / L_p, t_a = q o S_b and t_b = q o S_a (kept in
// LDS for the whole block), and the outside vectors of internal children.
// After a barrier, wavefront w accumulates rows 16 w .. 16 w + 15 of both
// children's dlogL/dP over all 64 patterns (A = t from LDS times w_p/L_p,
// B = child partials from L2, or the tip indicator), so each wavefront holds
// only 2 x 16 accumulator registers; the loads of its next tile are issued
// before that second phase and arrive while it runs.
// Rows 16 w .. 16 w + 15 of one child's dlogL/dP over the 64 patterns of a
// block tile (contraction over patterns: k-step ks takes pattern 4 ks + g):
// A = t[p][16 w + r] w_p / L_p, B = the child's partials (internal child) or
// its tip-state indicator.  One loop per kind of child, with no branch inside,
// so the LDS reads of later k-steps are issued ahead of the matrix-core work.
// With 32 states (NT = 2) the four wavefronts split the 2 x 2 tiles of
// dlogL/dP instead: wavefront w takes row tile w % NT and NCT column tiles
// from ct0 = (w / NT) NCT (for 64 states: rows 16 w .. 16 w + 15, every column).
template <int NT, typename T>
__device__ inline void grad_rows_internal(v4<T>* G, const T* __restrict__ tcol, const T* __restrict__ sCF,
                                          const T* __restrict__ sL, int ct0, int g, int r) {
  EPOCH_DIMS(NT);
  constexpr int NCT = Dim<NT>::NCT;
#pragma unroll 8
  for (int ks = 0; ks < TILE / 4; ++ks) {
    const int pl = 4 * ks + g;
    const T av = tcol[pl * LDP] * sCF[pl];
    v4<T> B;
#pragma unroll
    for (int c = 0; c < NCT; ++c) B[c] = sL[pl * LDP + 16 * (ct0 + c) + r];
#pragma unroll
    for (int c = 0; c < NCT; ++c) G[c] = mfma(av, B[c], G[c]);
  }
}
// FP32 tip child without ambiguity codes, on the bf16 matrix cores
// (v_mfma_f32_16x16x32_bf16, 32 patterns per instruction against 4): the B
// operand is the 0/1 tip indicator, which bf16 holds exactly, and the A
// operand t w_p / L_p is split into three bf16 parts h + m + l that add up to
// the FP32 value (each part takes the next 8 significand bits, and the
// remainders are exact in FP32), so the three products accumulated in FP32
// give dlogL/dP to FP32 rounding, as the FP32 product would.  Lane (g, r)
// supplies patterns 8 g .. 8 g + 7 of each 32-pattern block for row r of A
// and column r of B; D has the FP32 layout.
typedef __bf16 bf8 __attribute__((ext_vector_type(8)));
typedef int i4 __attribute__((ext_vector_type(4)));
template <int NT>
__device__ inline void grad_rows_tip_bf16(f4* G, const float* __restrict__ tcol, const float* __restrict__ sCF,
                                          const int* __restrict__ sCol, int K, int ct0, int g, int r) {
  EPOCH_DIMS(NT);
  constexpr int NCT = Dim<NT>::NCT;
#pragma unroll
  for (int kb = 0; kb < TILE / 32; ++kb) {
    const int p0 = 32 * kb + 8 * g;
    const f4 cf0 = *reinterpret_cast<const f4*>(sCF + p0), cf1 = *reinterpret_cast<const f4*>(sCF + p0 + 4);
    const float cf[8] = {cf0.x, cf0.y, cf0.z, cf0.w, cf1.x, cf1.y, cf1.z, cf1.w};
    bf8 ah, am, al;
#pragma unroll
    for (int e = 0; e < 8; ++e) {
      const float av = tcol[(p0 + e) * LDP] * cf[e];
      const __bf16 h = (__bf16)av;
      const float r1 = av - (float)h;
      const __bf16 m = (__bf16)r1;
      ah[e] = h;
      am[e] = m;
      al[e] = (__bf16)(r1 - (float)m);
    }
    const i4 cl0 = *reinterpret_cast<const i4*>(sCol + p0), cl1 = *reinterpret_cast<const i4*>(sCol + p0 + 4);
    const int col[8] = {cl0.x, cl0.y, cl0.z, cl0.w, cl1.x, cl1.y, cl1.z, cl1.w};
#pragma unroll
    for (int c = 0; c < NCT; ++c) {
      const int j = 16 * (ct0 + c) + r;
      bf8 B;
#pragma unroll
      for (int e = 0; e < 8; ++e) B[e] = (col[e] == j || (col[e] == KP && j < K)) ? (__bf16)1.0f : (__bf16)0.0f;
      G[c] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(al, B, G[c], 0, 0, 0);
      G[c] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(am, B, G[c], 0, 0, 0);
      G[c] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(ah, B, G[c], 0, 0, 0);
    }
  }
}

template <int NT, bool AMB, typename T>
__device__ inline void grad_rows_tip(v4<T>* G, const T* __restrict__ tcol, const T* __restrict__ sCF,
                                     const int* __restrict__ sCol, int K, int ct0, int g, int r,
                                     const uint64_t* __restrict__ amb) {
  EPOCH_DIMS(NT);
  constexpr int NCT = Dim<NT>::NCT;
  if constexpr (sizeof(T) == 4 && !AMB && NCT >= 4) {  // the split pays off over four column tiles, not one
    grad_rows_tip_bf16<NT>(G, tcol, sCF, sCol, K, ct0, g, r);
    return;
  }
#pragma unroll 8
  for (int ks = 0; ks < TILE / 4; ++ks) {
    const int pl = 4 * ks + g;
    const T av = tcol[pl * LDP] * sCF[pl];
    const int col = sCol[pl];
    v4<T> B;
#pragma unroll
    for (int c = 0; c < NCT; ++c) {
      const int j = 16 * (ct0 + c) + r;
      B[c] = (col == j || (col == KP && j < K)) ? T(1) : T(0);
    }
    if (AMB && col > KP) {  // the 0/1 row of an ambiguity set
      const uint64_t set = amb[col - KP - 1];
#pragma unroll
      for (int c = 0; c < NCT; ++c) B[c] = ((set >> (16 * (ct0 + c) + r)) & 1) ? T(1) : T(0);
    }
#pragma unroll
    for (int c = 0; c < NCT; ++c) G[c] = mfma(av, B[c], G[c]);
  }
}

// A block past the last tile of a pattern chunk shorter than the one the
// schedule was built for still owns a dlogL/dP slot of each child branch (the
// slot count covers the longest chunk): it writes zeros there.  Blocks past a
// batch member's own tiles own no slot and write nothing.
template <typename T, int NT>
__device__ inline void zero_unused_slot(const CodonProblem& pr, int child, int nthreads) {
  EPOCH_DIMS(NT);
  if ((int)blockIdx.x >= pr.gslots[child]) return;
  EPOCH_GLOBAL T* dst = gptr(reinterpret_cast<T*>(pr.Gpart) + ((size_t)pr.gslots[pr.n_nodes + child] + blockIdx.x) * KK);
  for (int e = threadIdx.x; e < KK / 4; e += nthreads) reinterpret_cast<EPOCH_GLOBAL v4<T>*>(dst)[e] = v4<T>{0, 0, 0, 0};
}

template <typename T, int NT>
struct PreTileLoads {
  v4<T> La[NT], Lb[NT];  // rows of 4 states of internal children's partials (child product A operand)
  v4<T> Q[NT];           // q_u in the D layout
  int cola[4], colb[4];
};

template <int NT, typename T>
__device__ inline void pre_load_tile(PreTileLoads<T, NT>& ld, const CodonProblem& pr, const T* La, const T* Lb,
                                     const T* Qu, int a, int b, int p0, int g, int r) {
  EPOCH_DIMS(NT);
  const int P = pr.P, K = pr.K, N = pr.N;
  const int pa = min(p0 + r, P - 1);
  if (La) {
    const EPOCH_GLOBAL v4<T>* row = gptr(reinterpret_cast<const v4<T>*>(La + (size_t)pa * KP)) + g;
#pragma unroll
    for (int t = 0; t < NT; ++t) ld.La[t] = row[4 * t];
  } else {
    tip_columns<NT, T>(ld.cola, pr.tips + (size_t)a * pr.tip_stride, P, p0, K, g);
  }
  if (Lb) {
    const EPOCH_GLOBAL v4<T>* row = gptr(reinterpret_cast<const v4<T>*>(Lb + (size_t)pa * KP)) + g;
#pragma unroll
    for (int t = 0; t < NT; ++t) ld.Lb[t] = row[4 * t];
  } else {
    tip_columns<NT, T>(ld.colb, pr.tips + (size_t)b * pr.tip_stride, P, p0, K, g);
  }
  if (Qu) load_dlayout<NT, T>(ld.Q, Qu, P, p0, g, r);
  (void)N;
}

// S[nt] (D layout) from 16-byte A-operand rows already in registers.
template <int NT, typename T>
__device__ inline void child_gemm_regs(v4<T> (&S)[NT], const v4<T> (&a)[NT], const T* __restrict__ sP, int g, int r) {
  EPOCH_DIMS(NT);
#pragma unroll
  for (int nt = 0; nt < NT; ++nt) S[nt] = v4<T>{0, 0, 0, 0};
#pragma unroll
  for (int t = 0; t < NT; ++t)
#pragma unroll
    for (int nt = 0; nt < NT; ++nt) {
      const v4<T> bv = *reinterpret_cast<const v4<T>*>(sP + (16 * nt + r) * LDP + 16 * t + 4 * g);
      S[nt] = mfma(a[t].x, bv.x, S[nt]);
      S[nt] = mfma(a[t].y, bv.y, S[nt]);
      S[nt] = mfma(a[t].z, bv.z, S[nt]);
      S[nt] = mfma(a[t].w, bv.w, S[nt]);
    }
}

// ---------------------------------------------------------------------------
template <typename T, int NT, bool AMB>
__global__ __launch_bounds__(256) void codon_post_level_kernel(const CodonProblem* __restrict__ probs,
                                                                const int2* __restrict__ items, int R) {
  EPOCH_DIMS(NT);
  __shared__ __align__(16) T sPa[KP * LDP];
  __shared__ __align__(16) T sPb[KP * LDP];
  const int2 it = items[blockIdx.y];
  const CodonProblem& pr = probs[it.x];
  const int N = pr.N, P = pr.P, K = pr.K;
  const int base = blockIdx.x * R * TILE;
  if (base >= P) return;  // uniform: this problem has fewer tiles
  const int end = min(P, base + R * TILE);
  const int u = it.y;
  const int a = pr.left[u], b = pr.right[u];
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6, g = lane >> 4, r = lane & 15;
  T* part = reinterpret_cast<T*>(pr.part);
  const T* La = a >= N ? part + (size_t)(a - N) * P * KP : nullptr;
  const T* Lb = b >= N ? part + (size_t)(b - N) * P * KP : nullptr;
  const int32_t* sca = a >= N ? pr.scales + (size_t)(a - N) * P : nullptr;
  const int32_t* scb = b >= N ? pr.scales + (size_t)(b - N) * P : nullptr;
  EPOCH_GLOBAL T* out = gptr(part + (size_t)(u - N) * P * KP);
  EPOCH_GLOBAL int32_t* sout = gptr(pr.scales + (size_t)(u - N) * P);
  // child rows (or tip columns) and the children's scale exponents of a tile: the first tile's loads
  // go out before the matrices are staged, so the two memory round trips overlap; each later tile's
  // at the end of the tile before it
  auto load = [&](PreTileLoads<T, NT>& ld, int (&csc)[4], int p0) {
    pre_load_tile<NT, T>(ld, pr, La, Lb, nullptr, a, b, p0, g, r);
#pragma unroll
    for (int v = 0; v < 4; ++v) {
      const int pc = min(p0 + drow<T>(g, v), P - 1);
      csc[v] = (sca ? gptr(sca)[pc] : 0) + (scb ? gptr(scb)[pc] : 0);
    }
  };
  PreTileLoads<T, NT> cur;
  int csc[4];
  load(cur, csc, base + WT * w);
  const T* Pm = reinterpret_cast<const T*>(pr.Pm);
  stage_matrix<NT>(sPa, Pm + (size_t)a * pr.pm_stride);
  stage_matrix<NT>(sPb, Pm + (size_t)b * pr.pm_stride);
  __syncthreads();
  stage_row_sums<NT>(sPa, K);
  stage_row_sums<NT>(sPb, K);
  __syncthreads();
  for (int p0 = base + WT * w; p0 < end; p0 += 4 * WT) {
    v4<T> Sa[NT], Sb[NT];
    if (La)
      child_gemm_regs<NT, T>(Sa, cur.La, sPa, g, r);
    else
      tip_lookup<NT, AMB, T>(Sa, cur.cola, sPa, r, pr.amb);
    if (Lb)
      child_gemm_regs<NT, T>(Sb, cur.Lb, sPb, g, r);
    else
      tip_lookup<NT, AMB, T>(Sb, cur.colb, sPb, r, pr.amb);
    int e[4];
#pragma unroll
    for (int v = 0; v < 4; ++v) {
      T m = 0;
#pragma unroll
      for (int nt = 0; nt < NT; ++nt) {
        Sa[nt][v] *= Sb[nt][v];
        m = dmax(m, Sa[nt][v]);
      }
      e[v] = scale_exponent(row16_max(m));
    }
#pragma unroll
    for (int v = 0; v < 4; ++v) {
      const int p = p0 + drow<T>(g, v);
      if (p < P) {
#pragma unroll
        for (int nt = 0; nt < NT; ++nt) __builtin_nontemporal_store(scale_by_pow2(Sa[nt][v], e[v]), &out[(size_t)p * KP + 16 * nt + r]);
        if (r == 0) sout[p] = e[v] + csc[v];
      }
    }
    if (p0 + 4 * WT < end) load(cur, csc, p0 + 4 * WT);
  }
}


template <typename T, int NT, bool AMB>
__global__ __launch_bounds__(256, sizeof(T) == 4 ? 2 : 1) void codon_pre_level_kernel(
    const CodonProblem* __restrict__ probs, const int2* __restrict__ items, int R) {
  EPOCH_DIMS(NT);
  constexpr int NCT = Dim<NT>::NCT;
  __shared__ __align__(16) T sPa[KP * LDP];
  __shared__ __align__(16) T sPb[KP * LDP];
  __shared__ __align__(16) T sT[TILE * LDP];  // t of one side for the block tile, pattern-major
  __shared__ __align__(16) T sL[TILE * LDP];  // that side's child partials for the block tile
  __shared__ __align__(16) T sCF[TILE];         // w_p / L_p of the block tile
  __shared__ __align__(16) int sCol[2][TILE];   // tip columns of the block tile
  const int2 it = items[blockIdx.y];
  const CodonProblem& pr = probs[it.x];
  const int N = pr.N, P = pr.P, K = pr.K;
  const int base = blockIdx.x * R * TILE;
  const int u = it.y;
  const int a = pr.left[u], b = pr.right[u];
  if (base >= P) {  // uniform: this problem (or pattern chunk) has fewer tiles
    zero_unused_slot<T, NT>(pr, a, 256);
    zero_unused_slot<T, NT>(pr, b, 256);
    return;
  }
  const int n_tiles = min(R, (P - base + TILE - 1) / TILE);  // uniform over the block
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6, g = lane >> 4, r = lane & 15;
  const T* part = reinterpret_cast<const T*>(pr.part);
  T* pre = reinterpret_cast<T*>(pr.pre);
  const T* La = a >= N ? part + (size_t)(a - N) * P * KP : nullptr;
  const T* Lb = b >= N ? part + (size_t)(b - N) * P * KP : nullptr;
  const T* Qu = u == pr.root ? nullptr : pre + (size_t)(u - N) * P * KP;
  // the first tile's loads go out before the matrices are staged, so the two wait together
  PreTileLoads<T, NT> cur, nxt;
  pre_load_tile<NT, T>(cur, pr, La, Lb, Qu, a, b, base + WT * w, g, r);
  const T* Pm = reinterpret_cast<const T*>(pr.Pm);
  stage_matrix<NT>(sPa, Pm + (size_t)a * pr.pm_stride);
  stage_matrix<NT>(sPb, Pm + (size_t)b * pr.pm_stride);
  __syncthreads();
  stage_row_sums<NT>(sPa, K);
  stage_row_sums<NT>(sPb, K);
  __syncthreads();
  T piv[NT];
#pragma unroll
  for (int nt = 0; nt < NT; ++nt) piv[nt] = 16 * nt + r < K ? (T)pr.pi[16 * nt + r] : T(0);
  // dlogL/dP accumulators: rows 16 rt + drow(g, v), columns 16 (ct0 + c) + r
  const int rt = w % NT, ct0 = (w / NT) * NCT;
  v4<T> Ga[NCT], Gb[NCT];
#pragma unroll
  for (int c = 0; c < NCT; ++c) {
    Ga[c] = v4<T>{0, 0, 0, 0};
    Gb[c] = v4<T>{0, 0, 0, 0};
  }
  T* trows = sT + (WT * w) * LDP;  // this wavefront's 16 pattern rows
  T* lrows = sL + (WT * w) * LDP;
  for (int bt = 0; bt < n_tiles; ++bt) {
    const int p0 = base + bt * TILE + WT * w;  // first pattern of this wavefront's part
    T wts[4];  // pattern weights of this wavefront's rows, in flight during the child products
#pragma unroll
    for (int v = 0; v < 4; ++v) wts[v] = gptr(reinterpret_cast<const T*>(pr.weightsT))[min(p0 + drow<T>(g, v), P - 1)];
    // ---- this wavefront's 16 patterns: child vectors, q_u, w_p / L_p
    v4<T> Sa[NT], Sb[NT];
    if (La)
      child_gemm_regs<NT, T>(Sa, cur.La, sPa, g, r);
    else
      tip_lookup<NT, AMB, T>(Sa, cur.cola, sPa, r, pr.amb);
    if (Lb)
      child_gemm_regs<NT, T>(Sb, cur.Lb, sPb, g, r);
    else
      tip_lookup<NT, AMB, T>(Sb, cur.colb, sPb, r, pr.amb);
    v4<T> Q[NT];
#pragma unroll
    for (int nt = 0; nt < NT; ++nt) Q[nt] = Qu ? cur.Q[nt] : v4<T>{piv[nt], piv[nt], piv[nt], piv[nt]};
#pragma unroll
    for (int v = 0; v < 4; ++v) {
      T sum = 0;
#pragma unroll
      for (int nt = 0; nt < NT; ++nt) sum += Q[nt][v] * Sa[nt][v] * Sb[nt][v];
      sum = row16_sum(sum);
      const int p = p0 + drow<T>(g, v);
      if (r == 0) {
        sCF[WT * w + drow<T>(g, v)] = (p < P && sum > T(0)) ? wts[v] / sum : T(0);
        if (!La) sCol[0][WT * w + drow<T>(g, v)] = cur.cola[v];
        if (!Lb) sCol[1][WT * w + drow<T>(g, v)] = cur.colb[v];
      }
    }
    // loads of this wavefront's part of the next tile, in flight during the rest
    if (bt + 1 < n_tiles) pre_load_tile<NT, T>(nxt, pr, La, Lb, Qu, a, b, p0 + TILE, g, r);
#pragma unroll
    for (int side = 0; side < 2; ++side) {
      const int child = side == 0 ? a : b;
      const T* Lc = side == 0 ? La : Lb;
      const v4<T>* So = side == 0 ? Sb : Sa;  // [NT]
      v4<T>* G = side == 0 ? Ga : Gb;
      const T* sP = side == 0 ? sPa : sPb;
      if (side == 1) __syncthreads();  // every wavefront is done with side a's t and L
      // t = q o S_sibling rows, and the child's partial rows, into LDS
#pragma unroll
      for (int nt = 0; nt < NT; ++nt)
#pragma unroll
        for (int v = 0; v < 4; ++v) trows[drow<T>(g, v) * LDP + 16 * nt + r] = Q[nt][v] * So[nt][v];
      if (Lc) {
        const v4<T>* lr = side == 0 ? cur.La : cur.Lb;
#pragma unroll
        for (int t = 0; t < NT; ++t) *reinterpret_cast<v4<T>*>(lrows + r * LDP + 16 * t + 4 * g) = lr[t];
      }
      wave_lds_sync();
      if (Lc) {
        // outside vector q_c[p][j] = sum_i t[p][i] P_c[i][j] of this wavefront's patterns
        v4<T> ta[NT];
#pragma unroll
        for (int tt = 0; tt < NT; ++tt) ta[tt] = *reinterpret_cast<const v4<T>*>(trows + r * LDP + 16 * tt + 4 * g);
        v4<T> Qo[NT];
#pragma unroll
        for (int nt = 0; nt < NT; ++nt) Qo[nt] = v4<T>{0, 0, 0, 0};
#pragma unroll
        for (int tt = 0; tt < NT; ++tt)
#pragma unroll
          for (int nt = 0; nt < NT; ++nt) {
            const T* prow = sP + (16 * tt + 4 * g) * LDP + 16 * nt + r;
            Qo[nt] = mfma(ta[tt].x, prow[0], Qo[nt]);
            Qo[nt] = mfma(ta[tt].y, prow[LDP], Qo[nt]);
            Qo[nt] = mfma(ta[tt].z, prow[2 * LDP], Qo[nt]);
            Qo[nt] = mfma(ta[tt].w, prow[3 * LDP], Qo[nt]);
          }
        EPOCH_GLOBAL T* out = gptr(pre + (size_t)(child - N) * P * KP);
#pragma unroll
        for (int v = 0; v < 4; ++v) {
          T m = 0;
#pragma unroll
          for (int nt = 0; nt < NT; ++nt) m = dmax(m, Qo[nt][v]);
          const int e = scale_exponent(row16_max(m));
          const int p = p0 + drow<T>(g, v);
          if (p < P)
#pragma unroll
            for (int nt = 0; nt < NT; ++nt) __builtin_nontemporal_store(scale_by_pow2(Qo[nt][v], e), &out[(size_t)p * KP + 16 * nt + r]);
        }
      }
      __syncthreads();  // t, L, w_p / L_p and tip columns of every wavefront are in LDS
      // this wavefront's tiles of dlogL/dP over the 64 patterns of the tile
      const T* tcol = sT + 16 * rt + r;  // column i = 16 rt + r of t
      if (Lc)
        grad_rows_internal<NT, T>(G, tcol, sCF, sL, ct0, g, r);
      else
        grad_rows_tip<NT, AMB, T>(G, tcol, sCF, sCol[side], K, ct0, g, r, pr.amb);
    }
    __syncthreads();  // the next tile overwrites t, L, w_p / L_p and tip columns
    if (bt + 1 < n_tiles) cur = nxt;
  }
  // this wavefront's rows of the block's slot of each child branch
#pragma unroll
  for (int side = 0; side < 2; ++side) {
    const int child = side == 0 ? a : b;
    const v4<T>* G = side == 0 ? Ga : Gb;
    EPOCH_GLOBAL T* dst = gptr(reinterpret_cast<T*>(pr.Gpart) + ((size_t)pr.gslots[pr.n_nodes + child] + blockIdx.x) * KK);
#pragma unroll
    for (int c = 0; c < NCT; ++c)
#pragma unroll
      for (int v = 0; v < 4; ++v)
        __builtin_nontemporal_store(G[c][v], &dst[(16 * rt + drow<T>(g, v)) * KP + 16 * (ct0 + c) + r]);
  }
}

// The same step with the two child branches on separate wavefronts, for
// levels too narrow to fill the GPU.  Eight wavefronts per block: wavefront
// 4 s + w takes side s (0: left child, 1: right child) of patterns 16 w ..
// 16 w + 15 of each 64-pattern tile.  The child vectors are swapped through
// LDS, so each wavefront runs one child product, one outside-vector product
// and its side's dlogL/dP rows per tile, half the serial work of the kernel
// above.  Tiles, slots and the order of every sum are those of the kernel
// above, so both give the same bits.
struct PreSplitShared {
  __align__(16) float sP[2][KP * LDP];    // P_left, P_right with row sums
  __align__(16) float sS[2][TILE * LDP];  // each side's child vectors for the block tile
  __align__(16) float sT[2][TILE * LDP];  // each side's t = q o S_sibling
  __align__(16) float sL[2][TILE * LDP];  // each side's child partials
  __align__(16) float sCF[TILE];
  __align__(16) int sCol[2][TILE];
};

struct SplitTileLoads {
  f4 L[4];  // 16-byte rows of this side's child partials (internal child)
  f4 Q[4];  // q_u in the D layout
  int col[4];
};

__device__ inline void split_load_tile(SplitTileLoads& ld, const CodonProblem& pr, const float* Lc, const float* Qu,
                                       int c, int p0, int g, int r) {
  const int P = pr.P;
  if (Lc) {
    const EPOCH_GLOBAL f4* row = gptr(reinterpret_cast<const f4*>(Lc + (size_t)min(p0 + r, P - 1) * KP)) + g;
#pragma unroll
    for (int t = 0; t < 4; ++t) ld.L[t] = row[4 * t];
  } else {
    tip_columns<4, float>(ld.col, pr.tips + (size_t)c * pr.tip_stride, P, p0, pr.K, g);
  }
  if (Qu) load_dlayout<4, float>(ld.Q, Qu, P, p0, g, r);
}

template <bool AMB>
__global__ __launch_bounds__(512, 1) void codon_pre_split_kernel(const CodonProblem* __restrict__ probs,
                                                                const int2* __restrict__ items, int R) {
  __shared__ PreSplitShared sh;
  const int2 it = items[blockIdx.y];
  const CodonProblem& pr = probs[it.x];
  const int N = pr.N, P = pr.P, K = pr.K;
  const int base = blockIdx.x * R * TILE;
  const int u = it.y;
  const int a = pr.left[u], b = pr.right[u];
  if (base >= P) {  // uniform: this problem (or pattern chunk) has fewer tiles
    zero_unused_slot<float, 4>(pr, a, 512);
    zero_unused_slot<float, 4>(pr, b, 512);
    return;
  }
  const int n_tiles = min(R, (P - base + TILE - 1) / TILE);  // uniform over the block
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6, w = wave & 3, s = wave >> 2;
  const int g = lane >> 4, r = lane & 15;
  const int c = s ? b : a;
  {  // threads 0..255 stage P_left, 256..511 P_right
    const int h = threadIdx.x >> 8;
    stage_matrix<4>(sh.sP[h], pr.Pm + (size_t)(h ? b : a) * pr.pm_stride, threadIdx.x & 255);
    __syncthreads();
    stage_row_sums<4>(sh.sP[h], K, threadIdx.x & 255);
    __syncthreads();
  }
  const float* sPc = sh.sP[s];
  const float* Lc = c >= N ? pr.part + (size_t)(c - N) * P * KP : nullptr;
  const float* Qu = u == pr.root ? nullptr : pr.pre + (size_t)(u - N) * P * KP;
  float piv[4];
#pragma unroll
  for (int nt = 0; nt < 4; ++nt) piv[nt] = 16 * nt + r < K ? (float)pr.pi[16 * nt + r] : 0.f;
  f4 G[4];
#pragma unroll
  for (int nt = 0; nt < 4; ++nt) G[nt] = f4{0.f, 0.f, 0.f, 0.f};
  SplitTileLoads cur, nxt;
  split_load_tile(cur, pr, Lc, Qu, c, base + WT * w, g, r);
  float* srows = sh.sS[s] + (WT * w) * LDP;
  const float* sibrows = sh.sS[1 - s] + (WT * w) * LDP;
  float* trows = sh.sT[s] + (WT * w) * LDP;
  float* lrows = sh.sL[s] + (WT * w) * LDP;
  for (int bt = 0; bt < n_tiles; ++bt) {
    const int p0 = base + bt * TILE + WT * w;
    f4 S[4];
    if (Lc)
      child_gemm_regs<4, float>(S, cur.L, sPc, g, r);
    else
      tip_lookup<4, AMB, float>(S, cur.col, sPc, r, pr.amb);
#pragma unroll
    for (int nt = 0; nt < 4; ++nt)
#pragma unroll
      for (int v = 0; v < 4; ++v) srows[(4 * g + v) * LDP + 16 * nt + r] = S[nt][v];
    // the other side's child vectors of the same patterns are in LDS after this
    // barrier; every wavefront has also finished the previous tile's dlogL/dP
    __syncthreads();
    f4 So[4], Q[4];
#pragma unroll
    for (int nt = 0; nt < 4; ++nt) {
#pragma unroll
      for (int v = 0; v < 4; ++v) So[nt][v] = sibrows[(4 * g + v) * LDP + 16 * nt + r];
      Q[nt] = Qu ? cur.Q[nt] : f4{piv[nt], piv[nt], piv[nt], piv[nt]};
    }
#pragma unroll
    for (int v = 0; v < 4; ++v) {
      if (s == 0) {  // uniform; S is the left child's vector, So the right child's
        float sum = 0.f;
#pragma unroll
        for (int nt = 0; nt < 4; ++nt) sum += Q[nt][v] * S[nt][v] * So[nt][v];
        sum = row16_sum(sum);
        const int p = p0 + 4 * g + v;
        if (r == 0) sh.sCF[WT * w + 4 * g + v] = (p < P && sum > 0.f) ? gptr(pr.weightsT)[p] / sum : 0.f;
      }
      if (r == 0 && !Lc) sh.sCol[s][WT * w + 4 * g + v] = cur.col[v];
    }
    if (bt + 1 < n_tiles) split_load_tile(nxt, pr, Lc, Qu, c, p0 + TILE, g, r);
#pragma unroll
    for (int nt = 0; nt < 4; ++nt)
#pragma unroll
      for (int v = 0; v < 4; ++v) trows[(4 * g + v) * LDP + 16 * nt + r] = Q[nt][v] * So[nt][v];
    if (Lc) {
#pragma unroll
      for (int t = 0; t < 4; ++t) *reinterpret_cast<f4*>(lrows + r * LDP + 16 * t + 4 * g) = cur.L[t];
    }
    wave_lds_sync();
    if (Lc) {
      f4 ta[4];
#pragma unroll
      for (int tt = 0; tt < 4; ++tt) ta[tt] = *reinterpret_cast<const f4*>(trows + r * LDP + 16 * tt + 4 * g);
      f4 Qo[4];
#pragma unroll
      for (int nt = 0; nt < 4; ++nt) Qo[nt] = f4{0.f, 0.f, 0.f, 0.f};
#pragma unroll
      for (int tt = 0; tt < 4; ++tt)
#pragma unroll
        for (int nt = 0; nt < 4; ++nt) {
          const float* prow = sPc + (16 * tt + 4 * g) * LDP + 16 * nt + r;
          Qo[nt] = mfma(ta[tt].x, prow[0], Qo[nt]);
          Qo[nt] = mfma(ta[tt].y, prow[LDP], Qo[nt]);
          Qo[nt] = mfma(ta[tt].z, prow[2 * LDP], Qo[nt]);
          Qo[nt] = mfma(ta[tt].w, prow[3 * LDP], Qo[nt]);
        }
      EPOCH_GLOBAL float* out = gptr(pr.pre + (size_t)(c - N) * P * KP);
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        float m = 0.f;
#pragma unroll
        for (int nt = 0; nt < 4; ++nt) m = fmaxf(m, Qo[nt][v]);
        const int e = scale_exponent(row16_max(m));
        const int p = p0 + 4 * g + v;
        if (p < P)
#pragma unroll
          for (int nt = 0; nt < 4; ++nt) __builtin_nontemporal_store(ldexpf(Qo[nt][v], -e), &out[(size_t)p * KP + 16 * nt + r]);
      }
    }
    __syncthreads();  // t, L, w_p / L_p and tip columns of the whole tile are in LDS
    const float* tcol = sh.sT[s] + WT * w + r;
    if (Lc)
      grad_rows_internal<4, float>(G, tcol, sh.sCF, sh.sL[s], 0, g, r);
    else
      grad_rows_tip<4, AMB, float>(G, tcol, sh.sCF, sh.sCol[s], K, 0, g, r, pr.amb);
    if (bt + 1 < n_tiles) cur = nxt;
  }
  EPOCH_GLOBAL float* dst = gptr(pr.Gpart + ((size_t)pr.gslots[pr.n_nodes + c] + blockIdx.x) * KK);
#pragma unroll
  for (int nt = 0; nt < 4; ++nt)
#pragma unroll
    for (int v = 0; v < 4; ++v) __builtin_nontemporal_store(G[nt][v], &dst[(WT * w + 4 * g + v) * KP + 16 * nt + r]);
}

// G[v] = sum of the FP32 slot partials in FP64 (fixed order): one block per
// (branch, 256 entries); also the block's share of <G, dP/dl>.
template <int NT>
constexpr int reduce_chunks() {
  return Dim<NT>::KK / 256;
}
template <typename T, int NT>
__global__ __launch_bounds__(256) void codon_grad_reduce_kernel(const CodonProblem* __restrict__ probs,
                                                                const int2* __restrict__ items,
                                                                double* __restrict__ dpart, int accumulate) {
  EPOCH_DIMS(NT);
  constexpr int kReduceChunks = reduce_chunks<NT>();
  __shared__ double sm[256];
  const int2 it = items[blockIdx.x / kReduceChunks];
  const int chunk = blockIdx.x % kReduceChunks;
  const CodonProblem& pr = probs[it.x];
  const int v = it.y;
  const int ns = v == pr.root ? 0 : pr.gslots[v];
  const int e = chunk * 256 + threadIdx.x;
  const EPOCH_GLOBAL T* src =
      gptr(reinterpret_cast<const T*>(pr.Gpart) + (size_t)(v == pr.root ? 0 : pr.gslots[pr.n_nodes + v]) * KK) + e;
  double s0 = 0.0, s1 = 0.0, s2 = 0.0, s3 = 0.0;
  int k = 0;
  for (; k + 4 <= ns; k += 4) {
    s0 += (double)src[(size_t)k * KK];
    s1 += (double)src[(size_t)(k + 1) * KK];
    s2 += (double)src[(size_t)(k + 2) * KK];
    s3 += (double)src[(size_t)(k + 3) * KK];
  }
  for (; k < ns; ++k) s0 += (double)src[(size_t)k * KK];
  double s = (s0 + s1) + (s2 + s3);
  if (accumulate) s += pr.G[(size_t)v * pr.pm_stride + e];  // earlier pattern chunks
  pr.G[(size_t)v * pr.pm_stride + e] = s;
  const double d = block_sum<256>(s * (double)reinterpret_cast<const T*>(pr.dPm)[(size_t)v * pr.pm_stride + e], sm);
  if (threadIdx.x == 0) dpart[blockIdx.x] = d;
}

// dlogL/dl of each branch from the chunk shares, in a fixed order: the sum over
// rate categories of <G_c, dP_c/dl> (the reduce items of an instance's
// categories are consecutive runs of n_nodes, category 0 first).
template <int NT>
__global__ __launch_bounds__(256) void codon_dbranch_kernel(const CodonProblem* __restrict__ probs,
                                                            const int2* __restrict__ items, int n_items,
                                                            const double* __restrict__ dpart) {
  constexpr int kReduceChunks = reduce_chunks<NT>();
  const int i = blockIdx.x * 256 + threadIdx.x;
  if (i >= n_items) return;
  const int2 it = items[i];
  const CodonProblem& pr = probs[it.x];
  if (pr.cat_index != 0) return;
  double d = 0.0;
  for (int c = 0; c < pr.n_cats; ++c)
    for (int k = 0; k < kReduceChunks; ++k) d += dpart[((size_t)i + (size_t)c * pr.n_nodes) * kReduceChunks + k];
  pr.dbranch[it.y] = it.y == pr.root ? 0.0 : d;
}

// Patterns the buffers and the launch schedule of an instance are sized for:
// all of them, or one chunk under an HBM budget.
int codon_chunk_patterns(const EpochInstance* in) { return in->codon_pc > 0 ? in->codon_pc : in->P; }

int codon_tiles_per_block(int tiles, int n_items, int target_blocks, int r_max) {
  const long per_item = ((long)target_blocks + n_items - 1) / n_items;
  long R = (tiles + per_item - 1) / per_item;
  if (R < 1) R = 1;
  if (R > r_max) R = r_max;
  return (int)R;
}

}  // namespace

// The descriptor of rate category c of an instance: its transition matrices,
// dP/dl and G are every C-th 64 x 64 block ([node][category]); its partials,
// outside vectors, scale exponents and weights are the c-th of C equal regions.
CodonProblem codon_descriptor(const EpochInstance* in, int c, const int32_t* gslots, float* gpart) {
  const size_t C = in->C, Nm1 = in->N - 1, P = in->P;
  // element offsets in the instance's compute type (the descriptor's float pointers
  // hold doubles in an FP64 instance)
  auto at = [&](void* base, size_t elems) -> float* {
    return base ? reinterpret_cast<float*>(static_cast<char*>(base) + elems * in->real_size) : nullptr;
  };
  CodonProblem d{};
  const size_t Kp = in->Kp, KKp = Kp * Kp;  // 64 or 32 padded states
  d.Pm = at(in->Pm.ptr, c * KKp);
  d.tips = static_cast<const uint8_t*>(in->tips.ptr);
  d.part = at(in->partials.ptr, c * Nm1 * P * Kp);
  d.pre = at(in->pre.ptr, c * Nm1 * P * Kp);
  d.scales = static_cast<int32_t*>(in->scales.ptr) + c * Nm1 * P;
  d.weightsT = at(in->weightsT.ptr, c * P);
  d.weights = static_cast<const double*>(in->weights.ptr);
  d.pi = static_cast<const double*>(in->pi.ptr);
  d.cat = static_cast<const double*>(in->cat.ptr);
  d.Gpart = gpart;
  d.dPm = at(in->dPm.ptr, c * KKp);
  d.G = in->G.ptr ? static_cast<double*>(in->G.ptr) + c * KKp : nullptr;
  d.dbranch = static_cast<double*>(in->dbranch.ptr);
  d.site = static_cast<double*>(in->site.ptr);
  d.blocksum = static_cast<double*>(in->blocksum.ptr);
  d.result = static_cast<double*>(in->result.ptr);
  d.left = in->d_left;
  d.right = in->d_right;
  d.amb = static_cast<const uint64_t*>(in->amb.ptr);
  d.gslots = gslots;
  d.N = in->N;
  d.P = in->P;
  d.tip_stride = in->P;
  d.K = in->K;
  d.root = in->plan.root;
  d.n_nodes = in->n_nodes;
  d.pm_stride = (int)(C * KKp);
  d.cat_index = c;
  d.n_cats = (int)C;
  return d;
}

// Merged level schedule over one or more problems (levels counted from the
// tips).  Each instance contributes one problem per rate category (its
// descriptors, consecutive, category 0 first: desc_inst / desc_cat).  Each
// level gets R 64-pattern tiles per block, with R chosen so that the level's
// launch has about target_blocks blocks; every block of a node writes one
// dlogL/dP slot for each of the node's two child branches.  gslots[q] holds,
// per node, the number of slots of its branch and then the index of its first
// slot in problem q's slot array.
void codon_build_schedule(const std::vector<const EpochInstance*>& insts, int target_blocks, CodonSchedule& out,
                          std::vector<std::vector<int32_t>>& gslots) {
  out.items.clear();
  out.level_off.assign(1, 0);
  out.level_R.clear();
  out.reduce_items.clear();
  out.desc_inst.clear();
  out.desc_cat.clear();
  for (size_t i = 0; i < insts.size(); ++i)
    for (int c = 0; c < insts[i]->C; ++c) {
      out.desc_inst.push_back((int)i);
      out.desc_cat.push_back(c);
    }
  const size_t nd = out.desc_inst.size();
  auto inst = [&](size_t q) { return insts[out.desc_inst[q]]; };
  int n_levels = 0, max_tiles = 0, max_pblocks = 0;
  for (auto* in : insts) {
    n_levels = std::max(n_levels, in->plan.n_levels);
    max_tiles = std::max(max_tiles, (codon_chunk_patterns(in) + TILE - 1) / TILE);
    max_pblocks = std::max(max_pblocks, (codon_chunk_patterns(in) + 255) / 256);
  }
  gslots.assign(nd, {});
  out.slot_total.assign(nd, 0);
  for (size_t q = 0; q < nd; ++q) gslots[q].assign(2 * (size_t)inst(q)->n_nodes, 0);
  for (int l = 1; l <= n_levels; ++l) {
    const size_t begin = out.items.size();
    for (size_t q = 0; q < nd; ++q) {
      const auto& pl = inst(q)->plan;
      if (l > pl.n_levels) continue;
      for (int k = pl.level_offset[l]; k < pl.level_offset[l + 1]; ++k) out.items.push_back(make_int2((int)q, pl.level_nodes[k]));
    }
    const int n_items = (int)(out.items.size() - begin);
    const int R = codon_tiles_per_block(max_tiles, std::max(1, n_items), target_blocks, max_tiles);
    out.level_off.push_back((int)out.items.size());
    out.level_R.push_back(R);
    for (size_t k = begin; k < out.items.size(); ++k) {
      const int q = out.items[k].x, u = out.items[k].y;
      const auto& pl = inst(q)->plan;
      const int tiles = (codon_chunk_patterns(inst(q)) + TILE - 1) / TILE;
      const int used = (tiles + R - 1) / R;
      const int n = inst(q)->n_nodes;
      for (int child : {pl.left[u], pl.right[u]}) {
        gslots[q][child] = used;
        gslots[q][n + child] = (int32_t)out.slot_total[q];
        out.slot_total[q] += used;
      }
    }
  }
  for (size_t q = 0; q < nd; ++q)
    for (int v = 0; v < inst(q)->n_nodes; ++v) out.reduce_items.push_back(make_int2((int)q, v));
  out.amb = false;
  for (auto* in : insts) out.amb = out.amb || in->tips_amb;
  out.fp64 = !insts.empty() && insts[0]->fp64;
  out.nt = !insts.empty() && insts[0]->Kp == 32 ? 2 : 4;
  out.n_levels = n_levels;
  out.max_tiles = max_tiles;
  out.max_pattern_blocks = max_pblocks;
  out.n_problems = (int)nd;
}

namespace {
template <typename T, int NT>
void post_levels(const CodonSchedule& sc, const CodonProblem* d_probs, const int2* d_items, hipStream_t st) {
  for (int l = 1; l <= sc.n_levels; ++l) {
    const int b = sc.level_off[l - 1], n = sc.level_off[l] - b;
    if (!n) continue;
    const int R = sc.level_R[l - 1];
    const int blocks = (sc.max_tiles + R - 1) / R;
    if (sc.amb)
      hipLaunchKernelGGL((codon_post_level_kernel<T, NT, true>), dim3(blocks, n), dim3(256), 0, st, d_probs, d_items + b,
                         R);
    else
      hipLaunchKernelGGL((codon_post_level_kernel<T, NT, false>), dim3(blocks, n), dim3(256), 0, st, d_probs,
                         d_items + b, R);
  }
}

// 64-state FP32: levels of at most split_blocks blocks on the side-split
// kernel.  FP64 (the split kernel's LDS would not hold doubles) and 32 states:
// the level kernel throughout.
template <typename T, int NT>
void pre_levels(const CodonSchedule& sc, const CodonProblem* d_probs, const int2* d_items, hipStream_t st) {
  for (int l = sc.n_levels; l >= 1; --l) {
    const int b = sc.level_off[l - 1], n = sc.level_off[l] - b;
    if (!n) continue;
    const int R = sc.level_R[l - 1];
    const int blocks = (sc.max_tiles + R - 1) / R;
    if (sizeof(T) == 4 && NT == 4 && (long)blocks * n <= sc.split_blocks) {
      if (sc.amb)
        hipLaunchKernelGGL(codon_pre_split_kernel<true>, dim3(blocks, n), dim3(512), 0, st, d_probs, d_items + b, R);
      else
        hipLaunchKernelGGL(codon_pre_split_kernel<false>, dim3(blocks, n), dim3(512), 0, st, d_probs, d_items + b, R);
    } else if (sc.amb) {
      hipLaunchKernelGGL((codon_pre_level_kernel<T, NT, true>), dim3(blocks, n), dim3(256), 0, st, d_probs,
                         d_items + b, R);
    } else {
      hipLaunchKernelGGL((codon_pre_level_kernel<T, NT, false>), dim3(blocks, n), dim3(256), 0, st, d_probs,
                         d_items + b, R);
    }
  }
}

template <typename T, int NT>
void root_launch(const CodonSchedule& sc, const CodonProblem* d_probs, hipStream_t st) {
  hipLaunchKernelGGL((codon_root_kernel<T, NT>), dim3(sc.max_pattern_blocks, sc.n_problems), dim3(256), 0, st, d_probs);
}

template <typename T, int NT>
void reduce_launch(const CodonSchedule& sc, const CodonProblem* d_probs, const int2* d_reduce_items, double* dpart,
                   hipStream_t st, bool accumulate, bool finish) {
  const int n_items = (int)sc.reduce_items.size();
  hipLaunchKernelGGL((codon_grad_reduce_kernel<T, NT>), dim3((unsigned)(n_items * reduce_chunks<NT>())), dim3(256), 0,
                     st, d_probs, d_reduce_items, dpart, accumulate ? 1 : 0);
  if (finish)
    hipLaunchKernelGGL(codon_dbranch_kernel<NT>, dim3((unsigned)((n_items + 255) / 256)), dim3(256), 0, st, d_probs,
                       d_reduce_items, n_items, static_cast<const double*>(dpart));
}
}  // namespace

// One call per compute type and padded state count (64: NT = 4, 32: NT = 2).
#define EPOCH_CODON_DISPATCH(sc, FN, ...)      \
  do {                                         \
    if ((sc).fp64) {                           \
      if ((sc).nt == 2)                        \
        FN<double, 2>(__VA_ARGS__);            \
      else                                     \
        FN<double, 4>(__VA_ARGS__);            \
    } else if ((sc).nt == 2) {                 \
      FN<float, 2>(__VA_ARGS__);               \
    } else {                                   \
      FN<float, 4>(__VA_ARGS__);               \
    }                                          \
  } while (0)

int codon_launch_post(const CodonSchedule& sc, const CodonProblem* d_probs, const int2* d_items, hipStream_t st) {
  EPOCH_CODON_DISPATCH(sc, post_levels, sc, d_probs, d_items, st);
  return hip_check(hipGetLastError(), "codon_post_level launch");
}

int codon_launch_root(const CodonSchedule& sc, const CodonProblem* d_probs, hipStream_t st) {
  EPOCH_CODON_DISPATCH(sc, root_launch, sc, d_probs, st);
  hipLaunchKernelGGL(codon_final_kernel, dim3(sc.n_problems), dim3(256), 0, st, d_probs);
  return hip_check(hipGetLastError(), "codon_root launch");
}

size_t codon_dpart_bytes(const CodonSchedule& sc) {
  return sc.reduce_items.size() * (sc.nt == 2 ? reduce_chunks<2>() : reduce_chunks<4>()) * sizeof(double);
}

int codon_launch_pre_grad(const CodonSchedule& sc, const CodonProblem* d_probs, const int2* d_items,
                          const int2* d_reduce_items, double* dpart, hipStream_t st, bool accumulate, bool finish) {
  EPOCH_CODON_DISPATCH(sc, pre_levels, sc, d_probs, d_items, st);
  int rc = hip_check(hipGetLastError(), "codon_pre_level launch");
  if (rc) return rc;
  EPOCH_CODON_DISPATCH(sc, reduce_launch, sc, d_probs, d_reduce_items, dpart, st, accumulate, finish);
  return hip_check(hipGetLastError(), "codon_grad_reduce launch");
}

// ---- single-instance entry points (schedule built when the tree changes).
// Under an HBM budget the patterns run in chunks of codon_pc: chunk j has its
// own descriptor (pattern count, and tips, weights and per-pattern outputs
// offset to its first pattern) over the shared chunk-sized buffers.
int codon_prepare(EpochInstance* in) {
  std::vector<std::vector<int32_t>> gslots;
  codon_build_schedule({in}, in->codon_target_blocks, in->codon_sched, gslots);
  in->codon_sched.split_blocks = in->codon_split_blocks;
  const auto& sc = in->codon_sched;
  const bool grad = (in->cfg.flags & (EPOCH_GRAD_BRANCH | EPOCH_GRAD_Q)) != 0;
  const int C = in->C;  // one problem per category (C > 1 only without pattern chunks)
  const size_t gs = gslots[0].size();
  int rc = ensure(in->gslots, C * gs * sizeof(int32_t));
  const size_t slot_floats = (size_t)in->Kp * in->Kp * (in->fp64 ? 2 : 1);  // one slot, in floats
  if (!rc && grad) rc = ensure(in->Gpart, std::max<size_t>(1, C * sc.slot_total[0]) * slot_floats * sizeof(float));
  if (!rc && grad) rc = ensure(in->codon_aux, codon_dpart_bytes(sc));
  if (rc) return rc;
  const int nc = in->codon_nchunks;
  std::vector<CodonProblem> desc(nc * C);
  for (int c = 0; c < C; ++c) {
    const CodonProblem d =
        codon_descriptor(in, c, static_cast<const int32_t*>(in->gslots.ptr) + c * gs,
                         static_cast<float*>(in->Gpart.ptr) + c * sc.slot_total[0] * slot_floats);
    for (int j = 0; j < nc; ++j) {  // nc > 1 only with one category
      const int p0 = j * codon_chunk_patterns(in);
      CodonProblem& dj = desc[j * C + c];
      dj = d;
      dj.P = std::min(in->P - p0, codon_chunk_patterns(in));
      dj.tips = d.tips + p0;
      dj.weightsT = d.weightsT + p0;
      dj.weights = d.weights + p0;
      dj.site = d.site + p0;
      dj.result = nc > 1 ? d.result + 1 + j : d.result;
    }
  }
  const size_t dbytes = sizeof(CodonProblem) * desc.size();
  const size_t bytes = dbytes + sizeof(int2) * (sc.items.size() + sc.reduce_items.size());
  rc = ensure(in->codon_dev, bytes);
  if (rc) return rc;
  std::vector<char> h(bytes);
  memcpy(h.data(), desc.data(), dbytes);
  memcpy(h.data() + dbytes, sc.items.data(), sizeof(int2) * sc.items.size());
  memcpy(h.data() + dbytes + sizeof(int2) * sc.items.size(), sc.reduce_items.data(),
         sizeof(int2) * sc.reduce_items.size());
  std::vector<int32_t> hg(C * gs);
  for (int c = 0; c < C; ++c) std::copy(gslots[c].begin(), gslots[c].end(), hg.begin() + c * gs);
  rc = hip_check(hipMemcpyAsync(in->codon_dev.ptr, h.data(), bytes, hipMemcpyHostToDevice, in->stream), "codon schedule upload");
  if (!rc)
    rc = hip_check(hipMemcpyAsync(in->gslots.ptr, hg.data(), hg.size() * sizeof(int32_t), hipMemcpyHostToDevice,
                                  in->stream), "gslots upload");
  if (!rc) rc = hip_check(hipStreamSynchronize(in->stream), "codon schedule sync");
  return rc;
}

namespace {
const CodonProblem* dev_probs(EpochInstance* in) { return static_cast<const CodonProblem*>(in->codon_dev.ptr); }
const int2* dev_items(EpochInstance* in) {
  return reinterpret_cast<const int2*>(static_cast<const char*>(in->codon_dev.ptr) +
                                       sizeof(CodonProblem) * in->codon_nchunks * in->C);
}
const int2* dev_reduce_items(EpochInstance* in) { return dev_items(in) + in->codon_sched.items.size(); }
}  // namespace

// Post-order pass.  In chunks, each chunk's root reduction follows its partials
// (the next chunk overwrites them), and the chunk log-likelihoods are summed.
int launch_codon_post(EpochInstance* in) {
  in->codon_sched.amb = in->tips_amb;
  const int nc = in->codon_nchunks;
  if (nc == 1) return codon_launch_post(in->codon_sched, dev_probs(in), dev_items(in), in->stream);
  for (int j = 0; j < nc; ++j) {
    int rc = codon_launch_post(in->codon_sched, dev_probs(in) + j, dev_items(in), in->stream);
    if (!rc) rc = codon_launch_root(in->codon_sched, dev_probs(in) + j, in->stream);
    if (rc) return rc;
  }
  return launch_chunk_sum(in, nc);
}

int launch_codon_post_schedule(EpochInstance* in, const CodonSchedule& sc, const int2* d_items) {
  return codon_launch_post(sc, dev_probs(in), d_items, in->stream);
}

int launch_codon_root(EpochInstance* in) {
  if (in->codon_nchunks > 1) return EPOCH_OK;  // formed with the chunks' partials
  return codon_launch_root(in->codon_sched, dev_probs(in), in->stream);
}

// Pre-order pass and dlogL/dP.  In chunks, each chunk's partials are formed
// again first (only one chunk's fit), and dlogL/dP accumulates over chunks.
int launch_codon_pre_grad(EpochInstance* in) {
  in->codon_sched.amb = in->tips_amb;
  const int nc = in->codon_nchunks;
  double* dpart = static_cast<double*>(in->codon_aux.ptr);
  for (int j = 0; j < nc; ++j) {
    int rc = nc > 1 ? codon_launch_post(in->codon_sched, dev_probs(in) + j, dev_items(in), in->stream) : EPOCH_OK;
    if (!rc)
      rc = codon_launch_pre_grad(in->codon_sched, dev_probs(in) + j, dev_items(in), dev_reduce_items(in), dpart,
                                 in->stream, j > 0, j == nc - 1);
    if (rc) return rc;
  }
  return EPOCH_OK;
}

}  // namespace epochlik
