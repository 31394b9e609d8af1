// 64-state (codon) kernels on FP32 matrix cores (v_mfma_f32_16x16x4f32).
//
// Applies to FP32 instances with 48 < K <= 64 (padded to 64) and one rate
// category.  Layout as elsewhere: partials / outside vectors [slot][P][64],
// transition matrices [node][64][64] row-major.
//
// MFMA operand mapping (16x16x4, wavefront of 64 lanes, g = lane / 16,
// r = lane % 16):  A[m][k]: m = r, k = g;  B[k][n]: k = g, n = r;
// D[m][n] (4 registers v): m = 4 g + v, n = r.
//
// Block = 4 wavefronts = one node and one tile of 64 patterns; wavefront w
// produces output states 16 w .. 16 w + 15 for all 64 patterns (four 16x16
// blocks along the patterns).  The contraction index k runs over states; its
// order inside a 16-wide group is permuted (k = 16 t + 4 g + e) so that both
// operands come from 16-byte loads.
//   codon_post_level : Eq. 4 for one level, per-pattern power-of-two scale
//                      agreed across the four wavefronts through LDS.
//   codon_pre_level  : outside vectors of one level and dlogL/dP of the two
//                      child branches, accumulated over R tiles as MFMA
//                      outer products; rows 16 w .. 16 w + 15 of G per wavefront.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstring>

#include "device_common.h"
#include "instance.h"

namespace epochlik {

namespace {

typedef float f4 __attribute__((ext_vector_type(4)));

constexpr int KP = 64;
constexpr int LDP = 68;  // padded LDS row stride (floats) against bank conflicts
constexpr int TILE = 64;
constexpr int kMaxSlots = 64;  // partial-sum slots per branch (blocks sharing one node)

__device__ inline f4 mfma(float a, float b, f4 c) { return __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c, 0, 0, 0); }

// Stage a 64x64 row-major matrix into LDS with row stride LDP.
__device__ inline void stage_matrix(float* __restrict__ s, const float* __restrict__ g) {
  for (int e = threadIdx.x; e < KP * KP / 4; e += 256) {
    const int row = e / 16, c4 = e % 16;
    const float4 v = reinterpret_cast<const float4*>(g)[e];
    *reinterpret_cast<float4*>(s + row * LDP + 4 * c4) = v;
  }
}

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

// S[mb] (D layout: pattern 16 mb + 4 g + v, state 16 w + r) = sum_j L[p][j] P[i][j]
// for an internal child whose 64x64 partial tile starts at Lg (row stride 64).
__device__ inline void child_gemm(f4 (&S)[4], const float* __restrict__ Lg, int P, int p0,
                                  const float* __restrict__ sP, int w, int g, int r) {
#pragma unroll
  for (int mb = 0; mb < 4; ++mb) S[mb] = f4{0.f, 0.f, 0.f, 0.f};
  const float* prow = sP + (16 * w + r) * LDP;  // B[k][n] = P[n][k], n = 16 w + r
#pragma unroll
  for (int t = 0; t < 4; ++t) {
    const float4 b4 = *reinterpret_cast<const float4*>(prow + 16 * t + 4 * g);
#pragma unroll
    for (int mb = 0; mb < 4; ++mb) {
      const int p = p0 + 16 * mb + r;  // A[m][k]: m = r (pattern), k over states
      float4 a4 = make_float4(0.f, 0.f, 0.f, 0.f);
      if (p < P) a4 = *reinterpret_cast<const float4*>(Lg + (size_t)p * KP + 16 * t + 4 * g);
      S[mb] = mfma(a4.x, b4.x, S[mb]);
      S[mb] = mfma(a4.y, b4.y, S[mb]);
      S[mb] = mfma(a4.z, b4.z, S[mb]);
      S[mb] = mfma(a4.w, b4.w, S[mb]);
    }
  }
}

// Tip child: S = P[i][state_p] looked up from LDS (missing state K: row sum).
__device__ inline void tip_lookup(f4 (&S)[4], const uint8_t* __restrict__ tipst, int P, int p0, int K,
                                  const float* __restrict__ sP, int w, int g, int r) {
  const float* prow = sP + (16 * w + r) * LDP;
#pragma unroll
  for (int mb = 0; mb < 4; ++mb)
#pragma unroll
    for (int v = 0; v < 4; ++v) {
      const int p = p0 + 16 * mb + 4 * g + v;
      const int st = p < P ? tipst[p] : 0;
      float val;
      if (st < K) {
        val = prow[st];
      } else {
        val = 0.f;
        for (int j = 0; j < K; ++j) val += prow[j];
      }
      S[mb][v] = val;
    }
}

// ---------------------------------------------------------------------------
__global__ __launch_bounds__(256) void codon_post_level_kernel(const CodonProblem* __restrict__ probs,
                                                                const int2* __restrict__ items) {
  __shared__ __align__(16) float sPa[KP * LDP];
  __shared__ __align__(16) float sPb[KP * LDP];
  __shared__ float smax[4][TILE];
  const int2 it = items[blockIdx.y];
  const CodonProblem& pr = probs[it.x];
  const int N = pr.N, P = pr.P, K = pr.K;
  const int p0 = blockIdx.x * TILE;
  if (p0 >= P) return;  // uniform: this problem has fewer tiles
  const float* __restrict__ Pm = pr.Pm;
  const uint8_t* __restrict__ tips = pr.tips;
  const float* __restrict__ part_in = pr.part;
  float* __restrict__ part_out = pr.part;
  const int32_t* __restrict__ scale_in = pr.scales;
  int32_t* __restrict__ scale_out = pr.scales;
  const int u = it.y;
  const int a = pr.left[u], b = pr.right[u];
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6, g = lane >> 4, r = lane & 15;
  stage_matrix(sPa, Pm + (size_t)a * KP * KP);
  stage_matrix(sPb, Pm + (size_t)b * KP * KP);
  __syncthreads();
  f4 Sa[4], Sb[4];
  if (a < N)
    tip_lookup(Sa, tips + (size_t)a * P, P, p0, K, sPa, w, g, r);
  else
    child_gemm(Sa, part_in + (size_t)(a - N) * P * KP, P, p0, sPa, w, g, r);
  if (b < N)
    tip_lookup(Sb, tips + (size_t)b * P, P, p0, K, sPb, w, g, r);
  else
    child_gemm(Sb, part_in + (size_t)(b - N) * P * KP, P, p0, sPb, w, g, r);
  // x = Sa * Sb; per-pattern max over this wavefront's 16 states, then over wavefronts
  float m[4][4];
#pragma unroll
  for (int mb = 0; mb < 4; ++mb)
#pragma unroll
    for (int v = 0; v < 4; ++v) {
      Sa[mb][v] *= Sb[mb][v];
      m[mb][v] = row16_max(Sa[mb][v]);
    }
  if (r == 0)
#pragma unroll
    for (int mb = 0; mb < 4; ++mb)
#pragma unroll
      for (int v = 0; v < 4; ++v) smax[w][16 * mb + 4 * g + v] = m[mb][v];
  __syncthreads();
#pragma unroll
  for (int mb = 0; mb < 4; ++mb)
#pragma unroll
    for (int v = 0; v < 4; ++v) {
      const int pl = 16 * mb + 4 * g + v;
      const float mm = fmaxf(fmaxf(smax[0][pl], smax[1][pl]), fmaxf(smax[2][pl], smax[3][pl]));
      const int e = scale_exponent(mm);
      const int p = p0 + pl;
      if (p < P) {
        part_out[((size_t)(u - N) * P + p) * KP + 16 * w + r] = ldexpf(Sa[mb][v], -e);
        if (w == 0 && r == 0) {
          int s = e;
          if (a >= N) s += scale_in[(size_t)(a - N) * P + p];
          if (b >= N) s += scale_in[(size_t)(b - N) * P + p];
          scale_out[(size_t)(u - N) * P + p] = s;
        }
      }
    }
}

// ---------------------------------------------------------------------------
// Root: one thread per pattern, L_p = sum_i pi_i x_root(p, i) in FP64; block
// partial sums of w_p log L_p per problem (blockIdx.y).
__global__ __launch_bounds__(256) void codon_root_kernel(const CodonProblem* __restrict__ probs) {
  __shared__ double sm[256];
  const CodonProblem& pr = probs[blockIdx.y];
  const int P = pr.P, K = pr.K;
  if ((int)blockIdx.x * 256 >= P) return;  // uniform
  const int p = blockIdx.x * 256 + threadIdx.x;
  const size_t slot = pr.root - pr.N;
  double contrib = 0.0;
  if (p < P) {
    double L = 0.0;
    const float* x = pr.part + (slot * P + p) * KP;
    for (int i = 0; i < K; ++i) L += pr.pi[i] * (double)x[i];
    const double s = log(L) + (double)pr.scales[slot * P + p] * kLn2;
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
  const int nb = (pr.P + 255) / 256;
  double acc = 0.0;
  for (int k = threadIdx.x; k < nb; k += 256) acc += pr.blocksum[k];
  const double tot = block_sum<256>(acc, sm);
  if (threadIdx.x == 0) pr.result[0] = tot;
}

// ---------------------------------------------------------------------------
// Loads of one pattern block in the D layout (pattern 16 mb + 4 g + v, state
// 16 nb + r): outside vector q, or a stored partial, or a tip indicator.
__device__ inline float dval_partial(const float* __restrict__ Lg, int P, int p, int col) {
  return p < P ? Lg[(size_t)p * KP + col] : 0.f;
}

__global__ __launch_bounds__(256) void codon_pre_level_kernel(const CodonProblem* __restrict__ probs,
                                                               const int2* __restrict__ items, int R) {
  __shared__ __align__(16) float sPa[KP * LDP];
  __shared__ __align__(16) float sPb[KP * LDP];
  __shared__ __align__(16) float sT[TILE * LDP];  // t_a or t_b tile [pattern][state]
  __shared__ float sx[4][TILE];
  const int2 it = items[blockIdx.y];
  const CodonProblem& pr = probs[it.x];
  const int N = pr.N, P = pr.P, K = pr.K, root = pr.root, n_slots = pr.n_slots;
  if ((int)blockIdx.x * R * TILE >= P) return;  // uniform: this problem has fewer tiles
  const float* __restrict__ Pm = pr.Pm;
  const uint8_t* __restrict__ tips = pr.tips;
  const float* __restrict__ part = pr.part;
  const float* __restrict__ pre_in = pr.pre;
  float* __restrict__ pre_out = pr.pre;
  const double* __restrict__ pi = pr.pi;
  const float* __restrict__ weights = pr.weightsT;
  float* __restrict__ Gpart = pr.Gpart;
  const int u = it.y;
  const int a = pr.left[u], b = pr.right[u];
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6, g = lane >> 4, r = lane & 15;
  stage_matrix(sPa, Pm + (size_t)a * KP * KP);
  stage_matrix(sPb, Pm + (size_t)b * KP * KP);
  __syncthreads();
  // G accumulators: rows 16 w + (4 g + v), columns 16 nb + r, per child
  f4 Ga[4], Gb[4];
#pragma unroll
  for (int nb = 0; nb < 4; ++nb) {
    Ga[nb] = f4{0.f, 0.f, 0.f, 0.f};
    Gb[nb] = f4{0.f, 0.f, 0.f, 0.f};
  }
  const float* La = a >= N ? part + (size_t)(a - N) * P * KP : nullptr;
  const float* Lb = b >= N ? part + (size_t)(b - N) * P * KP : nullptr;
  const float* Qu = u == root ? nullptr : pre_in + (size_t)(u - N) * P * KP;
  const int my_state = 16 * w + r;
  const float piv = my_state < K ? (float)pi[my_state] : 0.f;
  for (int rr = 0; rr < R; ++rr) {
    const int p0 = (blockIdx.x * R + rr) * TILE;
    if (p0 >= P) break;  // uniform
    f4 Sa[4], Sb[4];
    if (a < N)
      tip_lookup(Sa, tips + (size_t)a * P, P, p0, K, sPa, w, g, r);
    else
      child_gemm(Sa, La, P, p0, sPa, w, g, r);
    if (b < N)
      tip_lookup(Sb, tips + (size_t)b * P, P, p0, K, sPb, w, g, r);
    else
      child_gemm(Sb, Lb, P, p0, sPb, w, g, r);
    // q in the D layout and the per-pattern likelihood contributions
    f4 Q[4];
    float lsum[4][4];
#pragma unroll
    for (int mb = 0; mb < 4; ++mb)
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        const int p = p0 + 16 * mb + 4 * g + v;
        Q[mb][v] = Qu ? dval_partial(Qu, P, p, my_state) : piv;
        lsum[mb][v] = row16_sum(Q[mb][v] * Sa[mb][v] * Sb[mb][v]);
      }
    if (r == 0)
#pragma unroll
      for (int mb = 0; mb < 4; ++mb)
#pragma unroll
        for (int v = 0; v < 4; ++v) sx[w][16 * mb + 4 * g + v] = lsum[mb][v];
    __syncthreads();
    float coef[4][4];
#pragma unroll
    for (int mb = 0; mb < 4; ++mb)
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        const int pl = 16 * mb + 4 * g + v;
        const float L = (sx[0][pl] + sx[1][pl]) + (sx[2][pl] + sx[3][pl]);
        const int p = p0 + pl;
        coef[mb][v] = (p < P && L > 0.f) ? weights[p] / L : 0.f;
      }
    // G_a[i][j] += sum_p coef_p t_a[p][i] L_a[p][j] with t_a = q * S_b:
    // A[m = i][k = p] is the D-layout register (k-step v), B[k = p][n = j] the child vector.
#pragma unroll
    for (int side = 0; side < 2; ++side) {
      const int child = side == 0 ? a : b;
      const float* Lc = side == 0 ? La : Lb;
      f4* G = side == 0 ? Ga : Gb;
      const uint8_t* tipst = child < N ? tips + (size_t)child * P : nullptr;
#pragma unroll
      for (int mb = 0; mb < 4; ++mb)
#pragma unroll
        for (int v = 0; v < 4; ++v) {
          const float t = Q[mb][v] * (side == 0 ? Sb[mb][v] : Sa[mb][v]);
          const float av = coef[mb][v] * t;
          const int p = p0 + 16 * mb + 4 * g + v;
          int st = 0;
          if (tipst) st = p < P ? tipst[p] : K;
#pragma unroll
          for (int nb = 0; nb < 4; ++nb) {
            const int col = 16 * nb + r;
            float bv;
            if (tipst)
              bv = (p < P && (st == col || (st >= K && col < K))) ? 1.f : 0.f;
            else
              bv = dval_partial(Lc, P, p, col);
            G[nb] = mfma(av, bv, G[nb]);
          }
        }
    }
    // outside vectors of internal children: q_c[p][j] = sum_i t_c[p][i] P_c[i][j]
#pragma unroll
    for (int side = 0; side < 2; ++side) {
      const int child = side == 0 ? a : b;
      if (child < N) continue;  // uniform
      __syncthreads();  // sT is free
#pragma unroll
      for (int mb = 0; mb < 4; ++mb)
#pragma unroll
        for (int v = 0; v < 4; ++v)
          sT[(16 * mb + 4 * g + v) * LDP + my_state] = Q[mb][v] * (side == 0 ? Sb[mb][v] : Sa[mb][v]);
      __syncthreads();
      const float* sP = side == 0 ? sPa : sPb;
      // D[m = p][n = j], j = 16 w + r: A[m = p][k = i] from sT, B[k = i][n = j] = P[i][j]
      f4 Qo[4];
#pragma unroll
      for (int mb = 0; mb < 4; ++mb) Qo[mb] = f4{0.f, 0.f, 0.f, 0.f};
#pragma unroll
      for (int t = 0; t < 4; ++t) {
        float b4[4];
#pragma unroll
        for (int e = 0; e < 4; ++e) b4[e] = sP[(16 * t + 4 * g + e) * LDP + my_state];
#pragma unroll
        for (int mb = 0; mb < 4; ++mb) {
          const float4 a4 = *reinterpret_cast<const float4*>(sT + (16 * mb + r) * LDP + 16 * t + 4 * g);
          Qo[mb] = mfma(a4.x, b4[0], Qo[mb]);
          Qo[mb] = mfma(a4.y, b4[1], Qo[mb]);
          Qo[mb] = mfma(a4.z, b4[2], Qo[mb]);
          Qo[mb] = mfma(a4.w, b4[3], Qo[mb]);
        }
      }
      float mx[4][4];
#pragma unroll
      for (int mb = 0; mb < 4; ++mb)
#pragma unroll
        for (int v = 0; v < 4; ++v) mx[mb][v] = row16_max(Qo[mb][v]);
      __syncthreads();  // every wavefront is done reading sx
      if (r == 0)
#pragma unroll
        for (int mb = 0; mb < 4; ++mb)
#pragma unroll
          for (int v = 0; v < 4; ++v) sx[w][16 * mb + 4 * g + v] = mx[mb][v];
      __syncthreads();
#pragma unroll
      for (int mb = 0; mb < 4; ++mb)
#pragma unroll
        for (int v = 0; v < 4; ++v) {
          const int pl = 16 * mb + 4 * g + v;
          const float mm = fmaxf(fmaxf(sx[0][pl], sx[1][pl]), fmaxf(sx[2][pl], sx[3][pl]));
          const int e = scale_exponent(mm);
          const int p = p0 + pl;
          if (p < P) pre_out[((size_t)(child - N) * P + p) * KP + my_state] = ldexpf(Qo[mb][v], -e);
        }
    }
    __syncthreads();  // sx and sT reuse by the next tile
  }
  // partial G of this block: rows 16 w + 4 g + v, columns 16 nb + r
#pragma unroll
  for (int side = 0; side < 2; ++side) {
    const int child = side == 0 ? a : b;
    const f4* G = side == 0 ? Ga : Gb;
    float* dst = Gpart + ((size_t)child * n_slots + blockIdx.x) * (KP * KP);
#pragma unroll
    for (int nb = 0; nb < 4; ++nb)
#pragma unroll
      for (int v = 0; v < 4; ++v) dst[(16 * w + 4 * g + v) * KP + 16 * nb + r] = G[nb][v];
  }
}

// G[v] = sum of the FP32 slot partials in FP64 (fixed order), then dlogL/dl.
__global__ __launch_bounds__(256) void codon_grad_reduce_kernel(const CodonProblem* __restrict__ probs,
                                                                const int2* __restrict__ items) {
  __shared__ double sm[256];
  const int2 it = items[blockIdx.x];
  const CodonProblem& pr = probs[it.x];
  const int v = it.y;
  const int ns = v == pr.root ? 0 : pr.gslots[v];
  const float* src = pr.Gpart + (size_t)v * pr.n_slots * (KP * KP);
  double d = 0.0;
  for (int e = threadIdx.x; e < KP * KP; e += 256) {
    double s = 0.0;
    for (int k = 0; k < ns; ++k) s += (double)src[(size_t)k * (KP * KP) + e];
    pr.G[(size_t)v * KP * KP + e] = s;
    d += s * (double)pr.dPm[(size_t)v * KP * KP + e];
  }
  const double tot = block_sum<256>(d, sm);
  if (threadIdx.x == 0) pr.dbranch[v] = (v == pr.root) ? 0.0 : tot;
}

int codon_tiles_per_block(int tiles, int n_items, int target_blocks, int r_max) {
  const long per_item = ((long)target_blocks + n_items - 1) / n_items;
  long R = (tiles + per_item - 1) / per_item;
  if (R < 1) R = 1;
  if (R > r_max) R = r_max;
  return (int)R;
}

}  // namespace

// Partial-sum slots per branch: at most kMaxSlots blocks share a node, so the
// dlogL/dP partials of a branch take at most kMaxSlots x 16 KB.
int codon_max_slots(int P) { return std::min((P + TILE - 1) / TILE, kMaxSlots); }

CodonProblem codon_descriptor(const EpochInstance* in, const int32_t* gslots) {
  CodonProblem d{};
  d.Pm = static_cast<const float*>(in->Pm.ptr);
  d.tips = static_cast<const uint8_t*>(in->tips.ptr);
  d.part = static_cast<float*>(in->partials.ptr);
  d.pre = static_cast<float*>(in->pre.ptr);
  d.scales = static_cast<int32_t*>(in->scales.ptr);
  d.weightsT = static_cast<const float*>(in->weightsT.ptr);
  d.weights = static_cast<const double*>(in->weights.ptr);
  d.pi = static_cast<const double*>(in->pi.ptr);
  d.Gpart = static_cast<float*>(in->Gpart.ptr);
  d.dPm = static_cast<const float*>(in->dPm.ptr);
  d.G = static_cast<double*>(in->G.ptr);
  d.dbranch = static_cast<double*>(in->dbranch.ptr);
  d.site = static_cast<double*>(in->site.ptr);
  d.blocksum = static_cast<double*>(in->blocksum.ptr);
  d.result = static_cast<double*>(in->result.ptr);
  d.left = in->d_left;
  d.right = in->d_right;
  d.gslots = gslots;
  d.N = in->N;
  d.P = in->P;
  d.K = in->K;
  d.root = in->plan.root;
  d.n_slots = codon_max_slots(in->P);
  d.n_nodes = in->n_nodes;
  return d;
}

// Merged level schedule over one or more problems (levels counted from the tips).
void codon_build_schedule(const std::vector<const EpochInstance*>& insts, int target_blocks, CodonSchedule& out,
                          std::vector<std::vector<int32_t>>& gslots) {
  out.items.clear();
  out.level_off.assign(1, 0);
  out.level_R.clear();
  out.reduce_items.clear();
  int n_levels = 0, max_tiles = 0, max_pblocks = 0;
  for (auto* in : insts) {
    n_levels = std::max(n_levels, in->plan.n_levels);
    max_tiles = std::max(max_tiles, (in->P + TILE - 1) / TILE);
    max_pblocks = std::max(max_pblocks, (in->P + 255) / 256);
  }
  gslots.assign(insts.size(), {});
  for (size_t q = 0; q < insts.size(); ++q) gslots[q].assign(insts[q]->n_nodes, 0);
  for (int l = 1; l <= n_levels; ++l) {
    const size_t begin = out.items.size();
    for (size_t q = 0; q < insts.size(); ++q) {
      const auto& pl = insts[q]->plan;
      if (l > pl.n_levels) continue;
      for (int k = pl.level_offset[l]; k < pl.level_offset[l + 1]; ++k) out.items.push_back(make_int2((int)q, pl.level_nodes[k]));
    }
    const int n_items = (int)(out.items.size() - begin);
    int R = codon_tiles_per_block(max_tiles, std::max(1, n_items), target_blocks, 64);
    R = std::max(R, (max_tiles + kMaxSlots - 1) / kMaxSlots);  // at most kMaxSlots blocks per node
    out.level_off.push_back((int)out.items.size());
    out.level_R.push_back(R);
    for (size_t k = begin; k < out.items.size(); ++k) {
      const int q = out.items[k].x, u = out.items[k].y;
      const auto& pl = insts[q]->plan;
      const int tiles = (insts[q]->P + TILE - 1) / TILE;
      const int used = (tiles + R - 1) / R;
      gslots[q][pl.left[u]] = used;
      gslots[q][pl.right[u]] = used;
    }
  }
  for (size_t q = 0; q < insts.size(); ++q)
    for (int v = 0; v < insts[q]->n_nodes; ++v) out.reduce_items.push_back(make_int2((int)q, v));
  out.n_levels = n_levels;
  out.max_tiles = max_tiles;
  out.max_pattern_blocks = max_pblocks;
  out.n_problems = (int)insts.size();
}

int codon_launch_post(const CodonSchedule& sc, const CodonProblem* d_probs, const int2* d_items, hipStream_t st) {
  for (int l = 1; l <= sc.n_levels; ++l) {
    const int b = sc.level_off[l - 1], n = sc.level_off[l] - b;
    if (!n) continue;
    hipLaunchKernelGGL(codon_post_level_kernel, dim3(sc.max_tiles, n), dim3(256), 0, st, d_probs, d_items + b);
  }
  return hip_check(hipGetLastError(), "codon_post_level launch");
}

int codon_launch_root(const CodonSchedule& sc, const CodonProblem* d_probs, hipStream_t st) {
  hipLaunchKernelGGL(codon_root_kernel, dim3(sc.max_pattern_blocks, sc.n_problems), dim3(256), 0, st, d_probs);
  hipLaunchKernelGGL(codon_final_kernel, dim3(sc.n_problems), dim3(256), 0, st, d_probs);
  return hip_check(hipGetLastError(), "codon_root launch");
}

int codon_launch_pre_grad(const CodonSchedule& sc, const CodonProblem* d_probs, const int2* d_items,
                          const int2* d_reduce_items, hipStream_t st) {
  for (int l = sc.n_levels; l >= 1; --l) {
    const int b = sc.level_off[l - 1], n = sc.level_off[l] - b;
    if (!n) continue;
    const int R = sc.level_R[l - 1];
    const int blocks = (sc.max_tiles + R - 1) / R;
    hipLaunchKernelGGL(codon_pre_level_kernel, dim3(blocks, n), dim3(256), 0, st, d_probs, d_items + b, R);
  }
  int rc = hip_check(hipGetLastError(), "codon_pre_level launch");
  if (rc) return rc;
  hipLaunchKernelGGL(codon_grad_reduce_kernel, dim3((unsigned)sc.reduce_items.size()), dim3(256), 0, st, d_probs,
                     d_reduce_items);
  return hip_check(hipGetLastError(), "codon_grad_reduce launch");
}

// ---- single-instance entry points (schedule built when the tree changes)
int codon_prepare(EpochInstance* in) {
  std::vector<std::vector<int32_t>> gslots;
  codon_build_schedule({in}, in->codon_target_blocks, in->codon_sched, gslots);
  const CodonProblem d = codon_descriptor(in, static_cast<const int32_t*>(in->gslots.ptr));
  const auto& sc = in->codon_sched;
  const size_t bytes = sizeof(CodonProblem) + sizeof(int2) * (sc.items.size() + sc.reduce_items.size());
  int rc = ensure(in->codon_dev, bytes);
  if (rc) return rc;
  std::vector<char> h(bytes);
  memcpy(h.data(), &d, sizeof(d));
  memcpy(h.data() + sizeof(d), sc.items.data(), sizeof(int2) * sc.items.size());
  memcpy(h.data() + sizeof(d) + sizeof(int2) * sc.items.size(), sc.reduce_items.data(),
         sizeof(int2) * sc.reduce_items.size());
  rc = hip_check(hipMemcpyAsync(in->codon_dev.ptr, h.data(), bytes, hipMemcpyHostToDevice, in->stream), "codon schedule upload");
  if (!rc && in->gslots.ptr)
    rc = hip_check(hipMemcpyAsync(in->gslots.ptr, gslots[0].data(), gslots[0].size() * sizeof(int32_t),
                                  hipMemcpyHostToDevice, in->stream), "gslots upload");
  if (!rc) rc = hip_check(hipStreamSynchronize(in->stream), "codon schedule sync");
  return rc;
}

namespace {
const CodonProblem* dev_probs(EpochInstance* in) { return static_cast<const CodonProblem*>(in->codon_dev.ptr); }
const int2* dev_items(EpochInstance* in) {
  return reinterpret_cast<const int2*>(static_cast<const char*>(in->codon_dev.ptr) + sizeof(CodonProblem));
}
const int2* dev_reduce_items(EpochInstance* in) { return dev_items(in) + in->codon_sched.items.size(); }
}  // namespace

int launch_codon_post(EpochInstance* in) { return codon_launch_post(in->codon_sched, dev_probs(in), dev_items(in), in->stream); }
int launch_codon_root(EpochInstance* in) { return codon_launch_root(in->codon_sched, dev_probs(in), in->stream); }
int launch_codon_pre_grad(EpochInstance* in) {
  return codon_launch_pre_grad(in->codon_sched, dev_probs(in), dev_items(in), dev_reduce_items(in), in->stream);
}

}  // namespace epochlik
