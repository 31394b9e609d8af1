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

#include "device_common.h"
#include "instance.h"

namespace epochlik {

namespace {

typedef float f4 __attribute__((ext_vector_type(4)));

constexpr int KP = 64;
constexpr int LDP = 68;  // padded LDS row stride (floats) against bank conflicts
constexpr int TILE = 64;

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
__global__ __launch_bounds__(256) void codon_post_level_kernel(
    const int32_t* __restrict__ nodes, const int32_t* __restrict__ left, const int32_t* __restrict__ right,
    const float* __restrict__ Pm, const uint8_t* __restrict__ tips, const float* __restrict__ part_in,
    float* __restrict__ part_out, const int32_t* __restrict__ scale_in, int32_t* __restrict__ scale_out,
    int N, int P, int K) {
  __shared__ __align__(16) float sPa[KP * LDP];
  __shared__ __align__(16) float sPb[KP * LDP];
  __shared__ float smax[4][TILE];
  const int u = nodes[blockIdx.y];
  const int a = left[u], b = right[u];
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6, g = lane >> 4, r = lane & 15;
  const int p0 = blockIdx.x * TILE;
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
// Root: L_p = sum_i pi_i x_root(p, i); one wavefront per 64 patterns? no: one
// thread per pattern, 64 states read as float4.
__global__ __launch_bounds__(256) void codon_root_kernel(const float* __restrict__ rootp,
                                                         const int32_t* __restrict__ scale_root,
                                                         const double* __restrict__ pi,
                                                         const double* __restrict__ weights,
                                                         double* __restrict__ site, double* __restrict__ block_out,
                                                         int P, int K) {
  __shared__ double sm[256];
  const int p = blockIdx.x * 256 + threadIdx.x;
  double contrib = 0.0;
  if (p < P) {
    double L = 0.0;
    const float* x = rootp + (size_t)p * KP;
    for (int i = 0; i < K; ++i) L += pi[i] * (double)x[i];
    const double s = log(L) + (double)scale_root[p] * kLn2;
    site[p] = s;
    contrib = weights[p] * s;
  }
  const double tot = block_sum<256>(contrib, sm);
  if (threadIdx.x == 0) block_out[blockIdx.x] = tot;
}

// ---------------------------------------------------------------------------
// Loads of one pattern block in the D layout (pattern 16 mb + 4 g + v, state
// 16 nb + r): outside vector q, or a stored partial, or a tip indicator.
__device__ inline float dval_partial(const float* __restrict__ Lg, int P, int p, int col) {
  return p < P ? Lg[(size_t)p * KP + col] : 0.f;
}

__global__ __launch_bounds__(256) void codon_pre_level_kernel(
    const int32_t* __restrict__ nodes, const int32_t* __restrict__ left, const int32_t* __restrict__ right,
    const float* __restrict__ Pm, const uint8_t* __restrict__ tips, const float* __restrict__ part,
    const float* __restrict__ pre_in, float* __restrict__ pre_out, const double* __restrict__ pi,
    const float* __restrict__ weights, int root, int N, int P, int K, int R, int n_slots,
    float* __restrict__ Gpart) {
  __shared__ __align__(16) float sPa[KP * LDP];
  __shared__ __align__(16) float sPb[KP * LDP];
  __shared__ __align__(16) float sT[TILE * LDP];  // t_a or t_b tile [pattern][state]
  __shared__ float sx[4][TILE];
  const int u = nodes[blockIdx.y];
  const int a = left[u], b = right[u];
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
__global__ __launch_bounds__(256) void codon_grad_reduce_kernel(const float* __restrict__ Gpart,
                                                                const float* __restrict__ dP,
                                                                const int32_t* __restrict__ slots_per_node,
                                                                int n_slots, int root, double* __restrict__ G,
                                                                double* __restrict__ dbranch) {
  __shared__ double sm[256];
  const int v = blockIdx.x;
  const int ns = v == root ? 0 : slots_per_node[v];
  const float* src = Gpart + (size_t)v * n_slots * (KP * KP);
  double d = 0.0;
  for (int e = threadIdx.x; e < KP * KP; e += 256) {
    double s = 0.0;
    for (int k = 0; k < ns; ++k) s += (double)src[(size_t)k * (KP * KP) + e];
    G[(size_t)v * KP * KP + e] = s;
    d += s * (double)dP[(size_t)v * KP * KP + e];
  }
  const double tot = block_sum<256>(d, sm);
  if (threadIdx.x == 0) dbranch[v] = (v == root) ? 0.0 : tot;
}

int codon_tiles_per_block(int tiles, int n_l, int r_max) {
  const long target_blocks = 1024;
  const long per_node = (target_blocks + n_l - 1) / n_l;
  long R = (tiles + per_node - 1) / per_node;
  if (R < 1) R = 1;
  if (R > r_max) R = r_max;
  return (int)R;
}

}  // namespace

int codon_blocks(const EpochInstance* in, int n_l) {
  const int tiles = (in->P + TILE - 1) / TILE;
  const int R = codon_tiles_per_block(tiles, n_l, 64);
  return (tiles + R - 1) / R;
}

int codon_max_slots(int P) { return (P + TILE - 1) / TILE; }

int launch_codon_post(EpochInstance* in) {
  const auto& pl = in->plan;
  const int tiles = (in->P + TILE - 1) / TILE;
  for (int l = 1; l <= pl.n_levels; ++l) {
    const int n_l = pl.level_offset[l + 1] - pl.level_offset[l];
    if (!n_l) continue;
    hipLaunchKernelGGL(codon_post_level_kernel, dim3(tiles, n_l), dim3(256), 0, in->stream,
                       in->d_level_nodes + pl.level_offset[l], in->d_left, in->d_right,
                       static_cast<const float*>(in->Pm.ptr), static_cast<const uint8_t*>(in->tips.ptr),
                       static_cast<const float*>(in->partials.ptr), static_cast<float*>(in->partials.ptr),
                       static_cast<const int32_t*>(in->scales.ptr), static_cast<int32_t*>(in->scales.ptr),
                       in->N, in->P, in->K);
  }
  return hip_check(hipGetLastError(), "codon_post_level launch");
}

int launch_codon_root(EpochInstance* in) {
  const int nb = (in->P + 255) / 256;
  const size_t slot = in->plan.root - in->N;
  hipLaunchKernelGGL(codon_root_kernel, dim3(nb), dim3(256), 0, in->stream,
                     static_cast<const float*>(in->partials.ptr) + slot * (size_t)in->P * KP,
                     static_cast<const int32_t*>(in->scales.ptr) + slot * (size_t)in->P,
                     static_cast<const double*>(in->pi.ptr), static_cast<const double*>(in->weights.ptr),
                     static_cast<double*>(in->site.ptr), static_cast<double*>(in->blocksum.ptr), in->P, in->K);
  int rc = hip_check(hipGetLastError(), "codon_root launch");
  if (rc) return rc;
  return launch_final_sum(in, nb);
}

int launch_codon_pre_grad(EpochInstance* in) {
  const auto& pl = in->plan;
  const int tiles = (in->P + TILE - 1) / TILE;
  const int n_slots = codon_max_slots(in->P);
  for (int l = pl.n_levels; l >= 1; --l) {
    const int n_l = pl.level_offset[l + 1] - pl.level_offset[l];
    if (!n_l) continue;
    const int R = codon_tiles_per_block(tiles, n_l, 64);
    const int blocks = (tiles + R - 1) / R;
    hipLaunchKernelGGL(codon_pre_level_kernel, dim3(blocks, n_l), dim3(256), 0, in->stream,
                       in->d_level_nodes + pl.level_offset[l], in->d_left, in->d_right,
                       static_cast<const float*>(in->Pm.ptr), static_cast<const uint8_t*>(in->tips.ptr),
                       static_cast<const float*>(in->partials.ptr), static_cast<const float*>(in->pre.ptr),
                       static_cast<float*>(in->pre.ptr), static_cast<const double*>(in->pi.ptr),
                       static_cast<const float*>(in->weightsT.ptr), pl.root, in->N, in->P, in->K, R, n_slots,
                       static_cast<float*>(in->Gpart.ptr));
  }
  int rc = hip_check(hipGetLastError(), "codon_pre_level launch");
  if (rc) return rc;
  hipLaunchKernelGGL(codon_grad_reduce_kernel, dim3(in->n_nodes), dim3(256), 0, in->stream,
                     static_cast<const float*>(in->Gpart.ptr), static_cast<const float*>(in->dPm.ptr),
                     static_cast<const int32_t*>(in->gslots.ptr), n_slots, pl.root,
                     static_cast<double*>(in->G.ptr), static_cast<double*>(in->dbranch.ptr));
  return hip_check(hipGetLastError(), "codon_grad_reduce launch");
}

// slots written per branch (the block count of its parent's level)
void codon_slots_per_node(const EpochInstance* in, std::vector<int32_t>& out) {
  const auto& pl = in->plan;
  out.assign(in->n_nodes, 0);
  for (int l = 1; l <= pl.n_levels; ++l) {
    const int n_l = pl.level_offset[l + 1] - pl.level_offset[l];
    if (!n_l) continue;
    const int blocks = codon_blocks(in, n_l);
    for (int k = pl.level_offset[l]; k < pl.level_offset[l + 1]; ++k) {
      const int u = pl.level_nodes[k];
      out[pl.left[u]] = blocks;
      out[pl.right[u]] = blocks;
    }
  }
}

}  // namespace epochlik
