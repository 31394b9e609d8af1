// Generic (any K <= 64) HIP kernels: the reference GPU path in FP32 or FP64.
//
//   pstage   : transition matrices as ordered products of eigen-reconstructed
//              exponentials (Eq. 3, 6, 7; Appendix A), plus dP/dl.
//   post     : level-synchronous Felsenstein pruning with power-of-two
//              rescaling (Eq. 4).
//   root     : root sum over pi and categories, FP64 log-sum (text after Eq. 4).
//   pre      : level-synchronous outside (pre-order) vectors for the adjoint.
//   grad     : dlogL/dP per branch (rank-P accumulation), FP64 chunk reduction,
//              and dlogL/dl = <G, dP/dl>.
//   eigcheck : FP64 reconstruction residual of each eigensystem.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>

#include "device_common.h"
#include "eigen_block.h"
#include "instance.h"

namespace epochlik {

namespace {

// ---------------------------------------------------------------------------
// P stage.  One item = (node v, category c).  For Kp^2 <= 256 several items
// share a block; otherwise one item per block and EPT elements per thread.
// ---------------------------------------------------------------------------
template <typename T, typename TO, bool GRAD, int EPT>
__global__ __launch_bounds__(256) void pstage_generic_kernel(
    int n_nodes, const int32_t* __restrict__ node_list, int Kp, int C, const T* __restrict__ eigV,
    const T* __restrict__ eigVi,
    const T* __restrict__ lre, const T* __restrict__ lim, const int32_t* __restrict__ seg_offset,
    const int32_t* __restrict__ seg_process, const double* __restrict__ seg_time,
    const double* __restrict__ seg_frac, const double* __restrict__ rate,
    const double* __restrict__ cat_rates, TO* __restrict__ Pout, TO* __restrict__ dPout) {
  extern __shared__ __align__(16) unsigned char smem_raw[];
  const int KK = Kp * Kp;
  const int ipb = (EPT == 1) ? max(1, 256 / KK) : 1;
  const int tid = threadIdx.x;
  const int slot = (EPT == 1) ? tid / KK : 0;
  const bool in_slot = slot < ipb;
  const int item = blockIdx.x * ipb + slot;
  const bool valid = in_slot && item < n_nodes * C;
  // node_list (or null: every node) names the branches whose matrices are formed
  const int v = valid ? (node_list ? node_list[item / C] : item / C) : 0;
  const int c = valid ? item % C : 0;
  T* sX = reinterpret_cast<T*>(smem_raw) + (in_slot ? slot : 0) * KK;
  T* sD = reinterpret_cast<T*>(smem_raw) + ipb * KK + (in_slot ? slot : 0) * KK;
  __shared__ int s_maxm;

  int idx[EPT];
  bool eok[EPT];
#pragma unroll
  for (int e = 0; e < EPT; ++e) {
    idx[e] = (EPT == 1) ? tid % KK : tid + e * 256;
    eok[e] = valid && idx[e] < KK;
  }
  const int seg0 = valid ? seg_offset[v] : 0;
  const int m = valid ? seg_offset[v + 1] - seg0 : 0;
  if constexpr (EPT == 1) {
    if (tid == 0) s_maxm = 0;
    __syncthreads();
    if (valid) atomicMax(&s_maxm, m);
  }
#pragma unroll
  for (int e = 0; e < EPT; ++e)
    if (eok[e]) {
      const int i = idx[e] / Kp, j = idx[e] % Kp;
      sX[idx[e]] = (i == j) ? T(1) : T(0);
      if (GRAD) sD[idx[e]] = T(0);
    }
  __syncthreads();
  int maxm = m;  // one item per block when EPT > 1
  if constexpr (EPT == 1) maxm = s_maxm;
  const double rho = valid ? cat_rates[c] : 0.0;
  for (int k = 0; k < maxm; ++k) {
    const bool act = valid && k < m;
    const int s = act ? seg_process[seg0 + k] : 0;
    const T tau = act ? T(rho * rate[v] * seg_time[seg0 + k]) : T(0);
    const T dsc = act ? T(rho * seg_frac[seg0 + k]) : T(0);
    const T* V = eigV + (size_t)s * KK;
    const T* Vi = eigVi + (size_t)s * KK;
    const T* lr = lre + (size_t)s * Kp;
    const T* li = lim + (size_t)s * Kp;
    T y[EPT], yd[EPT], xold[EPT], dold[EPT];
    // Y = X V, YD = D V
#pragma unroll
    for (int e = 0; e < EPT; ++e) {
      y[e] = 0;
      yd[e] = 0;
      xold[e] = eok[e] ? sX[idx[e]] : T(0);
      dold[e] = (GRAD && eok[e]) ? sD[idx[e]] : T(0);
      if (eok[e] && act) {
        const int i = idx[e] / Kp, j = idx[e] % Kp;
        for (int l = 0; l < Kp; ++l) {
          const T vv = V[l * Kp + j];
          y[e] += sX[i * Kp + l] * vv;
          if (GRAD) yd[e] += sD[i * Kp + l] * vv;
        }
      }
    }
    __syncthreads();
#pragma unroll
    for (int e = 0; e < EPT; ++e)
      if (eok[e] && act) {
        sX[idx[e]] = y[e];
        if (GRAD) sD[idx[e]] = yd[e];
      }
    __syncthreads();
    // X' = Y (E - I), D' = YD (E - I) + Y dE   (dE = dsc * d/dtau E)
#pragma unroll
    for (int e = 0; e < EPT; ++e)
      if (eok[e] && act) {
        const int i = idx[e] / Kp, j = idx[e] % Kp;
        BlockCoef<T> bc = block_coef(lr, li, j, tau);
        const T xs = sX[idx[e]];
        const T xo = bc.partner >= 0 ? sX[i * Kp + bc.partner] : T(0);
        y[e] = bc.m_self * xs + bc.m_other * xo;
        if (GRAD) {
          const T ds = sD[idx[e]];
          const T dd = bc.partner >= 0 ? sD[i * Kp + bc.partner] : T(0);
          yd[e] = bc.m_self * ds + bc.m_other * dd + dsc * (bc.dm_self * xs + bc.dm_other * xo);
        }
      }
    __syncthreads();
#pragma unroll
    for (int e = 0; e < EPT; ++e)
      if (eok[e] && act) {
        sX[idx[e]] = y[e];
        if (GRAD) sD[idx[e]] = yd[e];
      }
    __syncthreads();
    // X = X_old + X' V^-1, D = D_old + D' V^-1
#pragma unroll
    for (int e = 0; e < EPT; ++e) {
      y[e] = xold[e];
      yd[e] = dold[e];
      if (eok[e] && act) {
        const int i = idx[e] / Kp, j = idx[e] % Kp;
        for (int l = 0; l < Kp; ++l) {
          const T vv = Vi[l * Kp + j];
          y[e] += sX[i * Kp + l] * vv;
          if (GRAD) yd[e] += sD[i * Kp + l] * vv;
        }
      }
    }
    __syncthreads();
#pragma unroll
    for (int e = 0; e < EPT; ++e)
      if (eok[e] && act) {
        sX[idx[e]] = y[e];
        if (GRAD) sD[idx[e]] = yd[e];
      }
    __syncthreads();
  }
  const size_t base = ((size_t)v * C + c) * KK;
#pragma unroll
  for (int e = 0; e < EPT; ++e)
    if (eok[e]) {
      Pout[base + idx[e]] = TO(sX[idx[e]]);
      if (GRAD) dPout[base + idx[e]] = TO(sD[idx[e]]);
    }
}

// ---------------------------------------------------------------------------
// Post-order, one level: block = (internal node, tile of 256/KQ patterns);
// thread = (pattern, state).  Children tiles staged through LDS per category.
// ---------------------------------------------------------------------------
// The 0/1 indicator of a tip state code (text after Eq. 4): code < K one state,
// K every state (missing), K + 1 + a the caller's ambiguity set a.
__device__ inline uint64_t tip_set(int st, int K, const uint64_t* __restrict__ amb) {
  if (st < K) return 1ull << st;
  if (st == K) return K == 64 ? ~0ull : ((1ull << K) - 1);
  return amb[st - K - 1];
}

// sum_j M[j * stride] * v[j] over j < n, summed in order of j, with the loads of
// up to 16 terms issued together (the matrix entries are mostly not in cache, so
// one load per step would pay the memory latency n times).
template <typename T>
__device__ inline T dot_strided(const T* __restrict__ M, size_t stride, const T* v, int n) {
  T r = 0;
  int j = 0;
  for (; j + 16 <= n; j += 16) {
    T m[16];
#pragma unroll
    for (int k = 0; k < 16; ++k) m[k] = M[(size_t)(j + k) * stride];
#pragma unroll
    for (int k = 0; k < 16; ++k) r += m[k] * v[j + k];
  }
  if (j + 8 <= n) {
    T m[8];
#pragma unroll
    for (int k = 0; k < 8; ++k) m[k] = M[(size_t)(j + k) * stride];
#pragma unroll
    for (int k = 0; k < 8; ++k) r += m[k] * v[j + k];
    j += 8;
  }
  if (j + 4 <= n) {
    T m[4];
#pragma unroll
    for (int k = 0; k < 4; ++k) m[k] = M[(size_t)(j + k) * stride];
#pragma unroll
    for (int k = 0; k < 4; ++k) r += m[k] * v[j + k];
    j += 4;
  }
  for (; j < n; ++j) r += M[(size_t)j * stride] * v[j];
  return r;
}

template <typename T>
__device__ inline T child_vector(int child, int N, int p, int tstride, int K, int Kp, int i, const T* Prow,
                                 const uint8_t* tips, const uint64_t* amb, const T* sL) {
  // (P_child L_child)(i) for a pattern; Prow points at row i of the child's matrix; tstride is the
  // row stride of the tip states (the instance's pattern count).
  if (child < N) {
    const int st = tips[(size_t)child * tstride + p];
    if (st < K) return Prow[st];
    const uint64_t set = tip_set(st, K, amb);
    T r = 0;
    for (int j = 0; j < K; ++j)
      if ((set >> j) & 1) r += Prow[j];
    return r;
  }
  return dot_strided(Prow, 1, sL, K);
}

template <typename T, int KQ>
__global__ __launch_bounds__(256) void post_level_generic_kernel(
    const int32_t* __restrict__ nodes, const int32_t* __restrict__ left,
    const int32_t* __restrict__ right, const T* __restrict__ Pm, const uint8_t* __restrict__ tips,
    const uint64_t* __restrict__ amb,
    T* __restrict__ partials, int32_t* __restrict__ scales, int N, int P, int tstride, int K, int Kp, int C) {
  constexpr int TP = 256 / KQ;
  __shared__ T sA[256], sB[256];
  const int u = nodes[blockIdx.y];
  const int a = left[u], b = right[u];
  const int pl = threadIdx.x / KQ, i = threadIdx.x % KQ;
  const int p = blockIdx.x * TP + pl;
  const bool pok = p < P;
  const size_t KK = (size_t)Kp * Kp;
  const size_t stride_c = (size_t)P * Kp;
  T x[kMaxCategories];
  for (int c = 0; c < C; ++c) {
    if (a >= N) sA[threadIdx.x] = (pok && i < Kp) ? partials[((size_t)(a - N) * C + c) * stride_c + (size_t)p * Kp + i] : T(0);
    if (b >= N) sB[threadIdx.x] = (pok && i < Kp) ? partials[((size_t)(b - N) * C + c) * stride_c + (size_t)p * Kp + i] : T(0);
    __syncthreads();
    T r = 0;
    if (pok && i < K) {
      const T va = child_vector(a, N, p, tstride, K, Kp, i, Pm + ((size_t)a * C + c) * KK + (size_t)i * Kp, tips, amb, sA + pl * KQ);
      const T vb = child_vector(b, N, p, tstride, K, Kp, i, Pm + ((size_t)b * C + c) * KK + (size_t)i * Kp, tips, amb, sB + pl * KQ);
      r = va * vb;
    }
    x[c] = r;
    __syncthreads();
  }
  T mx = 0;
  for (int c = 0; c < C; ++c) mx = x[c] > mx ? x[c] : mx;
  mx = group_max<KQ>(mx);
  const int e = scale_exponent(mx);
  if (pok && i < Kp)
    for (int c = 0; c < C; ++c)
      partials[((size_t)(u - N) * C + c) * stride_c + (size_t)p * Kp + i] = (i < K) ? scale_by_pow2(x[c], e) : T(0);
  // cumulative exponent of the subtree, so the root needs only its own
  if (pok && i == 0)
    scales[(size_t)(u - N) * P + p] = e + (a >= N ? scales[(size_t)(a - N) * P + p] : 0) +
                                     (b >= N ? scales[(size_t)(b - N) * P + p] : 0);
}

// ---------------------------------------------------------------------------
// Root: thread per pattern.  L_p = sum_c w_c sum_i pi_i x(c, p, i); site logL in
// FP64 with the summed scale exponents; block partial sums of w_p * logL_p.
// ---------------------------------------------------------------------------
template <typename T>
__global__ __launch_bounds__(256) void root_generic_kernel(
    const T* __restrict__ root_part, const int32_t* __restrict__ root_scales,
    const double* __restrict__ pi, const double* __restrict__ cat, const double* __restrict__ weights,
    double* __restrict__ site, double* __restrict__ block_out, int P, int K, int Kp, int C) {
  __shared__ double sm[256];
  const int p = blockIdx.x * 256 + threadIdx.x;
  double contrib = 0.0;
  if (p < P) {
    double L = 0.0;
    for (int c = 0; c < C; ++c) {
      double lc = 0.0;
      const T* x = root_part + ((size_t)c * P + p) * Kp;
      for (int i = 0; i < K; ++i) lc += pi[i] * (double)x[i];
      L += cat[kMaxCategories + c] * lc;
    }
    const double s = log(L) + (double)root_scales[p] * kLn2;
    site[p] = s;
    contrib = weights[p] * s;
  }
  const double tot = block_sum<256>(contrib, sm);
  if (threadIdx.x == 0) block_out[blockIdx.x] = tot;
}

// Ordered single-block sum of n doubles into out[0].
__global__ __launch_bounds__(256) void final_sum_kernel(const double* __restrict__ in, int n,
                                                        double* __restrict__ out) {
  __shared__ double sm[256];
  double acc = 0.0;
  for (int k = threadIdx.x; k < n; k += 256) acc += in[k];
  const double tot = block_sum<256>(acc, sm);
  if (threadIdx.x == 0) out[0] = tot;
}

// Log-likelihoods of pattern chunks 1 .. n (in result[1 .. n]) summed in order into result[0].
__global__ void chunk_sum_kernel(double* __restrict__ result, int n) {
  if (threadIdx.x == 0 && blockIdx.x == 0) {
    double acc = 0.0;
    for (int j = 1; j <= n; ++j) acc += result[j];
    result[0] = acc;
  }
}

// ---------------------------------------------------------------------------
// Pre-order, one level (root downwards): outside vectors of internal children.
//   child a of u (sibling b): t_a = q_u * (P_b L_b);  q_a = P_a^T t_a, rescaled.
// ---------------------------------------------------------------------------
template <typename T, int KQ>
__global__ __launch_bounds__(256) void pre_level_generic_kernel(
    const int32_t* __restrict__ nodes, const int32_t* __restrict__ left,
    const int32_t* __restrict__ right, const T* __restrict__ Pm, const uint8_t* __restrict__ tips,
    const uint64_t* __restrict__ amb,
    const T* __restrict__ partials, T* __restrict__ pre, const double* __restrict__ pi, int root,
    int N, int P, int tstride, int K, int Kp, int C) {
  constexpr int TP = 256 / KQ;
  __shared__ T sQ[256], sA[256], sB[256], sTa[256], sTb[256];
  const int u = nodes[blockIdx.y];
  const int a = left[u], b = right[u];
  if (a < N && b < N) return;
  const int pl = threadIdx.x / KQ, i = threadIdx.x % KQ;
  const int p = blockIdx.x * TP + pl;
  const bool pok = p < P;
  const size_t KK = (size_t)Kp * Kp;
  const size_t stride_c = (size_t)P * Kp;
  T qa[kMaxCategories], qb[kMaxCategories];
  for (int c = 0; c < C; ++c) {
    if (u == root)
      sQ[threadIdx.x] = (i < K) ? T(pi[i]) : T(0);
    else
      sQ[threadIdx.x] = (pok && i < Kp) ? pre[((size_t)(u - N) * C + c) * stride_c + (size_t)p * Kp + i] : T(0);
    if (a >= N) sA[threadIdx.x] = (pok && i < Kp) ? partials[((size_t)(a - N) * C + c) * stride_c + (size_t)p * Kp + i] : T(0);
    if (b >= N) sB[threadIdx.x] = (pok && i < Kp) ? partials[((size_t)(b - N) * C + c) * stride_c + (size_t)p * Kp + i] : T(0);
    __syncthreads();
    T ta = 0, tb = 0;
    if (pok && i < K) {
      const T va = child_vector(a, N, p, tstride, K, Kp, i, Pm + ((size_t)a * C + c) * KK + (size_t)i * Kp, tips, amb, sA + pl * KQ);
      const T vb = child_vector(b, N, p, tstride, K, Kp, i, Pm + ((size_t)b * C + c) * KK + (size_t)i * Kp, tips, amb, sB + pl * KQ);
      const T q = sQ[threadIdx.x];
      ta = q * vb;
      tb = q * va;
    }
    sTa[threadIdx.x] = ta;
    sTb[threadIdx.x] = tb;
    __syncthreads();
    T ra = 0, rb = 0;
    if (pok && i < K) {
      ra = dot_strided(Pm + ((size_t)a * C + c) * KK + i, (size_t)Kp, sTa + pl * KQ, K);
      rb = dot_strided(Pm + ((size_t)b * C + c) * KK + i, (size_t)Kp, sTb + pl * KQ, K);
    }
    qa[c] = ra;
    qb[c] = rb;
    __syncthreads();
  }
  T ma = 0, mb = 0;
  for (int c = 0; c < C; ++c) {
    ma = qa[c] > ma ? qa[c] : ma;
    mb = qb[c] > mb ? qb[c] : mb;
  }
  ma = group_max<KQ>(ma);
  mb = group_max<KQ>(mb);
  const int ea = scale_exponent(ma), eb = scale_exponent(mb);
  if (pok && i < Kp) {
    for (int c = 0; c < C; ++c) {
      if (a >= N) pre[((size_t)(a - N) * C + c) * stride_c + (size_t)p * Kp + i] = (i < K) ? scale_by_pow2(qa[c], ea) : T(0);
      if (b >= N) pre[((size_t)(b - N) * C + c) * stride_c + (size_t)p * Kp + i] = (i < K) ? scale_by_pow2(qb[c], eb) : T(0);
    }
  }
}

// ---------------------------------------------------------------------------
// dlogL/dP per branch: G_v[c](i, j) = sum_p (w_p / Lt_p) w_c t_v(i) L_v(j), with
// Lt_p = sum_c w_c sum_i q_u(i) (P_v L_v)(i) (P_w L_w)(i) formed from the same
// rescaled vectors (every rescaling cancels in the ratio).  Block = (branch,
// pattern chunk); per-chunk partial sums in the compute type, written as FP64.
// ---------------------------------------------------------------------------
template <typename T, int KQ, int GPT>
__global__ __launch_bounds__(256) void grad_G_generic_kernel(
    const int32_t* __restrict__ parent, const int32_t* __restrict__ left,
    const int32_t* __restrict__ right, const T* __restrict__ Pm, const uint8_t* __restrict__ tips,
    const uint64_t* __restrict__ amb,
    const T* __restrict__ partials, const T* __restrict__ pre, const double* __restrict__ pi,
    const double* __restrict__ cat, const double* __restrict__ weights, int root, int N, int n_nodes,
    int P, int tstride, int K, int Kp, int C, int n_chunks, double* __restrict__ Gpart,
    const T* __restrict__ dP, double* __restrict__ G, double* __restrict__ dbranch) {
  // With one partial-sum slot per branch (n_chunks == 1, G != nullptr) the block
  // writes G itself and dlogL/dl = <G, dP/dl> (no separate reduction).
  constexpr int TP = 256 / KQ;
  __shared__ T sQ[256], sV[256], sW[256];
  __shared__ T sAc[kMaxCategories][256];
  __shared__ T sBc[kMaxCategories][256];
  __shared__ double sRed[256];
  const int v = blockIdx.x;
  if (v == root) {  // uniform
    if (G) {
      for (int e = threadIdx.x; e < C * Kp * Kp; e += 256) G[(size_t)v * C * Kp * Kp + e] = 0.0;
      if (threadIdx.x == 0) dbranch[v] = 0.0;
    }
    return;
  }
  const int u = parent[v];
  const int w = (left[u] == v) ? right[u] : left[u];
  const int pl = threadIdx.x / KQ, i = threadIdx.x % KQ;
  const size_t KK = (size_t)Kp * Kp;
  const size_t stride_c = (size_t)P * Kp;
  const int nG = C * Kp * Kp;
  T g[GPT];
#pragma unroll
  for (int k = 0; k < GPT; ++k) g[k] = 0;
  for (int t = blockIdx.y; t * TP < P; t += n_chunks) {
    const int p = t * TP + pl;
    const bool pok = p < P;
    T acc = 0;
    T tv[kMaxCategories];
    for (int c = 0; c < C; ++c) {
      if (u == root)
        sQ[threadIdx.x] = (i < K) ? T(pi[i]) : T(0);
      else
        sQ[threadIdx.x] = (pok && i < Kp) ? pre[((size_t)(u - N) * C + c) * stride_c + (size_t)p * Kp + i] : T(0);
      if (v >= N) sV[threadIdx.x] = (pok && i < Kp) ? partials[((size_t)(v - N) * C + c) * stride_c + (size_t)p * Kp + i] : T(0);
      if (w >= N) sW[threadIdx.x] = (pok && i < Kp) ? partials[((size_t)(w - N) * C + c) * stride_c + (size_t)p * Kp + i] : T(0);
      __syncthreads();
      T lv = 0;  // L_v(i)
      T tvi = 0;
      if (pok && i < K) {
        const T sv = child_vector(v, N, p, tstride, K, Kp, i, Pm + ((size_t)v * C + c) * KK + (size_t)i * Kp, tips, amb, sV + pl * KQ);
        const T sw = child_vector(w, N, p, tstride, K, Kp, i, Pm + ((size_t)w * C + c) * KK + (size_t)i * Kp, tips, amb, sW + pl * KQ);
        const T q = sQ[threadIdx.x];
        tvi = q * sw;
        acc += T(cat[kMaxCategories + c]) * tvi * sv;
        if (v >= N) {
          lv = sV[threadIdx.x];
        } else {
          const int st = tips[(size_t)v * tstride + p];
          lv = ((tip_set(st, K, amb) >> i) & 1) ? T(1) : T(0);
        }
      }
      tv[c] = tvi;
      sBc[c][threadIdx.x] = lv;
      __syncthreads();
    }
    const T Lt = group_sum<KQ>(acc);
    const T coef = (pok && Lt > T(0)) ? T(weights[p]) / Lt : T(0);
    for (int c = 0; c < C; ++c) sAc[c][threadIdx.x] = coef * T(cat[kMaxCategories + c]) * tv[c];
    __syncthreads();
#pragma unroll
    for (int k = 0; k < GPT; ++k) {
      const int e = threadIdx.x + k * 256;
      if (e < nG) {
        const int c = e / (int)KK;
        const int r = e % (int)KK;
        const int ii = r / Kp, jj = r % Kp;
        if (ii < K && jj < K) {
          T s = 0;
#pragma unroll 4
          for (int q = 0; q < TP; ++q) s += sAc[c][q * KQ + ii] * sBc[c][q * KQ + jj];
          g[k] += s;
        }
      }
    }
    __syncthreads();
  }
  if (G) {
    double d = 0.0;
#pragma unroll
    for (int k = 0; k < GPT; ++k) {
      const int e = threadIdx.x + k * 256;
      if (e < nG) {
        G[(size_t)v * nG + e] = (double)g[k];
        d += (double)g[k] * (double)dP[(size_t)v * nG + e];
      }
    }
    d = block_sum<256>(d, sRed);
    if (threadIdx.x == 0) dbranch[v] = d;
    return;
  }
#pragma unroll
  for (int k = 0; k < GPT; ++k) {
    const int e = threadIdx.x + k * 256;
    if (e < nG) Gpart[((size_t)v * n_chunks + blockIdx.y) * nG + e] = (double)g[k];
  }
}

// G[v] = FP64 sum over chunks in a fixed order; d_branch[v] = sum_c <G[v][c], dP[v][c]>.
// Partial sums are laid out [v][chunk][nG]; thread (e, g) of the block sums
// chunks g, g + NG, ... of element e, then the NG groups are combined in order.
template <typename T>
__global__ __launch_bounds__(256) void grad_reduce_branch_kernel(
    const double* __restrict__ Gpart, const T* __restrict__ dP, int n_slots,
    const int32_t* __restrict__ chunks_per_node, int n_nodes, int nG, int root, double* __restrict__ G,
    double* __restrict__ dbranch, int accumulate) {
  __shared__ double sm[256];
  const int v = blockIdx.x;
  const double* src = Gpart + (size_t)v * n_slots * nG;
  const int n_chunks = chunks_per_node ? chunks_per_node[v] : n_slots;
  const int groups = nG >= 256 ? 1 : 256 / nG;  // nG is a multiple of 16
  double d = 0.0;
  for (int e0 = 0; e0 < nG; e0 += 256 / groups) {
    const int e = e0 + threadIdx.x % (256 / groups);
    const int g = threadIdx.x / (256 / groups);
    double s = 0.0;
    if (v != root && e < nG && g < groups)
      for (int k = g; k < n_chunks; k += groups) s += src[(size_t)k * nG + e];
    sm[threadIdx.x] = s;
    __syncthreads();
    if (g == 0 && e < nG) {
      double tot = 0.0;
      for (int q = 0; q < groups; ++q) tot += sm[q * (256 / groups) + threadIdx.x];
      if (accumulate) tot += G[(size_t)v * nG + e];  // earlier pattern chunks
      G[(size_t)v * nG + e] = tot;
      d += tot * (double)dP[(size_t)v * nG + e];
    }
    __syncthreads();
  }
  const double tot = block_sum<256>(d, sm);
  if (threadIdx.x == 0) dbranch[v] = (v == root) ? 0.0 : tot;
}

// ---------------------------------------------------------------------------
// FP64 eigen check: max|V B V^-1 - Q| / max|Q| and max|V V^-1 - I|.
// ---------------------------------------------------------------------------

template <typename T>
const T* eigT_ptr(EpochInstance* in, int which) {
  // which: 0 V, 1 Vinv, 2 lre, 3 lim
  const size_t KK = (size_t)in->Kp * in->Kp;
  const T* base = static_cast<const T*>(in->eigT.ptr);
  switch (which) {
    case 0: return base;
    case 1: return base + in->S * KK;
    case 2: return base + 2 * in->S * KK;
    default: return base + 2 * in->S * KK + (size_t)in->S * in->Kp;
  }
}

int lanes_per_pattern(int Kp) {
  int q = 4;
  while (q < Kp) q <<= 1;
  return q;
}

// T: arithmetic of the eigen reconstruction and chain products; TO: storage type
// of the transition matrices handed to pruning.
template <typename T, typename TO>
int pstage_dispatch(EpochInstance* in, const int32_t* d_nodes, int n_list) {
  const int Kp = in->Kp, KK = Kp * Kp, C = in->C, n = d_nodes ? n_list : in->n_nodes;
  const bool grad = (in->cfg.flags & (EPOCH_GRAD_BRANCH | EPOCH_GRAD_Q)) != 0;
  const int ept = KK <= 256 ? 1 : (KK + 255) / 256;
  const int ipb = ept == 1 ? std::max(1, 256 / KK) : 1;
  const int items = n * C;
  dim3 grid((items + ipb - 1) / ipb);
  const size_t shm = 2 * (size_t)ipb * KK * sizeof(T);
  const T* base = static_cast<const T*>(sizeof(T) == 8 ? in->eig64.ptr : in->eigT.ptr);
  const size_t S = in->S;
  const T* V = base;
  const T* Vi = base + S * KK;
  const T* lr = base + 2 * S * KK;
  const T* li = lr + S * Kp;
  const double* cat = static_cast<const double*>(in->cat.ptr);
  TO* Pout = static_cast<TO*>(in->Pm.ptr);
  TO* dPout = static_cast<TO*>(in->dPm.ptr);
#define EPOCH_PSTAGE(G, E)                                                                      \
  hipLaunchKernelGGL((pstage_generic_kernel<T, TO, G, E>), grid, dim3(256), shm, in->stream, n, d_nodes, Kp, C, \
                     V, Vi, lr, li, in->d_seg_offset, in->d_seg_process, in->d_seg_time,        \
                     in->d_seg_frac, in->d_rate, cat, Pout, dPout)
  if (ept == 1) {
    if (grad) EPOCH_PSTAGE(true, 1); else EPOCH_PSTAGE(false, 1);
  } else if (ept <= 4) {
    if (grad) EPOCH_PSTAGE(true, 4); else EPOCH_PSTAGE(false, 4);
  } else if (ept <= 9) {
    if (grad) EPOCH_PSTAGE(true, 9); else EPOCH_PSTAGE(false, 9);
  } else {
    if (grad) EPOCH_PSTAGE(true, 16); else EPOCH_PSTAGE(false, 16);
  }
#undef EPOCH_PSTAGE
  return hip_check(hipGetLastError(), "pstage_generic launch");
}

// The pattern chunk the launches below work on (all patterns unless a chunk
// is selected under an HBM budget): count, first pattern, and the slot of its
// log-likelihood in result.
int view_P(const EpochInstance* in) { return in->view_P > 0 ? in->view_P : in->P; }
size_t view_p0(const EpochInstance* in) { return in->view_P > 0 ? (size_t)in->view_p0 : 0; }
size_t view_result(const EpochInstance* in) { return in->view_P > 0 ? 1 + (size_t)in->view_j : 0; }

// level l's nodes are nodes[level_off[l] .. level_off[l + 1]) (the plan's level lists, or a
// restricted list of the same layout)
template <typename T>
int post_dispatch(EpochInstance* in, const int32_t* d_nodes, const int32_t* level_off) {
  const int KQ = lanes_per_pattern(in->Kp);
  const int TP = 256 / KQ;
  const auto& pl = in->plan;
  const T* Pm = static_cast<const T*>(in->Pm.ptr);
  const uint8_t* tips = static_cast<const uint8_t*>(in->tips.ptr) + view_p0(in);
  const uint64_t* amb = static_cast<const uint64_t*>(in->amb.ptr);
  T* part = static_cast<T*>(in->partials.ptr);
  int32_t* sc = static_cast<int32_t*>(in->scales.ptr);
  const int P = view_P(in);
  for (int l = 1; l <= pl.n_levels; ++l) {
    const int n_l = level_off[l + 1] - level_off[l];
    if (n_l == 0) continue;
    dim3 grid((P + TP - 1) / TP, n_l);
    const int32_t* nodes = d_nodes + level_off[l];
#define EPOCH_POST(Q)                                                                            \
  hipLaunchKernelGGL((post_level_generic_kernel<T, Q>), grid, dim3(256), 0, in->stream, nodes,    \
                     in->d_left, in->d_right, Pm, tips, amb, part, sc, in->N, P, in->P, in->K, in->Kp, in->C)
    switch (KQ) {
      case 4: EPOCH_POST(4); break;
      case 8: EPOCH_POST(8); break;
      case 16: EPOCH_POST(16); break;
      case 32: EPOCH_POST(32); break;
      default: EPOCH_POST(64); break;
    }
#undef EPOCH_POST
  }
  return hip_check(hipGetLastError(), "post_level_generic launch");
}

template <typename T>
int root_dispatch(EpochInstance* in) {
  const int P = view_P(in);
  const size_t p0 = view_p0(in);
  const int nb = (P + 255) / 256;
  const T* rootp = static_cast<const T*>(in->partials.ptr) +
                   (size_t)(in->plan.root - in->N) * in->C * (size_t)P * in->Kp;
  double* blk = static_cast<double*>(in->blocksum.ptr);
  hipLaunchKernelGGL((root_generic_kernel<T>), dim3(nb), dim3(256), 0, in->stream, rootp,
                     static_cast<const int32_t*>(in->scales.ptr) + (size_t)(in->plan.root - in->N) * P,
                     static_cast<const double*>(in->pi.ptr), static_cast<const double*>(in->cat.ptr),
                     static_cast<const double*>(in->weights.ptr) + p0, static_cast<double*>(in->site.ptr) + p0,
                     blk, P, in->K, in->Kp, in->C);
  hipLaunchKernelGGL(final_sum_kernel, dim3(1), dim3(256), 0, in->stream, blk, nb,
                     static_cast<double*>(in->result.ptr) + view_result(in));
  return hip_check(hipGetLastError(), "root_generic launch");
}

template <typename T>
int pre_dispatch(EpochInstance* in) {
  const int KQ = lanes_per_pattern(in->Kp);
  const int TP = 256 / KQ;
  const auto& pl = in->plan;
  const T* Pm = static_cast<const T*>(in->Pm.ptr);
  const uint8_t* tips = static_cast<const uint8_t*>(in->tips.ptr) + view_p0(in);
  const uint64_t* amb = static_cast<const uint64_t*>(in->amb.ptr);
  const T* part = static_cast<const T*>(in->partials.ptr);
  T* pre = static_cast<T*>(in->pre.ptr);
  const double* pi = static_cast<const double*>(in->pi.ptr);
  const int P = view_P(in);
  for (int l = pl.n_levels; l >= 1; --l) {
    const int n_l = pl.level_offset[l + 1] - pl.level_offset[l];
    if (n_l == 0) continue;
    dim3 grid((P + TP - 1) / TP, n_l);
    const int32_t* nodes = in->d_level_nodes + pl.level_offset[l];
#define EPOCH_PRE(Q)                                                                            \
  hipLaunchKernelGGL((pre_level_generic_kernel<T, Q>), grid, dim3(256), 0, in->stream, nodes,    \
                     in->d_left, in->d_right, Pm, tips, amb, part, pre, pi, pl.root, in->N, P, in->P,  \
                     in->K, in->Kp, in->C)
    switch (KQ) {
      case 4: EPOCH_PRE(4); break;
      case 8: EPOCH_PRE(8); break;
      case 16: EPOCH_PRE(16); break;
      case 32: EPOCH_PRE(32); break;
      default: EPOCH_PRE(64); break;
    }
#undef EPOCH_PRE
  }
  return hip_check(hipGetLastError(), "pre_level_generic launch");
}

template <typename T, int KQ, int GP>
void grad_G_launch(EpochInstance* in, dim3 grid, bool fused) {
  const T* Pm = static_cast<const T*>(in->Pm.ptr);
  const uint8_t* tips = static_cast<const uint8_t*>(in->tips.ptr) + view_p0(in);
  const uint64_t* amb = static_cast<const uint64_t*>(in->amb.ptr);
  const T* part = static_cast<const T*>(in->partials.ptr);
  const T* pre = static_cast<const T*>(in->pre.ptr);
  const double* pi = static_cast<const double*>(in->pi.ptr);
  const double* cat = static_cast<const double*>(in->cat.ptr);
  const double* wts = static_cast<const double*>(in->weights.ptr) + view_p0(in);
  double* Gp = static_cast<double*>(in->Gpart.ptr);
  hipLaunchKernelGGL((grad_G_generic_kernel<T, KQ, GP>), grid, dim3(256), 0, in->stream,
                     in->d_parent, in->d_left, in->d_right, Pm, tips, amb, part, pre, pi, cat, wts,
                     in->plan.root, in->N, in->n_nodes, view_P(in), in->P, in->K, in->Kp, in->C, in->n_chunks, Gp,
                     static_cast<const T*>(in->dPm.ptr), fused ? static_cast<double*>(in->G.ptr) : nullptr,
                     static_cast<double*>(in->dbranch.ptr));
}

template <typename T>
int grad_branch_dispatch(EpochInstance* in) {
  const int KQ = lanes_per_pattern(in->Kp);
  const int nG = in->C * in->Kp * in->Kp;
  const int gpt = (nG + 255) / 256;
  if (gpt > 64) return set_error(EPOCH_ERR_ARG, "generic gradient supports C*Kp*Kp <= 16384");
  dim3 grid(in->n_nodes, in->n_chunks);
  // one slot per branch and nothing to accumulate: the gradient kernel finishes G and dlogL/dl itself
  const bool fused = in->n_chunks == 1 && !in->view_accumulate;
  // lanes per pattern fix Kp, so only these (KQ, elements per thread) pairs occur
  switch (KQ) {
    case 4: grad_G_launch<T, 4, 1>(in, grid, fused); break;
    case 8: grad_G_launch<T, 8, 4>(in, grid, fused); break;
    case 16: grad_G_launch<T, 16, 16>(in, grid, fused); break;
    case 32: grad_G_launch<T, 32, 32>(in, grid, fused); break;
    default:
      if (gpt <= 16) grad_G_launch<T, 64, 16>(in, grid, fused);
      else grad_G_launch<T, 64, 64>(in, grid, fused);
      break;
  }
  int rc = hip_check(hipGetLastError(), "grad_G_generic launch");
  if (rc || fused) return rc;
  return launch_grad_reduce(in, in->n_chunks, nullptr);
}

template <typename T>
int grad_reduce_dispatch(EpochInstance* in, int n_slots, const int32_t* chunks_per_node) {
  const int nG = in->C * in->Kp * in->Kp;
  hipLaunchKernelGGL((grad_reduce_branch_kernel<T>), dim3(in->n_nodes), dim3(256), 0, in->stream,
                     static_cast<const double*>(in->Gpart.ptr), static_cast<const T*>(in->dPm.ptr),
                     n_slots, chunks_per_node, in->n_nodes, nG, in->plan.root,
                     static_cast<double*>(in->G.ptr), static_cast<double*>(in->dbranch.ptr),
                     in->view_accumulate ? 1 : 0);
  return hip_check(hipGetLastError(), "grad_reduce_branch launch");
}

}  // namespace


int launch_final_sum(EpochInstance* in, int n_blocks) {
  hipLaunchKernelGGL(final_sum_kernel, dim3(1), dim3(256), 0, in->stream,
                     static_cast<const double*>(in->blocksum.ptr), n_blocks,
                     static_cast<double*>(in->result.ptr));
  return hip_check(hipGetLastError(), "final_sum launch");
}

int launch_chunk_sum(EpochInstance* in, int n) {
  hipLaunchKernelGGL(chunk_sum_kernel, dim3(1), dim3(64), 0, in->stream, static_cast<double*>(in->result.ptr), n);
  return hip_check(hipGetLastError(), "chunk_sum launch");
}

int launch_grad_reduce(EpochInstance* in, int n_slots, const int32_t* chunks_per_node) {
  return in->fp64 ? grad_reduce_dispatch<double>(in, n_slots, chunks_per_node)
                  : grad_reduce_dispatch<float>(in, n_slots, chunks_per_node);
}

int launch_pstage_generic(EpochInstance* in) { return launch_pstage_generic_nodes(in, nullptr, 0); }
int launch_pstage_generic_nodes(EpochInstance* in, const int32_t* d_nodes, int n) {
  if (in->fp64) return pstage_dispatch<double, double>(in, d_nodes, n);
  return in->eig_fp64 ? pstage_dispatch<double, float>(in, d_nodes, n) : pstage_dispatch<float, float>(in, d_nodes, n);
}
int launch_post_generic(EpochInstance* in) {
  return launch_post_generic_nodes(in, in->d_level_nodes, in->plan.level_offset.data());
}
int launch_post_generic_nodes(EpochInstance* in, const int32_t* d_nodes, const int32_t* level_off) {
  return in->fp64 ? post_dispatch<double>(in, d_nodes, level_off) : post_dispatch<float>(in, d_nodes, level_off);
}
int launch_root_generic(EpochInstance* in) {
  return in->fp64 ? root_dispatch<double>(in) : root_dispatch<float>(in);
}
int launch_pre_generic(EpochInstance* in) {
  return in->fp64 ? pre_dispatch<double>(in) : pre_dispatch<float>(in);
}
int launch_grad_branch_generic(EpochInstance* in) {
  return in->fp64 ? grad_branch_dispatch<double>(in) : grad_branch_dispatch<float>(in);
}

}  // namespace epochlik
