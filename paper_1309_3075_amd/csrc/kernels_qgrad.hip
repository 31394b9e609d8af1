// dlogL/dQ_s: adjoint of the ordered product of exponentials.
//
// For a branch with factors F_0 .. F_{m-1} (parent side first) and
// G = dlogL/dP, the adjoint of factor k is G_k = A_k^T G B_k^T with
// A_k = F_0..F_{k-1} and B_k = F_{k+1}..F_{m-1}.  With F_k = exp(X_k),
// X_k = tau_k Q_s, tau_k = rho_c r_b t_bk and Q_s = Vc diag(lambda) Vc^-1
// (complex eigenvectors Vc = V T, V the real form passed in), the adjoint
// Frechet derivative of exp gives
//   dlogL/dQ_s += tau_k Vc^-T [ Phi(tau_k lambda) o (Vc^T G_k Vc^-T) ] Vc^T,
//   Phi_ij = (e^{x_i} - e^{x_j}) / (x_i - x_j)  (e^{x_i} when x_i = x_j).
// Per-segment terms W_k = tau_k Phi o (T^T (V^T G_k V^-T) T^-T) are written in
// FP64 complex; a second kernel sums them per process in a fixed order and
// maps back with V^-T T^-T (.) T^T V^T.
#include <hip/hip_runtime.h>

#include <cmath>

#include "device_common.h"
#include "eigen_block.h"
#include "instance.h"
#include "mfma_chain.h"

namespace epochlik {

namespace {

struct cplx {
  double re, im;
};
__device__ inline cplx cmul(cplx a, cplx b) { return {a.re * b.re - a.im * b.im, a.re * b.im + a.im * b.re}; }
__device__ inline cplx cdiv(cplx a, cplx b) {
  const double inv = 1.0 / (b.re * b.re + b.im * b.im);
  return {(a.re * b.re + a.im * b.im) * inv, (a.im * b.re - a.re * b.im) * inv};
}
// e^z - 1 without cancellation for small |z|
__device__ inline cplx cexpm1(cplx z) {
  const double sh = sin(0.5 * z.im);
  return {expm1(z.re) * cos(z.im) - 2.0 * sh * sh, exp(z.re) * sin(z.im)};
}
__device__ inline cplx cexp(cplx z) {
  const double e = exp(z.re);
  return {e * cos(z.im), e * sin(z.im)};
}
// (e^a - e^b) / (a - b), and e^a when a == b
__device__ inline cplx divided_difference_exp(cplx a, cplx b) {
  cplx d = {a.re - b.re, a.im - b.im};
  cplx eb = cexp(b);
  if (d.re == 0.0 && d.im == 0.0) return eb;
  return cmul(eb, cdiv(cexpm1(d), d));
}

// Column-pairing of the real eigen form: entries of T (Vc = V T) and T^-1.
//   real j:        T[j][j] = 1,                       Tinv[j][j] = 1
//   pair (j, j+1): T = [[1, 1], [i, -i]],             Tinv = [[1/2, -i/2], [1/2, i/2]]
struct PairIdx {
  int first;  // first column of the 2x2 block containing the index (== index if real)
  bool pair;
};
template <typename T>
__device__ inline PairIdx pair_of(const T* li, int j) {
  const T b = li[j];
  if (b == T(0)) return {j, false};
  return {b > T(0) ? j : j - 1, true};
}
__device__ inline cplx T_entry(int row, int col, int first, bool pair) {
  if (!pair) return {row == col ? 1.0 : 0.0, 0.0};
  const int r = row - first, c = col - first;
  if (r == 0) return {1.0, 0.0};
  return c == 0 ? cplx{0.0, 1.0} : cplx{0.0, -1.0};
}
__device__ inline cplx Tinv_entry(int row, int col, int first, bool pair) {
  if (!pair) return {row == col ? 1.0 : 0.0, 0.0};
  const int r = row - first, c = col - first;
  if (c == 0) return {0.5, 0.0};
  return r == 0 ? cplx{0.0, -0.5} : cplx{0.0, 0.5};
}

template <typename T, int EPT>
__device__ inline void store_regs(T* s, const T* y, const int* idx, const bool* ok) {
#pragma unroll
  for (int e = 0; e < EPT; ++e)
    if (ok[e]) s[idx[e]] = y[e];
}

// X <- X F(tau) (transposed = false) or X <- X F(tau)^T (transposed = true), with
// F = I + V (E - I) V^-1, using sX (LDS) and registers.
template <typename T, int EPT>
__device__ void apply_factor(T* sX, const T* V, const T* Vi, const T* lr, const T* li, T tau, int Kp,
                             const int* idx, const bool* ok, bool transposed) {
  T y[EPT], xold[EPT];
  // first multiply: X V (plain) or X V^-T (transposed)
#pragma unroll
  for (int e = 0; e < EPT; ++e) {
    y[e] = 0;
    xold[e] = ok[e] ? sX[idx[e]] : T(0);
    if (ok[e]) {
      const int i = idx[e] / Kp, j = idx[e] % Kp;
      for (int l = 0; l < Kp; ++l) y[e] += sX[i * Kp + l] * (transposed ? Vi[j * Kp + l] : V[l * Kp + j]);
    }
  }
  __syncthreads();
  store_regs<T, EPT>(sX, y, idx, ok);
  __syncthreads();
  // middle: E - I (plain) or (E - I)^T (transposed: the rotation angle changes sign)
#pragma unroll
  for (int e = 0; e < EPT; ++e) {
    y[e] = 0;
    if (ok[e]) {
      const int i = idx[e] / Kp, j = idx[e] % Kp;
      const T b = li[j];
      if (b == T(0)) {
        y[e] = sX[idx[e]] * dev_expm1(lr[j] * tau);
      } else {
        const bool first = b > T(0);
        const T bb = first ? b : -b;
        const T em1 = dev_expm1(lr[j] * tau);
        const T ea = em1 + T(1), cs = dev_cos(bb * tau), sn = dev_sin(bb * tau);
        const T hs = dev_sin(T(0.5) * bb * tau);
        const int jp = first ? j + 1 : j - 1;
        // plain:   first: ea(c x_j - s x_p), second: ea(s x_p + c x_j)
        // transp.: first: ea(c x_j + s x_p), second: ea(-s x_p + c x_j); minus x_j for E - I
        const T sgn = (first ? T(-1) : T(1)) * (transposed ? T(-1) : T(1));
        y[e] = (em1 * cs - T(2) * hs * hs) * sX[idx[e]] + sgn * ea * sn * sX[i * Kp + jp];
      }
    }
  }
  __syncthreads();
  store_regs<T, EPT>(sX, y, idx, ok);
  __syncthreads();
  // last multiply: V^-1 (plain) or V^T (transposed), plus the identity part
#pragma unroll
  for (int e = 0; e < EPT; ++e) {
    y[e] = xold[e];
    if (ok[e]) {
      const int i = idx[e] / Kp, j = idx[e] % Kp;
      for (int l = 0; l < Kp; ++l) y[e] += sX[i * Kp + l] * (transposed ? V[j * Kp + l] : Vi[l * Kp + j]);
    }
  }
  __syncthreads();
  store_regs<T, EPT>(sX, y, idx, ok);
  __syncthreads();
}

// One block per (node v, category c).
template <typename T, int EPT>
__global__ __launch_bounds__(256) void qgrad_segments_kernel(
    int n_nodes, int root, int Kp, int C, const T* __restrict__ eigV, const T* __restrict__ eigVi,
    const T* __restrict__ lre, const T* __restrict__ lim, const int32_t* __restrict__ seg_offset,
    const int32_t* __restrict__ seg_process, const double* __restrict__ seg_time,
    const double* __restrict__ rate, const double* __restrict__ cat_rates,
    const double* __restrict__ G, T* __restrict__ prefix, double* __restrict__ Wout) {
  extern __shared__ __align__(16) unsigned char smem_raw[];
  const int KK = Kp * Kp;
  T* sR = reinterpret_cast<T*>(smem_raw);
  T* sW = sR + KK;
  const int v = blockIdx.x / C, c = blockIdx.x % C;
  if (v >= n_nodes || v == root) return;
  const int seg0 = seg_offset[v];
  const int m = seg_offset[v + 1] - seg0;
  if (m == 0) return;
  int idx[EPT];
  bool ok[EPT];
#pragma unroll
  for (int e = 0; e < EPT; ++e) {
    idx[e] = threadIdx.x + e * 256;
    ok[e] = idx[e] < KK;
  }
  const double scale = cat_rates[c] * rate[v];
  // forward: prefix products A_k (A_0 = I) stored per segment
#pragma unroll
  for (int e = 0; e < EPT; ++e)
    if (ok[e]) sW[idx[e]] = (idx[e] / Kp == idx[e] % Kp) ? T(1) : T(0);
  __syncthreads();
  for (int k = 0; k < m; ++k) {
    T* A = prefix + ((size_t)(seg0 + k) * C + c) * KK;
#pragma unroll
    for (int e = 0; e < EPT; ++e)
      if (ok[e]) A[idx[e]] = sW[idx[e]];
    if (k + 1 < m) {
      const int s = seg_process[seg0 + k];
      apply_factor<T, EPT>(sW, eigV + (size_t)s * KK, eigVi + (size_t)s * KK, lre + (size_t)s * Kp,
                           lim + (size_t)s * Kp, T(scale * seg_time[seg0 + k]), Kp, idx, ok, false);
    }
  }
  __syncthreads();
  // backward: R = G B_k^T, starting from R = G
  const double* Gv = G + ((size_t)v * C + c) * KK;
#pragma unroll
  for (int e = 0; e < EPT; ++e)
    if (ok[e]) sR[idx[e]] = T(Gv[idx[e]]);
  __syncthreads();
  for (int k = m - 1; k >= 0; --k) {
    const int s = seg_process[seg0 + k];
    const double tau_d = scale * seg_time[seg0 + k];
    const T* V = eigV + (size_t)s * KK;
    const T* Vi = eigVi + (size_t)s * KK;
    const T* lr = lre + (size_t)s * Kp;
    const T* li = lim + (size_t)s * Kp;
    const T* A = prefix + ((size_t)(seg0 + k) * C + c) * KK;
    T y[EPT];
    // G_k = A_k^T R
#pragma unroll
    for (int e = 0; e < EPT; ++e) {
      y[e] = 0;
      if (ok[e]) {
        const int i = idx[e] / Kp, j = idx[e] % Kp;
        for (int l = 0; l < Kp; ++l) y[e] += A[l * Kp + i] * sR[l * Kp + j];
      }
    }
    store_regs<T, EPT>(sW, y, idx, ok);
    __syncthreads();
    // Y1 = V^T G_k
#pragma unroll
    for (int e = 0; e < EPT; ++e) {
      y[e] = 0;
      if (ok[e]) {
        const int i = idx[e] / Kp, j = idx[e] % Kp;
        for (int l = 0; l < Kp; ++l) y[e] += V[l * Kp + i] * sW[l * Kp + j];
      }
    }
    __syncthreads();
    store_regs<T, EPT>(sW, y, idx, ok);
    __syncthreads();
    // Y = Y1 V^-T
#pragma unroll
    for (int e = 0; e < EPT; ++e) {
      y[e] = 0;
      if (ok[e]) {
        const int i = idx[e] / Kp, j = idx[e] % Kp;
        for (int l = 0; l < Kp; ++l) y[e] += sW[i * Kp + l] * Vi[j * Kp + l];
      }
    }
    __syncthreads();
    store_regs<T, EPT>(sW, y, idx, ok);
    __syncthreads();
    // W = tau Phi o (T^T Y T^-T), in FP64 complex
    double2* Wk = reinterpret_cast<double2*>(Wout) + ((size_t)(seg0 + k) * C + c) * KK;
#pragma unroll
    for (int e = 0; e < EPT; ++e)
      if (ok[e]) {
        const int a = idx[e] / Kp, b = idx[e] % Kp;
        const PairIdx pa = pair_of(li, a), pb = pair_of(li, b);
        cplx z = {0.0, 0.0};
        const int na = pa.pair ? 2 : 1, nb = pb.pair ? 2 : 1;
        for (int ci = 0; ci < na; ++ci) {
          const int cc = pa.first + ci;
          const cplx t1 = T_entry(cc, a, pa.first, pa.pair);
          for (int di = 0; di < nb; ++di) {
            const int dd = pb.first + di;
            const cplx t2 = Tinv_entry(b, dd, pb.first, pb.pair);
            const cplx yv = {(double)sW[cc * Kp + dd], 0.0};
            const cplx term = cmul(cmul(t1, yv), t2);
            z.re += term.re;
            z.im += term.im;
          }
        }
        const cplx xa = {tau_d * (double)lr[a], tau_d * (double)li[a]};
        const cplx xb = {tau_d * (double)lr[b], tau_d * (double)li[b]};
        const cplx phi = divided_difference_exp(xa, xb);
        const cplx wv = cmul(phi, z);
        Wk[idx[e]] = make_double2(tau_d * wv.re, tau_d * wv.im);
      }
    // R <- R F_k^T
    if (k > 0)
      apply_factor<T, EPT>(sR, V, Vi, lr, li, T(tau_d), Kp, idx, ok, true);
  }
}

// One block per process s: H = sum of its segment terms (fixed order), then
// dQ_s = V^-T (T^-T H T^T) V^T in FP64.
template <int EPT>
__global__ __launch_bounds__(256) void qgrad_reduce_kernel(
    int K, int Kp, int C, const int32_t* __restrict__ list_off, const int32_t* __restrict__ list,
    const double* __restrict__ W, const double* __restrict__ V, const double* __restrict__ Vi,
    const double* __restrict__ li_all, double* __restrict__ Hbuf, double* __restrict__ dQ) {
  extern __shared__ __align__(16) unsigned char smem_raw[];
  double* sX = reinterpret_cast<double*>(smem_raw);
  const int s = blockIdx.x;
  const int KK = Kp * Kp;
  const double* Vs = V + (size_t)s * KK;
  const double* Vis = Vi + (size_t)s * KK;
  const double* li = li_all + (size_t)s * Kp;
  double2* H = reinterpret_cast<double2*>(Hbuf) + (size_t)s * KK;
  const double2* W2 = reinterpret_cast<const double2*>(W);
  const int b0 = list_off[s], b1 = list_off[s + 1];
  for (int e = threadIdx.x; e < KK; e += 256) {
    double re = 0.0, im = 0.0;
    for (int q = b0; q < b1; ++q) {
      const double2 w = W2[(size_t)list[q] * KK + e];  // list holds (segment * C + c)
      re += w.x;
      im += w.y;
    }
    H[e] = make_double2(re, im);
  }
  __threadfence_block();
  __syncthreads();
  // X = T^-T H T^T (real part; the imaginary part vanishes up to rounding)
  for (int e = threadIdx.x; e < KK; e += 256) {
    const int a = e / Kp, b = e % Kp;
    const PairIdx pa = pair_of(li, a), pb = pair_of(li, b);
    const int na = pa.pair ? 2 : 1, nb = pb.pair ? 2 : 1;
    double re = 0.0;
    for (int ci = 0; ci < na; ++ci) {
      const int cc = pa.first + ci;
      const cplx t1 = Tinv_entry(cc, a, pa.first, pa.pair);
      for (int di = 0; di < nb; ++di) {
        const int dd = pb.first + di;
        const cplx t2 = T_entry(b, dd, pb.first, pb.pair);
        const double2 h = H[cc * Kp + dd];
        const cplx term = cmul(cmul(t1, cplx{h.x, h.y}), t2);
        re += term.re;
      }
    }
    sX[e] = re;
  }
  __syncthreads();
  double y[EPT];
  // Y = V^-T X
#pragma unroll
  for (int k = 0; k < EPT; ++k) {
    const int e = threadIdx.x + k * 256;
    y[k] = 0.0;
    if (e < KK) {
      const int i = e / Kp, j = e % Kp;
      for (int l = 0; l < Kp; ++l) y[k] += Vis[l * Kp + i] * sX[l * Kp + j];
    }
  }
  __syncthreads();
#pragma unroll
  for (int k = 0; k < EPT; ++k) {
    const int e = threadIdx.x + k * 256;
    if (e < KK) sX[e] = y[k];
  }
  __syncthreads();
  // dQ = Y V^T, unpadded output [S][K][K]
#pragma unroll
  for (int k = 0; k < EPT; ++k) {
    const int e = threadIdx.x + k * 256;
    if (e < KK) {
      const int i = e / Kp, j = e % Kp;
      if (i < K && j < K) {
        double r = 0.0;
        for (int l = 0; l < Kp; ++l) r += sX[i * Kp + l] * Vs[j * Kp + l];
        dQ[((size_t)s * K + i) * K + j] = r;
      }
    }
  }
}

// ---------------------------------------------------------------------------
// Matrix-core form (padded K a multiple of 16).  With U_k = A_k V_s and
// W_k = R_k V_s^-T, where R_k = G B_k^T, the real-basis adjoint of segment k is
//   Y_k = V_s^T G_k V_s^-T = U_k^T W_k.
// One block per (branch, category), one wavefront per 16-row stripe.  The
// forward chain is the P stage's: it stores U_k = A_k V (its first product of
// each step) in a global scratch buffer.  The backward chain
// R_{k-1} = R_k + (W_k (E_k - I)^T) V^T keeps its stripes in registers (the
// layout of the P-stage kernel); Y_k contracts over all rows, so U_k and W_k
// meet in LDS and each wavefront writes 16 rows of Y_k.  The transposed factors V^T and
// V^-T are read as rows of host-transposed copies.
template <typename T, int NT>
__global__ __launch_bounds__(256) void qgrad_chain_kernel(
    int C, int root, const T* __restrict__ eigV, const T* __restrict__ eigVi, const T* __restrict__ eigVT,
    const T* __restrict__ eigViT, const T* __restrict__ lre, const T* __restrict__ lim,
    const int32_t* __restrict__ seg_offset, const int32_t* __restrict__ seg_process,
    const int4* __restrict__ items, const T* __restrict__ chain_scratch, const double* __restrict__ seg_time,
    const double* __restrict__ rate,
    const double* __restrict__ cat_rates, const double* __restrict__ G, T* __restrict__ Ubuf,
    double* __restrict__ Yseg, double* __restrict__ qtau,
    const double* __restrict__ lr64, const double* __restrict__ li64, double* __restrict__ qexp) {
  using acc = typename Mfma<T>::acc;
  constexpr int Kp = 16 * NT, KK = Kp * Kp, LD = Kp + 1;
  __shared__ T sU[Kp * LD];
  __shared__ T sW[Kp * LD];
  __shared__ T s_coef[NT][2 * 64][2];
  // work item: a node's whole chain, or the head or tail half of a long one, longest first
  const int4 wi = items[blockIdx.x / C];
  const int v = wi.x, c = blockIdx.x - (blockIdx.x / C) * C;
  const int k0 = wi.y, k1 = wi.z, kind = wi.w & 3, part = (wi.w >> 2) & 7, parts = (wi.w >> 5) & 15;
  if (v == root) return;
  const int seg0 = seg_offset[v];
  if (k1 == k0) return;  // uniform over the block
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  const int g = lane >> 4, n = lane & 15;
  const int row = 16 * w + n;
  const int arow = Mfma<T>::a_row(n);
  const double scale = cat_rates[c] * rate[v];
  T(*coef)[2] = s_coef[w];

  // tau and e^{tau lambda} of every segment term, for the divided differences of the sums;
  // the forward products A_k V were stored by the P stage
  for (int k = k0; k < k1; ++k) {
    const int s = seg_process[seg0 + k];
    const double tau_d = scale * seg_time[seg0 + k];
    if (threadIdx.x == 0) qtau[(size_t)(seg0 + k) * C + c] = tau_d;
    if (w == 0 && lane < Kp) {
      const double ea = exp(tau_d * lr64[(size_t)s * Kp + lane]);
      const double th = tau_d * li64[(size_t)s * Kp + lane];
      reinterpret_cast<double2*>(qexp)[((size_t)(seg0 + k) * C + c) * Kp + lane] = make_double2(ea * cos(th), ea * sin(th));
    }
  }

  // backward pass from R = G (rows of this stripe); part j < J - 1 of a split chain
  // starts from G S_j^T, S_j = X_{j+1} .. X_{J-1} being the product of the later parts' factors
  acc R[1][NT];
  {
    const double* Gr = G + ((size_t)v * C + c) * KK + (size_t)row * Kp + 4 * g;
#pragma unroll
    for (int mt = 0; mt < NT; ++mt)
#pragma unroll
      for (int q = 0; q < 4; ++q) R[0][mt][q] = T(Gr[16 * mt + q]);
    if (kind == 1 && part < parts - 1) {
      const T* XBT = chain_scratch + ((((size_t)(wi.w >> 9) * C + c) * kChainMaxParts + part) * 5 + 4) * KK;
      acc R1[1][NT];
#pragma unroll
      for (int mt = 0; mt < NT; ++mt) R1[0][mt] = acc{0, 0, 0, 0};
      stripe_gemm<T, NT, 1>(XBT, g, arow, R, R1);
#pragma unroll
      for (int mt = 0; mt < NT; ++mt) R[0][mt] = R1[0][mt];
    }
  }
  // Segment k - 1's column coefficients, U rows and first V^-T operands are
  // produced while the matrix cores run segment k (coefficients double-buffered
  // by k parity).
  auto make_coef = [&](int k) {
    if (k > k0 && lane < Kp) {
      const int s = seg_process[seg0 + k];
      const BlockCoef<T> bc = block_coef(lre + (size_t)s * Kp, lim + (size_t)s * Kp, lane, T(scale * seg_time[seg0 + k]));
      coef[64 * (k & 1) + lane][0] = bc.m_self;
      coef[64 * (k & 1) + lane][1] = -bc.m_other;
    }
  };
  auto load_u = [&](int k, T (&u)[NT][4]) {
    const T* U = Ubuf + ((size_t)(seg0 + k) * C + c) * KK + (size_t)row * Kp + 4 * g;
#pragma unroll
    for (int mt = 0; mt < NT; ++mt)
#pragma unroll
      for (int q = 0; q < 4; ++q) u[mt][q] = U[16 * mt + q];
  };
  T aw[2][4][NT], av[2][4][NT], u[NT][4], un[NT][4];
  make_coef(k1 - 1);
  load_u(k1 - 1, u);
  stripe_load<T, NT>(eigViT + (size_t)seg_process[seg0 + k1 - 1] * KK, 0, g, arow, aw[0]);
  for (int k = k1 - 1; k >= k0; --k) {
    const int s = seg_process[seg0 + k];
    const T* VT = eigVT + (size_t)s * KK;
    const T* ViT = eigViT + (size_t)s * KK;
    // W = R V^-T
    acc wk[1][NT];
#pragma unroll
    for (int mt = 0; mt < NT; ++mt) wk[0][mt] = acc{0, 0, 0, 0};
    stripe_gemm_from<T, NT, 1>(ViT, g, arow, aw, R, wk);
    if (k > k0) {  // while those MFMAs run
      stripe_load<T, NT>(VT, 0, g, arow, av[0]);
      stripe_load<T, NT>(eigViT + (size_t)seg_process[seg0 + k - 1] * KK, 0, g, arow, aw[0]);
      load_u(k - 1, un);
      make_coef(k - 1);
    }
    // stage this stripe's rows of W_k and U_k
#pragma unroll
    for (int mt = 0; mt < NT; ++mt)
#pragma unroll
      for (int q = 0; q < 4; ++q) {
        sW[row * LD + 16 * mt + 4 * g + q] = wk[0][mt][q];
        sU[row * LD + 16 * mt + 4 * g + q] = u[mt][q];
      }
    __syncthreads();
    // rows 16 w .. 16 w + 15 of Y_k = U_k^T W_k (contraction over every row i)
    acc yv[NT];
#pragma unroll
    for (int nt = 0; nt < NT; ++nt) yv[nt] = acc{0, 0, 0, 0};
#pragma unroll
    for (int kk = 0; kk < Kp / 4; ++kk) {
      const int i = 4 * kk + g;
      const T a = sU[i * LD + 16 * w + arow];
#pragma unroll
      for (int nt = 0; nt < NT; ++nt) yv[nt] = Mfma<T>::mma(a, sW[i * LD + 16 * nt + n], yv[nt]);
    }
    double* Y = Yseg + ((size_t)(seg0 + k) * C + c) * KK;
#pragma unroll
    for (int nt = 0; nt < NT; ++nt)
#pragma unroll
      for (int q = 0; q < 4; ++q) Y[(size_t)(16 * w + 4 * g + q) * Kp + 16 * nt + n] = (double)yv[nt][q];
    __syncthreads();  // also orders this wavefront's coefficient writes before the reads below
    if (k > k0) {
      // R <- R + (W (E_k - I)^T) V^T; the transposed rotation flips the partner sign
      const T(*ck)[2] = coef + 64 * (k & 1);
#pragma unroll
      for (int mt = 0; mt < NT; ++mt)
#pragma unroll
        for (int q = 0; q < 4; q += 2) {
          const int j = 16 * mt + 4 * g + q;
          const T y0 = wk[0][mt][q], y1 = wk[0][mt][q + 1];
          wk[0][mt][q] = ck[j][0] * y0 + ck[j][1] * y1;
          wk[0][mt][q + 1] = ck[j + 1][0] * y1 + ck[j + 1][1] * y0;
        }
      stripe_gemm_from<T, NT, 1>(VT, g, arow, av, wk, R);
#pragma unroll
      for (int mt = 0; mt < NT; ++mt)
#pragma unroll
        for (int q = 0; q < 4; ++q) u[mt][q] = un[mt][q];
    }
  }
}

// (e^{x_a} - e^{x_b}) / (x_a - x_b) from E_a = e^{x_a}, E_b = e^{x_b} and
// d = x_a - x_b: the quotient where |d| is large, E_b (e^d - 1)/d by its Taylor
// series where it is small (no cancellation; exact limit E_b at d = 0).
__device__ inline cplx divided_difference_from_exp(cplx Ea, cplx Eb, cplx d) {
  const double ad = fabs(d.re) + fabs(d.im);
  if (ad > 0.25) return cdiv(cplx{Ea.re - Eb.re, Ea.im - Eb.im}, d);
  // (e^d - 1)/d = sum_{k>=0} d^k / (k+1)! = 1 + d/2 (1 + d/3 (1 + ... (1 + d/15))),
  // terms through d^14/15!: the remainder is below 0.25^15 / 16! ~ 4e-23.  Each
  // step multiplies by the correctly rounded constant 1/k (no division).
  cplx s = {1.0, 0.0};
#pragma unroll
  for (int k = 15; k >= 2; --k) {
    constexpr double one = 1.0;
    const double inv_k = one / (double)k;  // folded to a constant once the loop is unrolled
    s = cmul(s, d);
    s.re = 1.0 + s.re * inv_k;
    s.im = s.im * inv_k;
  }
  return cmul(Eb, s);
}

// H_s partial sums: for every segment term of process s in this block's chunk,
// tau Phi(tau lambda) o (T^T Y T^-T) in FP64 complex, one entry per thread.
__global__ __launch_bounds__(256) void qgrad_h_kernel(int Kp, int n_chunks, int chunk,
                                                      const int32_t* __restrict__ list_off,
                                                      const int32_t* __restrict__ list, const double* __restrict__ Yseg,
                                                      const double* __restrict__ qtau, const double* __restrict__ qexp,
                                                      const double* __restrict__ lr_all,
                                                      const double* __restrict__ li_all, double* __restrict__ Hpart) {
  const int KK = Kp * Kp;
  const int e = blockIdx.x * 256 + threadIdx.x;
  const int ch = blockIdx.y, s = blockIdx.z;
  if (e >= KK) return;
  const int a = e / Kp, b = e - (e / Kp) * Kp;
  const double* lr = lr_all + (size_t)s * Kp;
  const double* li = li_all + (size_t)s * Kp;
  const PairIdx pa = pair_of(li, a), pb = pair_of(li, b);
  const int na = pa.pair ? 2 : 1, nb = pb.pair ? 2 : 1;
  cplx tt[2][2];
  for (int ci = 0; ci < na; ++ci)
    for (int di = 0; di < nb; ++di)
      tt[ci][di] = cmul(T_entry(pa.first + ci, a, pa.first, pa.pair), Tinv_entry(b, pb.first + di, pb.first, pb.pair));
  const cplx dl = {lr[a] - lr[b], li[a] - li[b]};
  const int q0 = list_off[s] + ch * chunk;
  const int q1 = min(list_off[s + 1], q0 + chunk);
  double re = 0.0, im = 0.0;
  const double2* E = reinterpret_cast<const double2*>(qexp);
#pragma unroll 4
  for (int qi = q0; qi < q1; ++qi) {
    const int item = list[qi];
    const double tau = qtau[item];
    const double* Y = Yseg + (size_t)item * KK;
    cplx z = {0.0, 0.0};
    for (int ci = 0; ci < na; ++ci)
      for (int di = 0; di < nb; ++di) {
        const double yv = Y[(pa.first + ci) * Kp + pb.first + di];
        z.re += tt[ci][di].re * yv;
        z.im += tt[ci][di].im * yv;
      }
    const double2 ea = E[(size_t)item * Kp + a], eb = E[(size_t)item * Kp + b];
    const cplx phi = divided_difference_from_exp(cplx{ea.x, ea.y}, cplx{eb.x, eb.y}, cplx{tau * dl.re, tau * dl.im});
    const cplx wv = cmul(phi, z);
    re += tau * wv.re;
    im += tau * wv.im;
  }
  reinterpret_cast<double2*>(Hpart)[((size_t)s * n_chunks + ch) * KK + e] = make_double2(re, im);
}

// H_s = fixed-order sum of the chunk partials, one entry per thread.
__global__ __launch_bounds__(256) void qgrad_hsum_kernel(int KK, int n_chunks, const double* __restrict__ Hpart,
                                                         double* __restrict__ Hsum) {
  const int e = blockIdx.x * 256 + threadIdx.x;
  const int s = blockIdx.y;
  if (e >= KK) return;
  const double2* src = reinterpret_cast<const double2*>(Hpart) + (size_t)s * n_chunks * KK + e;
  double2 a0 = make_double2(0.0, 0.0), a1 = a0;
  int ch = 0;
#pragma unroll 8
  for (; ch + 2 <= n_chunks; ch += 2) {
    const double2 h0 = src[(size_t)ch * KK], h1 = src[(size_t)(ch + 1) * KK];
    a0.x += h0.x;
    a0.y += h0.y;
    a1.x += h1.x;
    a1.y += h1.y;
  }
  if (ch < n_chunks) {
    const double2 h0 = src[(size_t)ch * KK];
    a0.x += h0.x;
    a0.y += h0.y;
  }
  reinterpret_cast<double2*>(Hsum)[(size_t)s * KK + e] = make_double2(a0.x + a1.x, a0.y + a1.y);
}

// dQ_s = V^-T Re(T^-T H_s T^T) V^T.  Block (s, band) forms rows kFinalRows band
// .. kFinalRows (band + 1) - 1: X = Re(T^-T H T^T) in LDS, then those rows of
// Y = V^-T X (the band's columns of V^-1 staged in LDS), then dQ rows =
// Y_rows V^T with V replacing X in LDS, its rows padded to Kp + 1 doubles so
// that lanes reading one column of different rows fall in different banks
// (Kp (Kp + 1) + 2 kFinalRows Kp doubles).  Bands of 4 rows give S Kp / 4
// blocks: every block forms the whole X, but the two products, serial per
// thread, are 4 times shorter than with bands of 16.
constexpr int kFinalRows = 4;
__global__ __launch_bounds__(256) void qgrad_final_kernel(int K, int Kp, const double* __restrict__ Hsum,
                                                          const double* __restrict__ V, const double* __restrict__ Vi,
                                                          const double* __restrict__ li_all, double* __restrict__ dQ) {
  extern __shared__ __align__(16) unsigned char smem_raw[];
  constexpr int BR = kFinalRows;
  const int s = blockIdx.x, r0 = BR * blockIdx.y;
  const int KK = Kp * Kp;
  double* sX = reinterpret_cast<double*>(smem_raw);
  double* sY = sX + Kp * (Kp + 1);  // BR x Kp
  double* sVi = sY + BR * Kp;       // Kp x BR: columns r0 .. r0 + BR - 1 of V^-1
  const double* li = li_all + (size_t)s * Kp;
  const double2* H = reinterpret_cast<const double2*>(Hsum) + (size_t)s * KK;
  const double* Vis = Vi + (size_t)s * KK;
  for (int e = threadIdx.x; e < BR * Kp; e += 256) sVi[e] = Vis[(e / BR) * Kp + r0 + e % BR];
  for (int e = threadIdx.x; e < KK; e += 256) {
    const int a = e / Kp, b = e % Kp;
    const PairIdx pa = pair_of(li, a), pb = pair_of(li, b);
    const int na = pa.pair ? 2 : 1, nb = pb.pair ? 2 : 1;
    double re = 0.0;
    for (int ci = 0; ci < na; ++ci) {
      const int cc = pa.first + ci;
      const cplx t1 = Tinv_entry(cc, a, pa.first, pa.pair);
      for (int di = 0; di < nb; ++di) {
        const int dd = pb.first + di;
        const cplx t2 = T_entry(b, dd, pb.first, pb.pair);
        const double2 h = H[cc * Kp + dd];
        re += cmul(cmul(t1, cplx{h.x, h.y}), t2).re;
      }
    }
    sX[e] = re;
  }
  __syncthreads();
  for (int e = threadIdx.x; e < BR * Kp; e += 256) {
    const int ii = e / Kp, j = e % Kp;
    double r = 0.0;
    for (int l = 0; l < Kp; ++l) r += sVi[l * BR + ii] * sX[l * Kp + j];
    sY[e] = r;
  }
  __syncthreads();
  double* sV = sX;  // row stride Kp + 1
  for (int e = threadIdx.x; e < KK; e += 256) sV[(e / Kp) * (Kp + 1) + e % Kp] = V[(size_t)s * KK + e];
  __syncthreads();
  for (int e = threadIdx.x; e < BR * Kp; e += 256) {
    const int i = r0 + e / Kp, j = e % Kp;
    if (i < K && j < K) {
      double r = 0.0;
      for (int l = 0; l < Kp; ++l) r += sY[(i - r0) * Kp + l] * sV[j * (Kp + 1) + l];
      dQ[((size_t)s * K + i) * K + j] = r;
    }
  }
}

template <typename T, int NT>
int qgrad_mfma_launch(EpochInstance* in) {
  const int Kp = in->Kp, C = in->C;
  const size_t KK = (size_t)Kp * Kp, S = in->S;
  const T* base = static_cast<const T*>(sizeof(T) == 8 ? in->eig64.ptr : in->eigT.ptr);
  const T* baseT = static_cast<const T*>(sizeof(T) == 8 ? in->eig64T.ptr : in->eigTT.ptr);
  const T* lr = base + 2 * S * KK;
  double* qexp = static_cast<double*>(in->qtau.ptr) + in->plan.seg_process.size() * C;
  // the work items of the P stage that formed A_k V: whole chains, or split ones
  const int4* items4 = static_cast<const int4*>(in->chain_items.ptr) + (in->pstage_split ? in->n_nodes : 0);
  const int n_work = in->pstage_split ? in->n_chain_split_items : in->n_nodes;
  hipLaunchKernelGGL((qgrad_chain_kernel<T, NT>), dim3(n_work * C), dim3(64 * NT), 0, in->stream, C,
                     in->plan.root, base, base + S * KK, baseT, baseT + S * KK, lr, lr + S * Kp, in->d_seg_offset,
                     in->d_seg_process, items4, static_cast<const T*>(in->chain_scratch.ptr), in->d_seg_time, in->d_rate,
                     static_cast<const double*>(in->cat.ptr),
                     static_cast<const double*>(in->G.ptr), static_cast<T*>(in->qscratch.ptr),
                     static_cast<double*>(in->qseg.ptr), static_cast<double*>(in->qtau.ptr),
                     static_cast<const double*>(in->eig64.ptr) + 2 * S * KK,
                     static_cast<const double*>(in->eig64.ptr) + 2 * S * KK + S * Kp, qexp);
  int rc = hip_check(hipGetLastError(), "qgrad_chain launch");
  if (rc) return rc;
  const double* b64 = static_cast<const double*>(in->eig64.ptr);
  const int32_t* lo = static_cast<const int32_t*>(in->seglist.ptr);
  const int32_t* items = lo + in->S + 1;
  const size_t nseg = in->plan.seg_process.size();
  double* Hpart = static_cast<double*>(in->qseg.ptr) + nseg * C * KK;
  double* Hsum = Hpart + 2 * S * in->q_chunks * KK;
  dim3 grid((unsigned)((KK + 255) / 256), (unsigned)in->q_chunks, (unsigned)S);
  hipLaunchKernelGGL(qgrad_h_kernel, grid, dim3(256), 0, in->stream, Kp, in->q_chunks, in->q_chunk_items, lo, items,
                     static_cast<const double*>(in->qseg.ptr), static_cast<const double*>(in->qtau.ptr), qexp,
                     b64 + 2 * S * KK, b64 + 2 * S * KK + S * Kp, Hpart);

  hipLaunchKernelGGL(qgrad_hsum_kernel, dim3((unsigned)((KK + 255) / 256), (unsigned)S), dim3(256), 0, in->stream,
                     (int)KK, in->q_chunks, static_cast<const double*>(Hpart), Hsum);
  rc = hip_check(hipGetLastError(), "qgrad_h launch");
  if (rc) return rc;
  hipLaunchKernelGGL(qgrad_final_kernel, dim3(in->S, Kp / kFinalRows), dim3(256),
                     (KK + (2 * kFinalRows + 1) * Kp) * sizeof(double),
                     in->stream, in->K, Kp, static_cast<const double*>(Hsum), b64, b64 + S * KK,
                     b64 + 2 * S * KK + S * Kp, static_cast<double*>(in->dQ.ptr));
  return hip_check(hipGetLastError(), "qgrad_final launch");
}

template <typename T>
int qgrad_mfma_dispatch(EpochInstance* in) {
  switch (in->Kp) {
    case 16: return qgrad_mfma_launch<T, 1>(in);
    case 32: return qgrad_mfma_launch<T, 2>(in);
    case 48: return qgrad_mfma_launch<T, 3>(in);
    case 64: return qgrad_mfma_launch<T, 4>(in);
    default: return set_error(EPOCH_ERR_STATE, "matrix-core dlogL/dQ needs Kp in {16, 32, 48, 64}, got %d", in->Kp);
  }
}

template <typename T>
int qgrad_dispatch(EpochInstance* in) {
  const int Kp = in->Kp, KK = Kp * Kp, C = in->C;
  const int ept = (KK + 255) / 256;
  const size_t S = in->S;
  const T* base = static_cast<const T*>(sizeof(T) == 8 ? in->eig64.ptr : in->eigT.ptr);
  const T* V = base;
  const T* Vi = base + S * KK;
  const T* lr = base + 2 * S * KK;
  const T* li = lr + S * Kp;
  const double* cat = static_cast<const double*>(in->cat.ptr);
  dim3 grid(in->n_nodes * C);
  const size_t shm = 2 * (size_t)KK * sizeof(T);
#define EPOCH_QSEG(E)                                                                            \
  hipLaunchKernelGGL((qgrad_segments_kernel<T, E>), grid, dim3(256), shm, in->stream, in->n_nodes, \
                     in->plan.root, Kp, C, V, Vi, lr, li, in->d_seg_offset, in->d_seg_process,     \
                     in->d_seg_time, in->d_rate, cat, static_cast<const double*>(in->G.ptr),       \
                     static_cast<T*>(in->qscratch.ptr), static_cast<double*>(in->qseg.ptr))
  if (ept <= 1) EPOCH_QSEG(1);
  else if (ept <= 4) EPOCH_QSEG(4);
  else if (ept <= 9) EPOCH_QSEG(9);
  else EPOCH_QSEG(16);
#undef EPOCH_QSEG
  int rc = hip_check(hipGetLastError(), "qgrad_segments launch");
  if (rc) return rc;
  const double* b64 = static_cast<const double*>(in->eig64.ptr);
  const int32_t* lo = static_cast<const int32_t*>(in->seglist.ptr);
  const int32_t* items = lo + in->S + 1;
  double* Hbuf = static_cast<double*>(in->qseg.ptr) +
                 2 * (size_t)in->plan.seg_process.size() * C * KK;  // tail of the qseg buffer
  const size_t shm2 = (size_t)KK * sizeof(double);
#define EPOCH_QRED(E)                                                                            \
  hipLaunchKernelGGL((qgrad_reduce_kernel<E>), dim3(in->S), dim3(256), shm2, in->stream, in->K, Kp, C, \
                     lo, items, static_cast<const double*>(in->qseg.ptr), b64, b64 + S * KK,      \
                     b64 + 2 * S * KK + S * Kp, Hbuf, static_cast<double*>(in->dQ.ptr))
  if (ept <= 1) EPOCH_QRED(1);
  else if (ept <= 4) EPOCH_QRED(4);
  else if (ept <= 9) EPOCH_QRED(9);
  else EPOCH_QRED(16);
#undef EPOCH_QRED
  return hip_check(hipGetLastError(), "qgrad_reduce launch");
}

}  // namespace

int launch_grad_Q_generic(EpochInstance* in) {
  return (in->fp64 || in->eig_fp64) ? qgrad_dispatch<double>(in) : qgrad_dispatch<float>(in);
}

bool grad_Q_mfma_supported(const EpochInstance* in) { return in->Kp >= 16 && in->Kp <= 64 && in->Kp % 16 == 0; }

int launch_grad_Q_mfma(EpochInstance* in) {
  return (in->fp64 || in->eig_fp64) ? qgrad_mfma_dispatch<double>(in) : qgrad_mfma_dispatch<float>(in);
}

}  // namespace epochlik
