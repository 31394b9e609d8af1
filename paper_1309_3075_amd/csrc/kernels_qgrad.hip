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
#include "instance.h"

namespace epochlik {

namespace {

struct cplx {
  double re, im;
};
__device__ inline cplx cmul(cplx a, cplx b) { return {a.re * b.re - a.im * b.im, a.re * b.im + a.im * b.re}; }
__device__ inline cplx cdiv(cplx a, cplx b) {
  const double d = b.re * b.re + b.im * b.im;
  return {(a.re * b.re + a.im * b.im) / d, (a.im * b.re - a.re * b.im) / d};
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

}  // namespace epochlik
