// Node-height and epoch-boundary gradients (an addition: the paper fixes the
// transition times and names estimating them as the next step, Discussion).
//
// Heights and boundaries enter the likelihood only through the stretch
// durations of Eq. 7 (branch rates held fixed).  With G_{v,c} = dlogL/dP_{v,c}
// from the gradient pass and x = rho_c r_v:
//   - raising the parent height lengthens branch v at its top, by a stretch of
//     the interval holding the parent:      dP/dh_parent =  x Q_top P;
//   - raising the child height shortens it at its bottom, in the interval
//     holding the child:                    dP/dh_v      = -x P Q_bottom;
//   - raising boundary b_m (interval m below, m + 1 above) moves time of every
//     branch spanning it (h_v <= b_m < h_parent) from interval m + 1 to m:
//     dP/db_m = x X (Q_phi(m) - Q_phi(m+1)) Y, X and Y the products of the
//     factors above and below b_m.
// Intervals are half-open, [b_{m-1}, b_m), so at a tie (a node exactly on a
// boundary) these are the one-sided derivatives for an increasing height or
// boundary.
//
// Everything here runs in FP64 on the FP64 eigensystems: the end terms need
// two K x K products per (branch, category); a boundary term carries
// G X^T ... Y^T through the branch's factors, each applied as
// F^T W = W + V^-T (E - I)^T V^T W (the form the P stage uses, Eq. 3 with
// Appendix A), with the two working matrices in LDS.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstring>
#include <vector>

#include "device_common.h"
#include "eigen_block.h"
#include "instance.h"

namespace epochlik {

namespace {

// Fixed-order block sum of one value per thread.
__device__ inline double block_sum256(double v, double* sm) {
  sm[threadIdx.x] = v;
  __syncthreads();
  for (int w = 128; w > 0; w >>= 1) {
    if (threadIdx.x < w) sm[threadIdx.x] += sm[threadIdx.x + w];
    __syncthreads();
  }
  const double r = sm[0];
  __syncthreads();
  return r;
}

// One block per (branch v, category c): the parent-end and child-end terms
//   top = x <G, Q_top P>,  bottom = x <G, P Q_bottom>.
template <typename T>
__global__ __launch_bounds__(256) void tgrad_end_kernel(const T* __restrict__ Pm, const double* __restrict__ G,
                                                        const double* __restrict__ Qrec,
                                                        const int32_t* __restrict__ proc_top,
                                                        const int32_t* __restrict__ proc_bot,
                                                        const double* __restrict__ rate,
                                                        const double* __restrict__ cat, int root, int K, int Kp,
                                                        int C, double* __restrict__ out) {
  __shared__ double sm[256];
  const int v = blockIdx.x / C, c = blockIdx.x % C;
  if (v == root) {  // no branch: uniform over the block, no barrier is skipped by part of it
    if (threadIdx.x == 0) out[2 * blockIdx.x] = out[2 * blockIdx.x + 1] = 0.0;
    return;
  }
  const size_t KK = (size_t)Kp * Kp;
  const T* P = Pm + ((size_t)v * C + c) * KK;
  const double* g = G + ((size_t)v * C + c) * KK;
  const double* Qt = Qrec + (size_t)proc_top[v] * KK;
  const double* Qb = Qrec + (size_t)proc_bot[v] * KK;
  double top = 0.0, bot = 0.0;
  for (int e = threadIdx.x; e < K * K; e += 256) {
    const int i = e / K, j = e % K;
    double qp = 0.0, pq = 0.0;
    for (int l = 0; l < K; ++l) {
      qp += Qt[(size_t)i * Kp + l] * (double)P[(size_t)l * Kp + j];
      pq += (double)P[(size_t)i * Kp + l] * Qb[(size_t)l * Kp + j];
    }
    const double gij = g[(size_t)i * Kp + j];
    top += gij * qp;
    bot += gij * pq;
  }
  const double x = rate[v] * cat[c];
  top = block_sum256(top, sm);
  bot = block_sum256(bot, sm);
  if (threadIdx.x == 0) {
    out[2 * blockIdx.x] = x * top;
    out[2 * blockIdx.x + 1] = x * bot;
  }
}

// One block per (crossing, category).  A crossing (v, m, j): branch v spans
// boundary m, and its first j segments (parent side) lie above it.  Forms
// Z = X^T G Y^T and returns x <Z, Q_phi(m) - Q_phi(m+1)>.
template <int KP>
__global__ __launch_bounds__(256) void tgrad_cross_kernel(
    const int4* __restrict__ cross, const double* __restrict__ G, const double* __restrict__ eigV,
    const double* __restrict__ eigVi, const double* __restrict__ lre, const double* __restrict__ lim,
    const double* __restrict__ Qrec, const int32_t* __restrict__ seg_offset, const int32_t* __restrict__ seg_process,
    const double* __restrict__ seg_time, const double* __restrict__ rate, const double* __restrict__ cat,
    const int32_t* __restrict__ phi, int K, int C, double* __restrict__ out) {
  constexpr int KK = KP * KP;
  __shared__ double sW[KK], sT[KK];
  __shared__ double sSelf[KP], sOther[KP];
  __shared__ int sPartner[KP];
  __shared__ double sm[256];
  const int4 cr = cross[blockIdx.x / C];
  const int c = blockIdx.x % C;
  const int v = cr.x, m = cr.y, j = cr.z;
  const double x = rate[v] * cat[c];
  const int seg0 = seg_offset[v], L = seg_offset[v + 1] - seg0;
  for (int e = threadIdx.x; e < KK; e += 256) sW[e] = G[((size_t)v * C + c) * KK + e];
  __syncthreads();
  // step k applies factor k: before the boundary W <- F_k^T W (k = 0 .. j-1, parent side first),
  // after it W <- W F_k^T (k = L-1 down to j)
  for (int step = 0; step < L; ++step) {
    const bool left = step < j;
    const int k = left ? step : L - 1 - (step - j);
    const int s = seg_process[seg0 + k];
    const double tau = x * seg_time[seg0 + k];
    const double* V = eigV + (size_t)s * KK;
    const double* Vi = eigVi + (size_t)s * KK;
    if (threadIdx.x < KP) {
      if (threadIdx.x < K) {
        const BlockCoef<double> bc = block_coef(lre + (size_t)s * KP, lim + (size_t)s * KP, threadIdx.x, tau);
        sSelf[threadIdx.x] = bc.m_self;
        sOther[threadIdx.x] = bc.m_other;
        sPartner[threadIdx.x] = bc.partner;
      } else {
        sSelf[threadIdx.x] = 0.0;
        sOther[threadIdx.x] = 0.0;
        sPartner[threadIdx.x] = -1;
      }
    }
    // T1 = V^T W (left) or W V^-T (right)
    for (int e = threadIdx.x; e < KK; e += 256) {
      const int r = e / KP, q = e % KP;
      double t = 0.0;
      if (left) {
        for (int l = 0; l < K; ++l) t += V[l * KP + r] * sW[l * KP + q];
      } else {
        for (int l = 0; l < K; ++l) t += sW[r * KP + l] * Vi[q * KP + l];
      }
      sT[e] = t;
    }
    __syncthreads();
    // T2 = (E - I)^T T1 (left: mixes the rows of a pair) or T1 (E - I)^T (right: its columns);
    // each thread updates both members of a pair at one position
    for (int e = threadIdx.x; e < KK; e += 256) {
      const int a = e / KP, q = e % KP;  // left: row a, column q; right: row q, column a
      const int pa = sPartner[a];
      if (pa >= 0 && pa < a) continue;  // the pair's first member does both
      const int ia = left ? a * KP + q : q * KP + a;
      if (pa < 0) {
        sT[ia] *= sSelf[a];
        continue;
      }
      const int ib = left ? pa * KP + q : q * KP + pa;
      const double ta = sT[ia], tb = sT[ib];
      if (left) {  // T2[a] = M_aa T1[a] + M_{pa,a} T1[pa];  T2[pa] = M_{pa,pa} T1[pa] + M_{a,pa} T1[a]
        sT[ia] = sSelf[a] * ta + sOther[a] * tb;
        sT[ib] = sSelf[pa] * tb + sOther[pa] * ta;
      } else {     // T2[.][a] = M_aa T1[.][a] + M_{a,pa} T1[.][pa];  T2[.][pa] = M_{pa,pa} T1[.][pa] + M_{pa,a} T1[.][a]
        sT[ia] = sSelf[a] * ta + sOther[pa] * tb;
        sT[ib] = sSelf[pa] * tb + sOther[a] * ta;
      }
    }
    __syncthreads();
    // W += V^-T T2 (left) or W += T2 V^T (right)
    for (int e = threadIdx.x; e < KK; e += 256) {
      const int r = e / KP, q = e % KP;
      if (r >= K || q >= K) continue;
      double t = 0.0;
      if (left) {
        for (int a = 0; a < K; ++a) t += Vi[a * KP + r] * sT[a * KP + q];
      } else {
        for (int a = 0; a < K; ++a) t += sT[r * KP + a] * V[q * KP + a];
      }
      sW[e] += t;
    }
    __syncthreads();
  }
  const double* Qa = Qrec + (size_t)phi[m] * KK;      // interval m, below the boundary
  const double* Qb = Qrec + (size_t)phi[m + 1] * KK;  // interval m + 1, above it
  double acc = 0.0;
  for (int e = threadIdx.x; e < K * K; e += 256) {
    const int r = e / K, q = e % K;
    acc += sW[r * KP + q] * (Qa[r * KP + q] - Qb[r * KP + q]);
  }
  acc = block_sum256(acc, sm);
  if (threadIdx.x == 0) out[blockIdx.x] = x * acc;
}

// dlogL/dh_u = sum over u's children of their top terms - u's own bottom term;
// dlogL/db_m = the sum of boundary m's crossing terms (fixed orders).
__global__ __launch_bounds__(256) void tgrad_finish_kernel(const double* __restrict__ ends,
                                                           const double* __restrict__ cross_terms,
                                                           const int32_t* __restrict__ cross_off,
                                                           const int32_t* __restrict__ parent,
                                                           const int32_t* __restrict__ left,
                                                           const int32_t* __restrict__ right, int n_nodes,
                                                           int n_bound, int C, double* __restrict__ d_height,
                                                           double* __restrict__ d_bound) {
  const int t = blockIdx.x * 256 + threadIdx.x;
  if (t < n_nodes) {
    const int u = t;
    double d = 0.0;
    if (left[u] >= 0)
      for (int side = 0; side < 2; ++side) {
        const int ch = side == 0 ? left[u] : right[u];
        for (int c = 0; c < C; ++c) d += ends[2 * ((size_t)ch * C + c)];
      }
    if (parent[u] >= 0)
      for (int c = 0; c < C; ++c) d -= ends[2 * ((size_t)u * C + c) + 1];
    d_height[u] = d;
  } else if (t < n_nodes + n_bound) {
    const int m = t - n_nodes;
    double d = 0.0;
    for (int k = cross_off[m]; k < cross_off[m + 1]; ++k)
      for (int c = 0; c < C; ++c) d += cross_terms[(size_t)k * C + c];
    d_bound[m] = d;
  }
}

int interval_of(const std::vector<double>& b, double h) {
  return (int)(std::upper_bound(b.begin(), b.end(), h) - b.begin());
}

}  // namespace

// Host lists of the time gradient for the current tree (after set_tree_epochs).
int tgrad_prepare(EpochInstance* in) {
  const auto& pl = in->plan;
  const int n = in->n_nodes, nb = (int)pl.boundaries.size();
  std::vector<int32_t> top(n, 0), bot(n, 0), off(nb + 1, 0);
  std::vector<int4> cross;
  for (int v = 0; v < n; ++v) {
    const int u = pl.parent[v];
    bot[v] = pl.interval_process[interval_of(pl.boundaries, pl.height[v])];
    top[v] = u >= 0 ? pl.interval_process[interval_of(pl.boundaries, pl.height[u])] : 0;
  }
  for (int m = 0; m < nb; ++m) {
    off[m] = (int32_t)cross.size();
    const double bm = pl.boundaries[m];
    for (int v = 0; v < n; ++v) {
      const int u = pl.parent[v];
      if (u < 0 || !(pl.height[v] <= bm && bm < pl.height[u])) continue;
      int j = 0;  // segments above the boundary: intervals m + 1 and older
      for (int g = pl.seg_offset[v]; g < pl.seg_offset[v + 1]; ++g)
        if (pl.seg_interval[g] > m) ++j;
      cross.push_back(make_int4(v, m, j, 0));
    }
  }
  off[nb] = (int32_t)cross.size();
  in->tg_n_cross = (int)cross.size();
  in->tg_n_bound = nb;
  // int32: top [n], bottom [n], crossing offsets [nb + 1], phi [M]; then int4 crossings (16-byte aligned)
  std::vector<int32_t> hi(top);
  hi.insert(hi.end(), bot.begin(), bot.end());
  hi.insert(hi.end(), off.begin(), off.end());
  hi.insert(hi.end(), pl.interval_process.begin(), pl.interval_process.end());
  while (hi.size() % 4) hi.push_back(0);
  in->tg_cross_offset = hi.size() * sizeof(int32_t);
  const size_t bytes = in->tg_cross_offset + cross.size() * sizeof(int4);
  int rc = ensure(in->tg_i, std::max<size_t>(bytes, 256));
  const size_t KK = (size_t)in->Kp * in->Kp;
  // FP64: Q_s [S][Kp][Kp] (zero padding), end terms [n][C][2], crossing terms [X][C], outputs [n + nb],
  // tile scratch of the Q reconstruction
  const size_t doubles = in->S * KK + (size_t)n * in->C * 2 + cross.size() * in->C + n + nb +
                         3 * (size_t)eigen_check_tiles(in->K) * in->S;
  if (!rc) rc = ensure(in->tg_d, doubles * sizeof(double));
  if (!rc) rc = hip_check(hipMemsetAsync(in->tg_d.ptr, 0, in->S * KK * sizeof(double), in->stream), "Q clear");
  std::vector<char> h(bytes);
  memcpy(h.data(), hi.data(), hi.size() * sizeof(int32_t));
  if (!cross.empty()) memcpy(h.data() + in->tg_cross_offset, cross.data(), cross.size() * sizeof(int4));
  if (!rc) rc = hip_check(hipMemcpyAsync(in->tg_i.ptr, h.data(), bytes, hipMemcpyHostToDevice, in->stream),
                          "time-gradient list upload");
  if (!rc) rc = hip_check(hipStreamSynchronize(in->stream), "time-gradient list sync");
  return rc;
}

int launch_time_gradient(EpochInstance* in, double** d_height, double** d_bound) {
  const int n = in->n_nodes, C = in->C, nb = in->tg_n_bound, X = in->tg_n_cross;
  const size_t KK = (size_t)in->Kp * in->Kp;
  double* Qrec = static_cast<double*>(in->tg_d.ptr);
  double* ends = Qrec + in->S * KK;
  double* cterms = ends + (size_t)n * C * 2;
  double* dh = cterms + (size_t)X * C;
  double* db = dh + n;
  double* part = db + nb;
  const int32_t* ti = static_cast<const int32_t*>(in->tg_i.ptr);
  const int32_t *top = ti, *bot = ti + n, *off = ti + 2 * n, *phi = ti + 2 * n + nb + 1;
  const int4* cross = reinterpret_cast<const int4*>(static_cast<const char*>(in->tg_i.ptr) + in->tg_cross_offset);
  const double* cat = static_cast<const double*>(in->cat.ptr);
  int rc = launch_q_reconstruct(in, Qrec, part);
  if (rc) return rc;
  if (in->fp64)
    hipLaunchKernelGGL((tgrad_end_kernel<double>), dim3(n * C), dim3(256), 0, in->stream,
                       static_cast<const double*>(in->Pm.ptr), static_cast<const double*>(in->G.ptr), Qrec, top, bot,
                       in->d_rate, cat, in->plan.root, in->K, in->Kp, C, ends);
  else
    hipLaunchKernelGGL((tgrad_end_kernel<float>), dim3(n * C), dim3(256), 0, in->stream,
                       static_cast<const float*>(in->Pm.ptr), static_cast<const double*>(in->G.ptr), Qrec, top, bot,
                       in->d_rate, cat, in->plan.root, in->K, in->Kp, C, ends);
  rc = hip_check(hipGetLastError(), "tgrad_end launch");
  if (rc) return rc;
  if (X > 0) {
    const double* base = static_cast<const double*>(in->eig64.ptr);
    const double* V = base;
    const double* Vi = base + in->S * KK;
    const double* lr = base + 2 * in->S * KK;
    const double* li = lr + (size_t)in->S * in->Kp;
#define EPOCH_TGRAD_CROSS(KPV)                                                                             \
  hipLaunchKernelGGL((tgrad_cross_kernel<KPV>), dim3(X * C), dim3(256), 0, in->stream, cross, static_cast<const double*>(in->G.ptr), \
                     V, Vi, lr, li, Qrec, in->d_seg_offset, in->d_seg_process, in->d_seg_time, in->d_rate, cat, phi, \
                     in->K, C, cterms)
    switch (in->Kp) {
      case 4: EPOCH_TGRAD_CROSS(4); break;
      case 8: EPOCH_TGRAD_CROSS(8); break;
      case 16: EPOCH_TGRAD_CROSS(16); break;
      case 32: EPOCH_TGRAD_CROSS(32); break;
      case 48: EPOCH_TGRAD_CROSS(48); break;
      case 64: EPOCH_TGRAD_CROSS(64); break;
      default: return set_error(EPOCH_ERR_STATE, "time gradient: unsupported padded state count %d", in->Kp);
    }
#undef EPOCH_TGRAD_CROSS
    rc = hip_check(hipGetLastError(), "tgrad_cross launch");
    if (rc) return rc;
  }
  hipLaunchKernelGGL(tgrad_finish_kernel, dim3((n + nb + 255) / 256), dim3(256), 0, in->stream, ends, cterms, off,
                     in->d_parent, in->d_left, in->d_right, n, nb, C, dh, db);
  *d_height = dh;
  *d_bound = db;
  return hip_check(hipGetLastError(), "tgrad_finish launch");
}

}  // namespace epochlik
