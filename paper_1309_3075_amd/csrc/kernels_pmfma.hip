// P stage on the matrix cores: the ordered product of eigen-reconstructed
// exponentials of one branch (Eq. 3, 6, 7; Appendix A) and its derivative
// with respect to the branch length, for padded state counts that are
// multiples of 16 (codon 61 -> 64, the 40-state trait model -> 48).
//
// Each factor is F_k = I + V (E_k - I) V^-1, so with X the running product
// (parent side first) one step is
//   X <- X + ((X V)(E_k - I)) V^-1,
//   D <- D + ((D V)(E_k - I) + (X V) dE_k) V^-1,   dE_k = dtau_k/dl * dE/dtau.
// Rows of P are independent through the whole chain, so one wavefront carries
// a 16-row stripe of one (branch, category) product from the identity to the
// end, entirely in registers: the kernel has no barriers and no LDS traffic
// apart from a per-wave table of column coefficients.
//
// Layout.  The wave holds the stripe transposed, X^T (Kp x 16), as Kp/16
// accumulator tiles of v_mfma_*_16x16x4: lane (g = lane / 16, n = lane % 16)
// holds X^T[16 t + 4 g + v][n], v = 0..3, of tile t.  A product Y^T = V^T X^T
// runs its contraction index l over (tile t, register v, lane group g) as
// l = 16 t + 4 g + v, which is a permutation of 0..Kp-1; with that ordering
// the B operand of every MFMA is a register the lane already holds, and the
// A operand is an entry of row l of V (a coalesced row read).  The result comes out
// in the same layout, so the chain never leaves the registers.  Complex pairs
// sit at even/odd column pairs (the host orders eigen-columns so), so the
// 2x2 rotation of E couples registers v and v ^ 1 of one lane.
#include <hip/hip_runtime.h>

#include <algorithm>

#include "device_common.h"
#include "eigen_block.h"
#include "instance.h"
#include "mfma_chain.h"

namespace epochlik {

namespace {

// Matrix `which` (0: X_j, 1: dX_j, 2: prefix, 3: suffix, 4: suffix transposed)
// of part j of split `slot`, category c, in the chain scratch.
template <typename T, int KK>
__device__ inline T* chain_mat(void* scratch, int slot, int C, int c, int part, int which) {
  return static_cast<T*>(scratch) + ((((size_t)slot * C + c) * kChainMaxParts + part) * 5 + which) * KK;
}

// One wavefront = one 16-row stripe of one (work item, category) of one
// problem.  A work item is a node's whole chain, or the head or tail half of a
// long one (written to scratch for pstage_combine_kernel).
template <typename T, typename TO, bool GRAD, int NT>
__device__ inline void pstage_stripe(const PStageDesc& pd, int gw, ColCoef<T>* coef) {
  using acc = typename Mfma<T>::acc;
  constexpr int Kp = 16 * NT;
  constexpr int KK = Kp * Kp;
  const int item = gw / NT, stripe = gw - item * NT;
  if (item >= pd.n_items) return;  // whole wavefronts only: no barrier follows
  const int C = pd.C;
  const int4 wi = pd.items[item / C];
  const int k0 = wi.y, k1 = wi.z, kind = wi.w & 3, part = (wi.w >> 2) & 7, slot = wi.w >> 9;
  const T* __restrict__ eigV = static_cast<const T*>(pd.V);
  const T* __restrict__ eigVi = static_cast<const T*>(pd.Vi);
  const T* __restrict__ lre = static_cast<const T*>(pd.lr);
  const T* __restrict__ lim = static_cast<const T*>(pd.li);
  const int32_t* __restrict__ seg_offset = pd.seg_offset;
  const int32_t* __restrict__ seg_process = pd.seg_process;
  const double* __restrict__ seg_time = pd.seg_time;
  const double* __restrict__ seg_frac = pd.seg_frac;
  const double* __restrict__ rate = pd.rate;
  const double* __restrict__ cat_rates = pd.cat_rates;
  TO* __restrict__ Pout = static_cast<TO*>(pd.Pout);
  TO* __restrict__ dPout = static_cast<TO*>(pd.dPout);
  const int lane = threadIdx.x & 63;
  const int v = wi.x, c = item - (item / C) * C;
  const int g = lane >> 4, n = lane & 15;
  const int row = 16 * stripe + n;  // row of P this lane's column of X^T belongs to
  const int arow = Mfma<T>::a_row(n);

  constexpr int NB = GRAD ? 2 : 1;  // the running product X and, with GRAD, its derivative D
  acc xd[NB][NT];
#pragma unroll
  for (int t = 0; t < NT; ++t)
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      xd[0][t][q] = (16 * t + 4 * g + q == row) ? T(1) : T(0);
      if (GRAD) xd[NB - 1][t][q] = T(0);
    }

  const int seg0 = seg_offset[v];
  const double rho = cat_rates[c];
  const double scale = rho * rate[v];
  // Column coefficients of segment k (double-buffered by k parity).  Those of
  // segment k + 1, and the first operands of its V product, are produced while
  // the matrix cores run segment k's products.
  auto make_coef = [&](int k, ColCoef<T>* dst) {
    const int s = seg_process[seg0 + k];
    if (lane < Kp) {
      const T tau = T(scale * seg_time[seg0 + k]);
      const T dsc = T(rho * seg_frac[seg0 + k]);
      const BlockCoef<T> bc = block_coef(lre + (size_t)s * Kp, lim + (size_t)s * Kp, lane, tau);
      dst[lane] = ColCoef<T>{bc.m_self, bc.m_other, dsc * bc.dm_self, dsc * bc.dm_other};
    }
  };
  T av[2][4][NT], ai[2][4][NT];
  if (k1 > k0) {
    make_coef(k0, coef + 64 * (k0 & 1));
    stripe_load<T, NT>(eigV + (size_t)seg_process[seg0 + k0] * KK, 0, g, arow, av[0]);
  }
  for (int k = k0; k < k1; ++k) {
    const int s = seg_process[seg0 + k];
    const ColCoef<T>* ck = coef + 64 * (k & 1);
    wave_lds_sync();  // segment k's coefficients are in LDS
    stripe_load<T, NT>(eigVi + (size_t)s * KK, 0, g, arow, ai[0]);

    // Y^T = V^T X^T (and V^T D^T)
    acc y[NB][NT];
#pragma unroll
    for (int b = 0; b < NB; ++b)
#pragma unroll
      for (int mt = 0; mt < NT; ++mt) y[b][mt] = acc{0, 0, 0, 0};
    stripe_gemm_from<T, NT, NB>(eigV + (size_t)s * KK, g, arow, av, xd, y);
    if (k + 1 < k1) {
      make_coef(k + 1, coef + 64 * ((k + 1) & 1));
      stripe_load<T, NT>(eigV + (size_t)seg_process[seg0 + k + 1] * KK, 0, g, arow, av[0]);
    }
    if (pd.Ubuf) {
      // A_k V (the running product times V before the column operator), the forward
      // half of the dlogL/dQ adjoint chain
      T* U = static_cast<T*>(pd.Ubuf) + ((size_t)(seg0 + k) * C + c) * KK + (size_t)row * Kp + 4 * g;
#pragma unroll
      for (int mt = 0; mt < NT; ++mt) store4<T, T>(U + 16 * mt, y[0][mt]);
    }

    // column operator on rows j = 16 mt + 4 g + q of Y^T
#pragma unroll
    for (int mt = 0; mt < NT; ++mt)
#pragma unroll
      for (int q = 0; q < 4; q += 2) {
        const ColCoef<T> c0 = ck[16 * mt + 4 * g + q];
        const ColCoef<T> c1 = ck[16 * mt + 4 * g + q + 1];
        const T y0 = y[0][mt][q], y1 = y[0][mt][q + 1];
        y[0][mt][q] = c0.ms * y0 + c0.mo * y1;
        y[0][mt][q + 1] = c1.ms * y1 + c1.mo * y0;
        if (GRAD) {
          const T d0 = y[NB - 1][mt][q], d1 = y[NB - 1][mt][q + 1];
          y[NB - 1][mt][q] = c0.ms * d0 + c0.mo * d1 + c0.dms * y0 + c0.dmo * y1;
          y[NB - 1][mt][q + 1] = c1.ms * d1 + c1.mo * d0 + c1.dms * y1 + c1.dmo * y0;
        }
      }

    // X^T += V^-T Y'^T (and D^T += V^-T YD'^T)
    stripe_gemm_from<T, NT, NB>(eigVi + (size_t)s * KK, g, arow, ai, y, xd);
  }

  if (kind == 0) {
    const size_t base = ((size_t)v * C + c) * KK + (size_t)row * Kp + 4 * g;
#pragma unroll
    for (int mt = 0; mt < NT; ++mt) {
      store4<T, TO>(Pout + base + 16 * mt, xd[0][mt]);
      if (GRAD) store4<T, TO>(dPout + base + 16 * mt, xd[NB - 1][mt]);
    }
    return;
  }
  // one part of a split chain: its product X_j and dX_j/dl
  T* X = chain_mat<T, KK>(pd.scratch, slot, C, c, part, 0);
#pragma unroll
  for (int mt = 0; mt < NT; ++mt) {
    store4<T, T>(X + (size_t)row * Kp + 4 * g + 16 * mt, xd[0][mt]);
    if (GRAD) store4<T, T>(X + KK + (size_t)row * Kp + 4 * g + 16 * mt, xd[NB - 1][mt]);
  }
}

// A split chain's parts combined, in order: (X, D) <- (X X_j, D X_j + X dX_j)
// from (X_0, dX_0) gives P and dP/dl (the product rule over the parts).  The
// prefix X_0 .. X_{j-1} of each part j >= 1 is kept for the forward products of
// the dlogL/dQ adjoint, and with it the suffixes X_{j+1} .. X_{J-1} (and their
// transposes) that start the parts' backward chains.  One block of NT
// wavefronts (16-row stripes) per (split, category).
template <typename T, typename TO, bool GRAD, int NT>
__global__ __launch_bounds__(256) void pstage_combine_kernel(PStageDesc pd, const int4* __restrict__ splits) {
  using acc = typename Mfma<T>::acc;
  constexpr int Kp = 16 * NT;
  constexpr int KK = Kp * Kp;
  constexpr int NB = GRAD ? 2 : 1;
  const int C = pd.C;
  const int sidx = blockIdx.x / C, c = blockIdx.x - sidx * C;
  const int4 sp = splits[sidx];  // node, m, parts, slot
  const int v = sp.x, J = sp.z, slot = sp.w;
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  const int g = lane >> 4, n = lane & 15;
  const int row = 16 * w + n;
  const int arow = Mfma<T>::a_row(n);
  const size_t rbase = (size_t)row * Kp + 4 * g;
  auto load_rows = [&](const T* M, acc (&x)[NT]) {
#pragma unroll
    for (int mt = 0; mt < NT; ++mt)
#pragma unroll
      for (int q = 0; q < 4; ++q) x[mt][q] = M[rbase + 16 * mt + q];
  };
  acc x[NB][NT];
#pragma unroll
  for (int b = 0; b < NB; ++b) load_rows(chain_mat<T, KK>(pd.scratch, slot, C, c, 0, b), x[b]);
  for (int j = 1; j < J; ++j) {
    if (pd.Ubuf) {
      T* pre = chain_mat<T, KK>(pd.scratch, slot, C, c, j, 2);
#pragma unroll
      for (int mt = 0; mt < NT; ++mt) store4<T, T>(pre + rbase + 16 * mt, x[0][mt]);
    }
    acc o[NB][NT];
#pragma unroll
    for (int b = 0; b < NB; ++b)
#pragma unroll
      for (int mt = 0; mt < NT; ++mt) o[b][mt] = acc{0, 0, 0, 0};
    stripe_gemm<T, NT, NB>(chain_mat<T, KK>(pd.scratch, slot, C, c, j, 0), g, arow, x, o);  // X X_j (and D X_j)
    if (GRAD) {
      acc xa[1][NT], d[1][NT];
#pragma unroll
      for (int mt = 0; mt < NT; ++mt) {
        xa[0][mt] = x[0][mt];
        d[0][mt] = o[NB - 1][mt];
      }
      stripe_gemm<T, NT, 1>(chain_mat<T, KK>(pd.scratch, slot, C, c, j, 1), g, arow, xa, d);  // + X dX_j
#pragma unroll
      for (int mt = 0; mt < NT; ++mt) o[NB - 1][mt] = d[0][mt];
    }
#pragma unroll
    for (int b = 0; b < NB; ++b)
#pragma unroll
      for (int mt = 0; mt < NT; ++mt) x[b][mt] = o[b][mt];
  }
  TO* Pout = static_cast<TO*>(pd.Pout);
  TO* dPout = static_cast<TO*>(pd.dPout);
  const size_t base = ((size_t)v * C + c) * KK + rbase;
#pragma unroll
  for (int mt = 0; mt < NT; ++mt) {
    store4<T, TO>(Pout + base + 16 * mt, x[0][mt]);
    if (GRAD) store4<T, TO>(dPout + base + 16 * mt, x[NB - 1][mt]);
  }
  if (!pd.Ubuf) return;  // uniform
  // suffixes, last part first: S_{J-2} = X_{J-1}, S_j = X_{j+1} S_{j+1}
  for (int j = J - 2; j >= 0; --j) {
    acc sfx[1][NT];
    if (j == J - 2) {
      load_rows(chain_mat<T, KK>(pd.scratch, slot, C, c, J - 1, 0), sfx[0]);
    } else {
      acc xr[1][NT];
      load_rows(chain_mat<T, KK>(pd.scratch, slot, C, c, j + 1, 0), xr[0]);
#pragma unroll
      for (int mt = 0; mt < NT; ++mt) sfx[0][mt] = acc{0, 0, 0, 0};
      stripe_gemm<T, NT, 1>(chain_mat<T, KK>(pd.scratch, slot, C, c, j + 1, 3), g, arow, xr, sfx);
    }
    T* S = chain_mat<T, KK>(pd.scratch, slot, C, c, j, 3);
    T* ST = chain_mat<T, KK>(pd.scratch, slot, C, c, j, 4);
#pragma unroll
    for (int mt = 0; mt < NT; ++mt) {
      store4<T, T>(S + rbase + 16 * mt, sfx[0][mt]);
#pragma unroll
      for (int q = 0; q < 4; ++q) ST[(size_t)(16 * mt + 4 * g + q) * Kp + row] = sfx[0][mt][q];
    }
    __syncthreads();  // S_j whole before the next suffix reads it
  }
}

// With dlogL/dQ, the stored products A_k V of parts j >= 1 (formed from the
// part's own start) become (X_0 .. X_{j-1}) (A_k V).  One block of NT
// wavefronts per (split, category, segment past part 0); the block reads its
// A_k V whole before any stripe overwrites its rows.
template <typename T, int NT>
__global__ __launch_bounds__(256) void pstage_tail_fix_kernel(PStageDesc pd, const int4* __restrict__ splits) {
  using acc = typename Mfma<T>::acc;
  constexpr int Kp = 16 * NT;
  constexpr int KK = Kp * Kp;
  const int C = pd.C;
  const int sidx = blockIdx.x / C, c = blockIdx.x - sidx * C;
  const int4 sp = splits[sidx];  // node, m, parts, slot
  const int m = sp.y, J = sp.z;
  const int k = m / J + blockIdx.y;
  if (k >= m) return;  // uniform: this chain is shorter
  int part = 1;
  while (part + 1 < J && (part + 1) * m / J <= k) ++part;
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  const int g = lane >> 4, n = lane & 15;
  const int row = 16 * w + n;
  const int arow = Mfma<T>::a_row(n);
  const T* XA = chain_mat<T, KK>(pd.scratch, sp.w, C, c, part, 2);  // the prefix of this part
  acc xa[1][NT], u[1][NT];
#pragma unroll
  for (int mt = 0; mt < NT; ++mt) {
#pragma unroll
    for (int q = 0; q < 4; ++q) xa[0][mt][q] = XA[(size_t)row * Kp + 16 * mt + 4 * g + q];
    u[0][mt] = acc{0, 0, 0, 0};
  }
  T* U = static_cast<T*>(pd.Ubuf) + ((size_t)(pd.seg_offset[sp.x] + k) * C + c) * KK;
  stripe_gemm<T, NT, 1>(U, g, arow, xa, u);
  __syncthreads();  // every stripe has read this A_k V
#pragma unroll
  for (int mt = 0; mt < NT; ++mt) store4<T, T>(U + (size_t)row * Kp + 4 * g + 16 * mt, u[0][mt]);
}

// One problem (descriptor passed by value).
template <typename T, typename TO, bool GRAD, int NT>
__global__ __launch_bounds__(256) void pstage_mfma_kernel(PStageDesc pd) {
  __shared__ ColCoef<T> s_coef[4][2 * 64];
  const int wave = threadIdx.x >> 6;
  pstage_stripe<T, TO, GRAD, NT>(pd, blockIdx.x * 4 + wave, s_coef[wave]);
}

// Several problems of one batch in one launch: blockIdx.y selects the problem.
template <typename T, typename TO, bool GRAD, int NT>
__global__ __launch_bounds__(256) void pstage_mfma_multi_kernel(const PStageDesc* __restrict__ descs) {
  __shared__ ColCoef<T> s_coef[4][2 * 64];
  const int wave = threadIdx.x >> 6;
  const PStageDesc pd = descs[blockIdx.y];
  pstage_stripe<T, TO, GRAD, NT>(pd, blockIdx.x * 4 + wave, s_coef[wave]);
}

template <typename T, typename TO, int NT>
int pstage_mfma_launch(EpochInstance* in, const int4* d_items, int n_items) {
  const bool split = !d_items && in->n_chain_splits > 0;
  PStageDesc pd = pstage_descriptor(in);
  if (d_items) {  // whole chains of the listed nodes only
    pd.items = d_items;
    pd.n_items = n_items * in->C;
  } else if (split) {
    pd.items = static_cast<const int4*>(in->chain_items.ptr) + in->n_nodes;
    pd.n_items = in->n_chain_split_items * in->C;
  }
  const long waves = (long)pd.n_items * NT;
  dim3 grid((unsigned)((waves + 3) / 4));
  if (pd.grad)
    hipLaunchKernelGGL((pstage_mfma_kernel<T, TO, true, NT>), grid, dim3(256), 0, in->stream, pd);
  else
    hipLaunchKernelGGL((pstage_mfma_kernel<T, TO, false, NT>), grid, dim3(256), 0, in->stream, pd);
  if (split) {
    const int4* splits = static_cast<const int4*>(in->chain_items.ptr) + in->n_nodes + in->n_chain_split_items;
    dim3 cgrid((unsigned)(in->n_chain_splits * in->C));
    if (pd.grad)
      hipLaunchKernelGGL((pstage_combine_kernel<T, TO, true, NT>), cgrid, dim3(64 * NT), 0, in->stream, pd, splits);
    else
      hipLaunchKernelGGL((pstage_combine_kernel<T, TO, false, NT>), cgrid, dim3(64 * NT), 0, in->stream, pd, splits);
    if (pd.Ubuf)
      hipLaunchKernelGGL((pstage_tail_fix_kernel<T, NT>), dim3(cgrid.x, (unsigned)in->chain_max_tail), dim3(64 * NT),
                         0, in->stream, pd, splits);
  }
  if (!d_items) in->pstage_split = split;  // a restricted launch leaves the other chains as they were
  return hip_check(hipGetLastError(), "pstage_mfma launch");
}

template <typename T, typename TO>
int pstage_mfma_dispatch(EpochInstance* in, const int4* d_items, int n_items) {
  switch (in->Kp) {
    case 16: return pstage_mfma_launch<T, TO, 1>(in, d_items, n_items);
    case 32: return pstage_mfma_launch<T, TO, 2>(in, d_items, n_items);
    case 48: return pstage_mfma_launch<T, TO, 3>(in, d_items, n_items);
    case 64: return pstage_mfma_launch<T, TO, 4>(in, d_items, n_items);
    default: return set_error(EPOCH_ERR_STATE, "matrix-core P stage needs Kp in {16, 32, 48, 64}, got %d", in->Kp);
  }
}

template <typename T, typename TO, int NT>
int pstage_multi_launch(const PStageDesc* d_descs, int n, int max_items, bool grad, hipStream_t st) {
  dim3 grid((unsigned)(((long)max_items * NT + 3) / 4), (unsigned)n);
  if (grad)
    hipLaunchKernelGGL((pstage_mfma_multi_kernel<T, TO, true, NT>), grid, dim3(256), 0, st, d_descs);
  else
    hipLaunchKernelGGL((pstage_mfma_multi_kernel<T, TO, false, NT>), grid, dim3(256), 0, st, d_descs);
  return hip_check(hipGetLastError(), "pstage_mfma_multi launch");
}

template <typename T, typename TO>
int pstage_multi_dispatch(int Kp, const PStageDesc* d_descs, int n, int max_items, bool grad, hipStream_t st) {
  switch (Kp) {
    case 16: return pstage_multi_launch<T, TO, 1>(d_descs, n, max_items, grad, st);
    case 32: return pstage_multi_launch<T, TO, 2>(d_descs, n, max_items, grad, st);
    case 48: return pstage_multi_launch<T, TO, 3>(d_descs, n, max_items, grad, st);
    case 64: return pstage_multi_launch<T, TO, 4>(d_descs, n, max_items, grad, st);
    default: return set_error(EPOCH_ERR_STATE, "matrix-core P stage needs Kp in {16, 32, 48, 64}, got %d", Kp);
  }
}

}  // namespace

bool pstage_mfma_supported(const EpochInstance* in) {
  return in->Kp >= 16 && in->Kp <= 64 && in->Kp % 16 == 0;
}

int launch_pstage_mfma(EpochInstance* in) { return launch_pstage_mfma_items(in, nullptr, 0); }

int launch_pstage_mfma_items(EpochInstance* in, const int4* d_items, int n_items) {
  if (in->fp64) return pstage_mfma_dispatch<double, double>(in, d_items, n_items);
  return in->eig_fp64 ? pstage_mfma_dispatch<double, float>(in, d_items, n_items)
                      : pstage_mfma_dispatch<float, float>(in, d_items, n_items);
}

// The device pointers and sizes one problem's P stage reads and writes, in the
// arithmetic type the instance uses (FP64 eigensystems when fp64 or eig_fp64).
PStageDesc pstage_descriptor(const EpochInstance* in) {
  PStageDesc d{};
  const size_t KK = (size_t)in->Kp * in->Kp, S = in->S;
  const bool dbl = in->fp64 || in->eig_fp64;
  const size_t es = dbl ? sizeof(double) : sizeof(float);
  const char* base = static_cast<const char*>(dbl ? in->eig64.ptr : in->eigT.ptr);
  d.V = base;
  d.Vi = base + S * KK * es;
  d.lr = base + 2 * S * KK * es;
  d.li = base + (2 * S * KK + S * in->Kp) * es;
  d.seg_offset = in->d_seg_offset;
  d.seg_process = in->d_seg_process;
  d.items = static_cast<const int4*>(in->chain_items.ptr);  // whole chains; the single-instance launch may split
  d.scratch = in->chain_scratch.ptr;
  d.seg_time = in->d_seg_time;
  d.seg_frac = in->d_seg_frac;
  d.rate = in->d_rate;
  d.cat_rates = static_cast<const double*>(in->cat.ptr);
  d.Pout = in->Pm.ptr;
  d.dPout = in->dPm.ptr;
  // the matrix-core dlogL/dQ chain reads A_k V from the P stage
  d.Ubuf = ((in->cfg.flags & EPOCH_GRAD_Q) && in->qscratch.ptr && grad_Q_mfma_supported(in) &&
            in->cfg.kernel_path == EPOCH_KERNEL_AUTO)
               ? in->qscratch.ptr
               : nullptr;
  d.n_items = in->n_nodes * in->C;
  d.C = in->C;
  d.grad = (in->cfg.flags & (EPOCH_GRAD_BRANCH | EPOCH_GRAD_Q)) != 0;
  return d;
}

// One launch for a group of problems that share Kp, precision, eigen arithmetic
// and gradient flag (their descriptors already on the device).
int launch_pstage_mfma_multi(const EpochInstance* like, const PStageDesc* d_descs, int n, int max_items,
                             hipStream_t st) {
  const bool grad = (like->cfg.flags & (EPOCH_GRAD_BRANCH | EPOCH_GRAD_Q)) != 0;
  if (like->fp64) return pstage_multi_dispatch<double, double>(like->Kp, d_descs, n, max_items, grad, st);
  if (like->eig_fp64) return pstage_multi_dispatch<double, float>(like->Kp, d_descs, n, max_items, grad, st);
  return pstage_multi_dispatch<float, float>(like->Kp, d_descs, n, max_items, grad, st);
}

}  // namespace epochlik
