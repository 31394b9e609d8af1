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

// One wavefront = one 16-row stripe of one (node, category) item.
template <typename T, typename TO, bool GRAD, int NT>
__global__ __launch_bounds__(256) void pstage_mfma_kernel(
    int n_items, int C, const T* __restrict__ eigV, const T* __restrict__ eigVi,
    const T* __restrict__ lre, const T* __restrict__ lim, const int32_t* __restrict__ seg_offset,
    const int32_t* __restrict__ seg_process, const double* __restrict__ seg_time,
    const double* __restrict__ seg_frac, const double* __restrict__ rate,
    const double* __restrict__ cat_rates, TO* __restrict__ Pout, TO* __restrict__ dPout) {
  using acc = typename Mfma<T>::acc;
  constexpr int Kp = 16 * NT;
  constexpr int KK = Kp * Kp;
  __shared__ ColCoef<T> s_coef[4][64];
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int gw = blockIdx.x * 4 + wave;
  const int item = gw / NT, stripe = gw - item * NT;
  if (item >= n_items) return;  // whole wavefronts only: no barrier follows
  const int v = item / C, c = item - v * C;
  const int g = lane >> 4, n = lane & 15;
  const int row = 16 * stripe + n;  // row of P this lane's column of X^T belongs to
  const int arow = Mfma<T>::a_row(n);

  acc x[NT], d[NT];
#pragma unroll
  for (int t = 0; t < NT; ++t)
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      x[t][q] = (16 * t + 4 * g + q == row) ? T(1) : T(0);
      d[t][q] = T(0);
    }

  const int seg0 = seg_offset[v];
  const int m = seg_offset[v + 1] - seg0;
  const double rho = cat_rates[c];
  const double scale = rho * rate[v];
  ColCoef<T>* coef = s_coef[wave];
  for (int k = 0; k < m; ++k) {
    const int s = seg_process[seg0 + k];
    const T tau = T(scale * seg_time[seg0 + k]);
    const T dsc = T(rho * seg_frac[seg0 + k]);
    const T* V = eigV + (size_t)s * KK;
    const T* Vi = eigVi + (size_t)s * KK;
    if (lane < Kp) {
      const BlockCoef<T> bc = block_coef(lre + (size_t)s * Kp, lim + (size_t)s * Kp, lane, tau);
      coef[lane] = ColCoef<T>{bc.m_self, bc.m_other, dsc * bc.dm_self, dsc * bc.dm_other};
    }
    __builtin_amdgcn_wave_barrier();

    // Y^T = V^T X^T (and V^T D^T)
    acc y[NT], yd[NT];
#pragma unroll
    for (int mt = 0; mt < NT; ++mt) {
      y[mt] = acc{0, 0, 0, 0};
      if (GRAD) yd[mt] = acc{0, 0, 0, 0};
    }
#pragma unroll
    for (int t = 0; t < NT; ++t)
#pragma unroll
      for (int q = 0; q < 4; ++q) {
        const T* vrow = V + (16 * t + 4 * g + q) * Kp + arow;
#pragma unroll
        for (int mt = 0; mt < NT; ++mt) {
          const T a = vrow[16 * mt];
          y[mt] = Mfma<T>::mma(a, x[t][q], y[mt]);
          if (GRAD) yd[mt] = Mfma<T>::mma(a, d[t][q], yd[mt]);
        }
      }

    // column operator on rows j = 16 mt + 4 g + q of Y^T
#pragma unroll
    for (int mt = 0; mt < NT; ++mt)
#pragma unroll
      for (int q = 0; q < 4; q += 2) {
        const ColCoef<T> c0 = coef[16 * mt + 4 * g + q];
        const ColCoef<T> c1 = coef[16 * mt + 4 * g + q + 1];
        const T y0 = y[mt][q], y1 = y[mt][q + 1];
        y[mt][q] = c0.ms * y0 + c0.mo * y1;
        y[mt][q + 1] = c1.ms * y1 + c1.mo * y0;
        if (GRAD) {
          const T d0 = yd[mt][q], d1 = yd[mt][q + 1];
          yd[mt][q] = c0.ms * d0 + c0.mo * d1 + c0.dms * y0 + c0.dmo * y1;
          yd[mt][q + 1] = c1.ms * d1 + c1.mo * d0 + c1.dms * y1 + c1.dmo * y0;
        }
      }
    __builtin_amdgcn_wave_barrier();

    // X^T += V^-T Y'^T (and D^T += V^-T YD'^T)
#pragma unroll
    for (int t = 0; t < NT; ++t)
#pragma unroll
      for (int q = 0; q < 4; ++q) {
        const T* vrow = Vi + (16 * t + 4 * g + q) * Kp + arow;
#pragma unroll
        for (int mt = 0; mt < NT; ++mt) {
          const T a = vrow[16 * mt];
          x[mt] = Mfma<T>::mma(a, y[t][q], x[mt]);
          if (GRAD) d[mt] = Mfma<T>::mma(a, yd[t][q], d[mt]);
        }
      }
  }

  const size_t base = ((size_t)v * C + c) * KK + (size_t)row * Kp + 4 * g;
#pragma unroll
  for (int mt = 0; mt < NT; ++mt) {
    store4<T, TO>(Pout + base + 16 * mt, x[mt]);
    if (GRAD) store4<T, TO>(dPout + base + 16 * mt, d[mt]);
  }
}

template <typename T, typename TO, int NT>
int pstage_mfma_launch(EpochInstance* in) {
  const int Kp = in->Kp, C = in->C;
  const size_t KK = (size_t)Kp * Kp, S = in->S;
  const bool grad = (in->cfg.flags & (EPOCH_GRAD_BRANCH | EPOCH_GRAD_Q)) != 0;
  const int items = in->n_nodes * C;
  const long waves = (long)items * NT;
  dim3 grid((unsigned)((waves + 3) / 4));
  const T* base = static_cast<const T*>(sizeof(T) == 8 ? in->eig64.ptr : in->eigT.ptr);
  const T* V = base;
  const T* Vi = base + S * KK;
  const T* lr = base + 2 * S * KK;
  const T* li = lr + S * Kp;
  const double* cat = static_cast<const double*>(in->cat.ptr);
  TO* Pout = static_cast<TO*>(in->Pm.ptr);
  TO* dPout = static_cast<TO*>(in->dPm.ptr);
  if (grad)
    hipLaunchKernelGGL((pstage_mfma_kernel<T, TO, true, NT>), grid, dim3(256), 0, in->stream, items, C, V, Vi,
                       lr, li, in->d_seg_offset, in->d_seg_process, in->d_seg_time, in->d_seg_frac, in->d_rate,
                       cat, Pout, dPout);
  else
    hipLaunchKernelGGL((pstage_mfma_kernel<T, TO, false, NT>), grid, dim3(256), 0, in->stream, items, C, V, Vi,
                       lr, li, in->d_seg_offset, in->d_seg_process, in->d_seg_time, in->d_seg_frac, in->d_rate,
                       cat, Pout, dPout);
  return hip_check(hipGetLastError(), "pstage_mfma launch");
}

template <typename T, typename TO>
int pstage_mfma_dispatch(EpochInstance* in) {
  switch (in->Kp) {
    case 16: return pstage_mfma_launch<T, TO, 1>(in);
    case 32: return pstage_mfma_launch<T, TO, 2>(in);
    case 48: return pstage_mfma_launch<T, TO, 3>(in);
    case 64: return pstage_mfma_launch<T, TO, 4>(in);
    default: return set_error(EPOCH_ERR_STATE, "matrix-core P stage needs Kp in {16, 32, 48, 64}, got %d", in->Kp);
  }
}

}  // namespace

bool pstage_mfma_supported(const EpochInstance* in) {
  return in->Kp >= 16 && in->Kp <= 64 && in->Kp % 16 == 0;
}

int launch_pstage_mfma(EpochInstance* in) {
  if (in->fp64) return pstage_mfma_dispatch<double, double>(in);
  return in->eig_fp64 ? pstage_mfma_dispatch<double, float>(in) : pstage_mfma_dispatch<float, float>(in);
}

}  // namespace epochlik
