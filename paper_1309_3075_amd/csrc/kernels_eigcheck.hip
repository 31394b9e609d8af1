// FP64 check of an eigensystem against its rate matrix.  One decomposition of
// each Q_s serves every rate and time (Appendix A), so it is checked once, on
// the device and in FP64:
//   R = V B V^-1 - Q   (B: the eigenvalues in real form, 2x2 rotation blocks
//                       [[a, b], [-b, a]] for a complex pair a +- ib)
//   E = V V^-1 - I
// residual = max(max|R| / max|Q|, max|E|)  (max|R| itself when Q is zero).
//
// A block forms one 16 x 16 tile of R and E for one system from LDS-staged
// tiles of V B, V and V^-1 (the contraction runs over the states in order)
// and writes the tile's three maxima to a scratch row; a second launch folds
// each system's tiles.  Maxima do not round, so the result does not depend on
// the tiling.
#include <hip/hip_runtime.h>

#include <cmath>
#include <mutex>

#include "instance.h"

namespace epochlik {

namespace {

constexpr int kTile = 16;

__global__ __launch_bounds__(256) void eigen_check_tile_kernel(const double* __restrict__ V,
                                                               const double* __restrict__ Vi,
                                                               const double* __restrict__ lr,
                                                               const double* __restrict__ li,
                                                               const double* __restrict__ Q, int K, int ld,
                                                               long mat_stride, int vec_stride,
                                                               double* __restrict__ part,
                                                               double* __restrict__ rec_out) {
  const int s = blockIdx.y;
  const int nt = (K + kTile - 1) / kTile;
  const int ti = blockIdx.x / nt, tj = blockIdx.x % nt;
  const int ty = threadIdx.x / kTile, tx = threadIdx.x % kTile;
  V += s * mat_stride;
  Vi += s * mat_stride;
  lr += (long)s * vec_stride;
  if (li) li += (long)s * vec_stride;
  if (Q) Q += (long)s * K * K;
  __shared__ double sVB[kTile][kTile + 1], sV[kTile][kTile + 1], sVi[kTile][kTile + 1];
  double rec = 0.0, id = 0.0;
  for (int l0 = 0; l0 < K; l0 += kTile) {
    {
      // row ty of this tile's V and V B, columns l0 .. l0 + 15
      const int gi = ti * kTile + ty, gl = l0 + tx;
      double v = 0.0, vb = 0.0;
      if (gi < K && gl < K) {
        v = V[(long)gi * ld + gl];
        const double b = li ? li[gl] : 0.0;
        // a pair's partner column always lies inside the matrix (a malformed pair at the edge
        // is taken as a real eigenvalue, which the residual then reports)
        if (b > 0.0 && gl + 1 < K)
          vb = v * lr[gl] - V[(long)gi * ld + gl + 1] * b;   // first column of a pair of V B
        else if (b < 0.0 && gl > 0)
          vb = -V[(long)gi * ld + gl - 1] * b + v * lr[gl];  // second column of the pair
        else
          vb = v * lr[gl];
      }
      sV[ty][tx] = v;
      sVB[ty][tx] = vb;
      // row l0 + ty of V^-1, columns of this tile
      const int gr = l0 + ty, gj = tj * kTile + tx;
      sVi[ty][tx] = (gr < K && gj < K) ? Vi[(long)gr * ld + gj] : 0.0;
    }
    __syncthreads();
    const int lend = min(kTile, K - l0);
    for (int l = 0; l < lend; ++l) {
      rec += sVB[ty][l] * sVi[l][tx];
      id += sV[ty][l] * sVi[l][tx];
    }
    __syncthreads();
  }
  const int i = ti * kTile + ty, j = tj * kTile + tx;
  double vals[3] = {0.0, 0.0, 0.0};
  if (i < K && j < K) {
    const double q = Q ? Q[i * K + j] : 0.0;
    vals[0] = fabs(rec - q);
    vals[1] = fabs(id - (i == j ? 1.0 : 0.0));
    vals[2] = fabs(q);
    if (rec_out) rec_out[s * mat_stride + (long)i * ld + j] = rec;  // Q_s = V B V^-1, same layout as V
  }
  __shared__ double sm[256];
  for (int q = 0; q < 3; ++q) {
    sm[threadIdx.x] = vals[q];
    __syncthreads();
    for (int w = 128; w > 0; w >>= 1) {
      if (threadIdx.x < w) sm[threadIdx.x] = fmax(sm[threadIdx.x], sm[threadIdx.x + w]);
      __syncthreads();
    }
    if (threadIdx.x == 0) part[((long)s * gridDim.x + blockIdx.x) * 3 + q] = sm[0];
    __syncthreads();
  }
}

__global__ __launch_bounds__(256) void eigen_check_finish_kernel(const double* __restrict__ part, int tiles, int n,
                                                                 double* __restrict__ out) {
  for (int s = blockIdx.x * 256 + threadIdx.x; s < n; s += 256 * gridDim.x) {
    double r1 = 0.0, r2 = 0.0, qm = 0.0;
    for (int t = 0; t < tiles; ++t) {
      const double* p = part + ((long)s * tiles + t) * 3;
      r1 = fmax(r1, p[0]);
      r2 = fmax(r2, p[1]);
      qm = fmax(qm, p[2]);
    }
    out[s] = fmax(qm > 0.0 ? r1 / qm : r1, r2);
  }
}

}  // namespace

int eigen_check_tiles(int K) {
  const int nt = (K + kTile - 1) / kTile;
  return nt * nt;
}

int launch_eigen_check_n(hipStream_t st, int K, int n, int ld, long mat_stride, int vec_stride, const double* V,
                         const double* Vi, const double* lr, const double* li, const double* Q, double* part,
                         double* out) {
  const int tiles = eigen_check_tiles(K);
  hipLaunchKernelGGL(eigen_check_tile_kernel, dim3(tiles, n), dim3(256), 0, st, V, Vi, lr, li, Q, K, ld, mat_stride,
                     vec_stride, part, nullptr);
  int rc = hip_check(hipGetLastError(), "eigen check launch");
  if (rc) return rc;
  hipLaunchKernelGGL(eigen_check_finish_kernel, dim3((n + 255) / 256), dim3(256), 0, st, part, tiles, n, out);
  return hip_check(hipGetLastError(), "eigen check finish launch");
}

int launch_q_reconstruct(EpochInstance* in, double* d_Q, double* part) {
  // every process's Q_s = V B V^-1 in FP64, padded layout [S][Kp][Kp] (padding left as it is)
  const size_t KK = (size_t)in->Kp * in->Kp;
  const double* base = static_cast<const double*>(in->eig64.ptr);
  const double* lr = base + 2 * in->S * KK;
  const double* li = lr + (size_t)in->S * in->Kp;
  hipLaunchKernelGGL(eigen_check_tile_kernel, dim3(eigen_check_tiles(in->K), in->S), dim3(256), 0, in->stream, base,
                     base + in->S * KK, lr, li, (const double*)nullptr, in->K, in->Kp, (long)KK, in->Kp, part, d_Q);
  return hip_check(hipGetLastError(), "Q reconstruction launch");
}

int launch_eigen_check(EpochInstance* in, int s, const double* dQ, double* d_out) {
  // the instance's FP64 eigensystem slices (padded, device column order); scratch follows the output
  const size_t KK = (size_t)in->Kp * in->Kp;
  const double* base = static_cast<const double*>(in->eig64.ptr);
  const double* V = base + s * KK;
  const double* Vi = base + in->S * KK + s * KK;
  const double* lr = base + 2 * in->S * KK + (size_t)s * in->Kp;
  const double* li = base + 2 * in->S * KK + (size_t)in->S * in->Kp + (size_t)s * in->Kp;
  return launch_eigen_check_n(in->stream, in->K, 1, in->Kp, (long)KK, in->Kp, V, Vi, lr, li, dQ, d_out + 1, d_out);
}

// ---- The check without allocation (epoch_eigen_residual_noalloc) ---------------------------
// The tile maxima live in a file-scope device array instead of library-allocated memory.  In
// host code `scratch` names a host-side stand-in, not device memory: the device address of each
// GPU's copy comes from hipGetSymbolAddress, taken once per device with that device current,
// and only that address is handed to kernels.
namespace {

constexpr size_t kNoAllocScratchDoubles = 131072;  // 1 MiB per device
static __device__ __align__(256) double scratch[kNoAllocScratchDoubles];

constexpr int kNoAllocMaxDevices = 64;
std::mutex g_scratch_mutex;
double* g_scratch_ptr[kNoAllocMaxDevices] = {};

int scratch_address(int device, double** out) {
  std::lock_guard<std::mutex> lock(g_scratch_mutex);
  if (!g_scratch_ptr[device]) {
    void* p = nullptr;
    const int rc = hip_check(hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)), "hipGetSymbolAddress(scratch)");
    if (rc) return rc;
    if (!p) return set_error(EPOCH_ERR_HIP, "hipGetSymbolAddress(scratch) returned a null address");
    g_scratch_ptr[device] = static_cast<double*>(p);
  }
  *out = g_scratch_ptr[device];
  return EPOCH_OK;
}

// The pointer must be device memory of the current device (a host pointer would fault the GPU).
int check_device_pointer(const void* p, int device, const char* name) {
  hipPointerAttribute_t attr;
  if (hipPointerGetAttributes(&attr, p) != hipSuccess) {
    (void)hipGetLastError();
    return set_error(EPOCH_ERR_ARG, "%s is not device memory", name);
  }
  if (attr.type != hipMemoryTypeDevice || attr.device != device)
    return set_error(EPOCH_ERR_ARG, "%s is not device memory of the current device", name);
  return EPOCH_OK;
}

}  // namespace
}  // namespace epochlik

using namespace epochlik;

extern "C" int epoch_eigen_residual_noalloc(int32_t n_states, int32_t n_systems, const double* V,
                                            const double* Vinv, const double* lambda_re,
                                            const double* lambda_im, const double* Q, double* residual,
                                            void* stream) {
  if (n_states < 2 || n_states > 64) return set_error(EPOCH_ERR_ARG, "n_states must be in [2, 64] (got %d)", n_states);
  if (n_systems < 1) return set_error(EPOCH_ERR_ARG, "n_systems must be >= 1 (got %d)", n_systems);
  if (!V || !Vinv || !lambda_re || !Q || !residual)
    return set_error(EPOCH_ERR_ARG, "V, Vinv, lambda_re, Q and residual must not be NULL");
  const size_t per_system = 3 * (size_t)eigen_check_tiles(n_states);
  if ((size_t)n_systems * per_system > kNoAllocScratchDoubles)
    return set_error(EPOCH_ERR_ARG,
                     "%d systems of %d states need %zu scratch doubles; the fixed scratch holds %zu "
                     "(at most %zu systems of this size per call)",
                     n_systems, n_states, (size_t)n_systems * per_system, kNoAllocScratchDoubles,
                     kNoAllocScratchDoubles / per_system);
  int device = 0;
  int rc = hip_check(hipGetDevice(&device), "hipGetDevice");
  if (rc) return rc;
  if (device < 0 || device >= kNoAllocMaxDevices)
    return set_error(EPOCH_ERR_ARG, "device %d beyond the %d devices this entry point serves", device,
                     kNoAllocMaxDevices);
  const void* ptrs[] = {V, Vinv, lambda_re, Q, residual, lambda_im};
  const char* names[] = {"V", "Vinv", "lambda_re", "Q", "residual", "lambda_im"};
  for (int k = 0; k < 6; ++k) {
    if (!ptrs[k]) continue;
    rc = check_device_pointer(ptrs[k], device, names[k]);
    if (rc) return rc;
  }
  double* part = nullptr;
  rc = scratch_address(device, &part);
  if (rc) return rc;
  const long KK = (long)n_states * n_states;
  return launch_eigen_check_n(static_cast<hipStream_t>(stream), n_states, n_systems, n_states, KK, n_states, V, Vinv,
                              lambda_re, lambda_im, Q, part, residual);
}
