// Column operator of exp(tau Q) in the eigen basis, shared by the P-stage
// kernels (Eq. 3 with the real 2x2 rotation blocks of complex pairs).
#pragma once
#include <hip/hip_runtime.h>

#include "device_common.h"

namespace epochlik {

// ---------------------------------------------------------------------------
// Eigen-basis column operator.  exp(tau Q) = I + V (E(tau) - I) V^-1 where E is
// exp(lambda tau) for a real eigenvalue and, for a pair (a +- ib) in columns
// (j, j+1), the block exp(a tau) [[cos b tau, sin b tau], [-sin b tau, cos b tau]].
// Working with E - I (expm1 on the diagonal) keeps the rounding error relative
// to the departure from the identity, which is small on short branches.
// ---------------------------------------------------------------------------
template <typename T>
struct BlockCoef {
  T m_self, m_other;    // (E - I) applied to a row: x'_j = m_self * x_j + m_other * x_partner
  T dm_self, dm_other;  // d/dtau of E (unit rate)
  int partner;          // -1 for a real eigenvalue
};

template <typename T>
__device__ inline BlockCoef<T> block_coef(const T* lr, const T* li, int j, T tau) {
  BlockCoef<T> r;
  T b = li[j];
  if (b == T(0)) {
    const T x = lr[j] * tau;
    r.m_self = dev_expm1(x);
    r.m_other = 0;
    r.dm_self = lr[j] * (r.m_self + T(1));
    r.dm_other = 0;
    r.partner = -1;
    return r;
  }
  const bool first = b > T(0);
  const int jp = first ? j + 1 : j - 1;
  const T a = lr[j];
  const T bb = first ? b : -b;  // the positive imaginary part
  const T em1 = dev_expm1(a * tau);
  const T ea = em1 + T(1);
  const T cs = dev_cos(bb * tau), sn = dev_sin(bb * tau);
  const T hs = dev_sin(T(0.5) * bb * tau);
  // M = ea [[c, s], [-s, c]]; M - I has diagonal ea c - 1 = em1 c - 2 sin^2(b tau / 2)
  const T diag_m1 = em1 * cs - T(2) * hs * hs;
  // first column (j is first):  x'_j = M00 x_j + M10 x_{j+1};  second: x'_j = M01 x_{j-1} + M11 x_j
  const T dM00 = ea * (a * cs - bb * sn), dM01 = ea * (a * sn + bb * cs);
  const T dM10 = ea * (-bb * cs - a * sn), dM11 = ea * (-bb * sn + a * cs);
  r.m_self = diag_m1;
  if (first) {
    r.m_other = -ea * sn;
    r.dm_self = dM00;
    r.dm_other = dM10;
  } else {
    r.m_other = ea * sn;
    r.dm_self = dM11;
    r.dm_other = dM01;
  }
  r.partner = jp;
  return r;
}

}  // namespace epochlik
