// Toeplitz symbol of the free-space Graf translation between two particles
// (Section 4.2), shared by the direct / near-field kernels and the assembly of
// the preconditioner's cluster blocks.
#pragma once

#include "dev.h"

namespace ems {

// Toeplitz symbol of one pair and wave number: t[2 PM + nu] = H_nu(k d)
// e^{-i nu (th - pi)} for |nu| <= 2 PM, (d, th) the polar form of (dx, dy),
// Hankel functions by forward recurrence from H_0, H_1 (stable because
// |Y_nu| dominates).
template <int PM, typename T, typename Cvt>
__device__ __forceinline__ void graf_symbol(double dx, double dy, double k, T *t, Cvt cvt) {
  const double d = sqrt(dx * dx + dy * dy);
  const double th = atan2(dy, dx);
  const double z = k * d;
  double sn, cs;
  sincos(th, &sn, &cs);
  const double2 e1 = make_double2(-cs, sn);  // e^{-i (th - pi)}
  double2 hm = make_double2(j0(z), y0(z));
  double2 h = make_double2(j1(z), y1(z));
  t[2 * PM] = cvt(hm);
  double2 ph = e1;
  t[2 * PM + 1] = cvt(cmul(h, ph));
  // t_{-nu} = (-1)^nu H_nu conj(e^{-i nu (th - pi)})
  t[2 * PM - 1] = cvt(cscale(cmul(h, cconj(ph)), -1.0));
  const double iz = 2.0 / z;
#pragma unroll
  for (int nu = 2; nu <= 2 * PM; ++nu) {
    const double2 hn = csub(cscale(h, (nu - 1) * iz), hm);
    hm = h;
    h = hn;
    ph = cmul(ph, e1);
    t[2 * PM + nu] = cvt(cmul(h, ph));
    const double sg = (nu & 1) ? -1.0 : 1.0;
    t[2 * PM - nu] = cvt(cscale(cmul(h, cconj(ph)), sg));
  }
}

}  // namespace ems
