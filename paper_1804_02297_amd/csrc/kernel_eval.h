// Device evaluation of the Nystrom weights of the dyadic Green's tensor.
//
// For r != 0: K(r) = h^3 G(R) [ (k^2 + ik/R - 1/R^2) I + (-k^2 - 3ik/R + 3/R^2) xhat xhat^T ]
// with x = h r, R = |x|, G = exp(ikR)/(4 pi R), i.e. h^3 (k^2 I + grad grad) G
// (Section 2: Helmholtz kernel; Nystrom weights h^3 G(ih - jh)).
// K(0) = {(2/3)[(1 - ika) e^{ika} - 1] - 1/3} I, a = h (3/(4 pi))^(1/3): the
// principal-value integral over the equal-volume ball plus the -1/3
// depolarisation term (the paper's near-diagonal correction is not given).
// Components are returned as (xx, yy, zz, xy, xz, yz).
#pragma once

#include "cplx.h"

namespace ls {

__device__ inline void dyadic_K(int r1, int r2, int r3, double k, double h, C<double> out[6]) {
  if (r1 == 0 && r2 == 0 && r3 == 0) {
    const double a = h * cbrt(3.0 / (4.0 * kPi));
    double sn, cs;
    sincos(k * a, &sn, &cs);
    const double br = cs + k * a * sn - 1.0, bi = sn - k * a * cs;   // (1 - ika) e^{ika} - 1
    const C<double> d = cmk((2.0 / 3.0) * br - 1.0 / 3.0, (2.0 / 3.0) * bi);
    out[0] = d;
    out[1] = d;
    out[2] = d;
    out[3] = out[4] = out[5] = cmk(0.0, 0.0);
    return;
  }
  const double x0 = h * r1, x1 = h * r2, x2 = h * r3;
  const double R2 = x0 * x0 + x1 * x1 + x2 * x2;
  const double R = sqrt(R2);
  double sn, cs;
  sincos(k * R, &sn, &cs);
  const double g = h * h * h / (4.0 * kPi * R);
  const C<double> G = cmk(cs * g, sn * g);
  const C<double> ciso = G * cmk(k * k - 1.0 / R2, k / R);
  const C<double> crad = G * cmk(-k * k + 3.0 / R2, -3.0 * k / R);
  const double u0 = x0 / R, u1 = x1 / R, u2 = x2 / R;
  out[0] = ciso + cscale(crad, u0 * u0);
  out[1] = ciso + cscale(crad, u1 * u1);
  out[2] = ciso + cscale(crad, u2 * u2);
  out[3] = cscale(crad, u0 * u1);
  out[4] = cscale(crad, u0 * u2);
  out[5] = cscale(crad, u1 * u2);
}

// index into (xx, yy, zz, xy, xz, yz) of entry (a, b)
__host__ __device__ inline int sym_index(int a, int b) {
  if (a == b) return a;
  const int lo = a < b ? a : b, hi = a < b ? b : a;
  return lo == 0 ? (hi == 1 ? 3 : 4) : 5;
}

}  // namespace ls
