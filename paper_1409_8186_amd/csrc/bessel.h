// FP64 integer-order Bessel J_n and Hankel H^(1)_n = J_n + i Y_n on the device.
//
// Written from the published methods, not from any library's internals:
//  * J_0..J_nmax(x): Miller's downward recurrence J_{n-1} = (2n/x) J_n - J_{n+1}
//    from a start order above max(nmax, x), normalised by
//    J_0 + 2 sum_{k>=1} J_{2k} = 1 (relative accuracy at every order).
//  * Y_0, Y_1 for x < X_ASY: Neumann series in the same J's,
//      Y_0 = (2/pi)(ln(x/2)+gamma) J_0 - (4/pi) sum_{k>=1} (-1)^k J_{2k}/k,
//      Y_1 = -Y_0' = -(2/pi) J_0/x + (2/pi)(ln(x/2)+gamma) J_1
//            + (2/pi) sum_{k>=1} (-1)^k (J_{2k-1} - J_{2k+1})/k.
//  * H_0, H_1 for x >= X_ASY: Hankel's large-argument expansion (DLMF 10.17.5)
//      H_nu(x) ~ sqrt(2/(pi x)) e^{i(x - nu pi/2 - pi/4)} sum_k i^k a_k(nu) / x^k,
//      a_k(nu) = prod_{j=1..k} (4 nu^2 - (2j-1)^2) / (k! 8^k),
//    with e^{ix} taken from sincos of the exact argument (the phase x - pi/4
//    formed in floating point would lose ~x ulp).
//  * Y_n (and H_n) for n >= 2: upward recurrence, stable for Y.
#pragma once

#include "common.h"

#define BESSEL_X_ASY 25.0

// Miller's algorithm.  Writes J_n(x) for n = 0..nmax to J[n * stride] and the
// Neumann sums S0 = sum_{k>=1} (-1)^k J_{2k}/k and
// S1 = sum_{k>=1} (-1)^k (J_{2k-1} - J_{2k+1})/k.  x > 0.
__device__ inline void bessel_j_miller(double x, int nmax, double* J, int stride, double* S0,
                                       double* S1) {
  int n0 = nmax > (int)x + 1 ? nmax : (int)x + 1;
  int nstart = 2 * ((n0 + (int)sqrt(160.0 * n0) + 16) / 2);
  double jp1 = 0.0, j = 1.0;  // J_{n+1}, J_n (unnormalised)
  double norm = 0.0, s0 = 0.0, s1 = 0.0;
  const double two_over_x = 2.0 / x;
  for (int n = nstart; n > 0; --n) {
    if (n <= nmax) J[(int64_t)n * stride] = j;
    if ((n & 1) == 0) {
      int kk = n >> 1;
      norm += 2.0 * j;
      s0 += ((kk & 1) ? -j : j) / kk;
    } else {
      int kk = (n - 1) >> 1;  // n = 2kk + 1: coefficient of J_{2kk+1} in S1
      if (kk == 0)
        s1 -= j;
      else
        s1 += (((kk + 1) & 1) ? -1.0 : 1.0) * (1.0 / kk + 1.0 / (kk + 1)) * j;
    }
    double jm1 = (double)n * two_over_x * j - jp1;
    jp1 = j;
    j = jm1;
    if (fabs(j) > 1e200) {  // rescale everything accumulated so far
      const double sc = 1e-200;
      j *= sc;
      jp1 *= sc;
      norm *= sc;
      s0 *= sc;
      s1 *= sc;
      int top = n - 1 < nmax ? n - 1 : nmax;
      for (int i = top + 1; i <= nmax; ++i) J[(int64_t)i * stride] *= sc;
    }
  }
  // j = J_0 (unnormalised)
  J[0] = j;
  norm += j;
  const double inv = 1.0 / norm;
  for (int i = 0; i <= nmax; ++i) J[(int64_t)i * stride] *= inv;
  *S0 = s0 * inv;
  *S1 = s1 * inv;
}

__device__ inline void bessel_y01_neumann(double x, double J0, double J1, double S0, double S1,
                                          double* Y0, double* Y1) {
  const double two_pi = 0.63661977236758134308;  // 2/pi
  const double euler = 0.57721566490153286061;
  double lg = log(0.5 * x) + euler;
  *Y0 = two_pi * lg * J0 - 2.0 * two_pi * S0;
  *Y1 = -two_pi * J0 / x + two_pi * lg * J1 + two_pi * S1;
}

// Hankel's expansion of H_0(x), H_1(x), x >= BESSEL_X_ASY.
__device__ inline void hankel01_asym(double x, cplx* H0, cplx* H1) {
  const double pi = 3.14159265358979323846;
  const double r2 = 0.70710678118654752440;
  cplx s[2];
  for (int nu = 0; nu < 2; ++nu) {
    double mu = 4.0 * nu * nu;
    cplx term = cmk(1.0, 0.0), sum = term;
    for (int kk = 1; kk <= 80; ++kk) {
      double f = (mu - (2.0 * kk - 1.0) * (2.0 * kk - 1.0)) / (8.0 * kk * x);
      term = cmk(-term.y * f, term.x * f);  // * i * f
      sum = cadd(sum, term);
      if (cabs2(term) < 1e-34 * cabs2(sum)) break;
    }
    s[nu] = sum;
  }
  double sn, cs;
  sincos(x, &sn, &cs);
  double amp = sqrt(2.0 / (pi * x));
  cplx e = cmk(amp * cs, amp * sn);
  // e^{-i pi/4} and e^{-3 i pi/4}
  *H0 = cmul(cmul(e, cmk(r2, -r2)), s[0]);
  *H1 = cmul(cmul(e, cmk(-r2, -r2)), s[1]);
}

// H_0(x), H_1(x) for any x > 0.
__device__ inline void hankel01(double x, cplx* H0, cplx* H1) {
  if (x >= BESSEL_X_ASY) {
    hankel01_asym(x, H0, H1);
    return;
  }
  double J[2], S0, S1, Y0, Y1;
  bessel_j_miller(x, 1, J, 1, &S0, &S1);
  bessel_y01_neumann(x, J[0], J[1], S0, S1, &Y0, &Y1);
  *H0 = cmk(J[0], Y0);
  *H1 = cmk(J[1], Y1);
}
