// Bessel functions J0, J1, Y0, Y1 of a real positive argument in FP64, for the
// 2D Green's function (i/4) H0^(1)(k r) and the cell weights of the discrete
// volume integral operator (Sec. II, "the Green's function ... is
// analytically known").
//
// Method (no vendor special-function library):
//  * x >= 25: Hankel's asymptotic expansion
//      H_nu(x) ~ sqrt(2/(pi x)) (P + i Q) e^{i (x - nu pi/2 - pi/4)},
//      P = sum_k (-1)^k a_2k / x^2k, Q = sum_k (-1)^k a_2k+1 / x^2k+1,
//      a_k(nu) = prod_{m=1..k} (4 nu^2 - (2m-1)^2) / (k! 8^k),
//    summed until the terms fall below 1e-18 (the series is enveloping for real
//    x, and at x >= 25 its smallest term is far below double precision).
//  * 0 < x < 25: Miller's backward recurrence J_{k-1} = (2k/x) J_k - J_{k+1}
//    from an even start index N >= x + 40, normalised by
//    J0 + 2 sum_k J_2k = 1, with Neumann's series
//      Y0 = (2/pi)(ln(x/2) + gamma) J0 - (4/pi) sum_k (-1)^k J_2k / k,
//    and its derivative (Y1 = -Y0')
//      Y1 = (2/pi)((ln(x/2) + gamma) J1 - J0/x)
//           + (2/pi) sum_k (-1)^k (J_2k-1 - J_2k+1) / k.
// Host-callable so it can be checked on the CPU against an independent library.
#pragma once

#include <hip/hip_runtime.h>
#include <cmath>

namespace fwi {

__host__ __device__ inline void bessel01(double x, double* j0, double* j1, double* y0, double* y1) {
  const double PI = 3.14159265358979323846;
  const double EULER = 0.57721566490153286061;
  if (x >= 25.0) {
    double P0 = 1.0, Q0 = 0.0, P1 = 1.0, Q1 = 0.0;
    double t0 = 1.0, t1 = 1.0;
    for (int k = 1; k <= 60; ++k) {
      const double f = (double)(2 * k - 1) * (double)(2 * k - 1);
      t0 *= (0.0 - f) / (8.0 * k * x);
      t1 *= (4.0 - f) / (8.0 * k * x);
      // P takes even k with sign (-1)^(k/2); Q takes odd k with sign (-1)^((k-1)/2)
      if (k & 1) {
        const double s = ((k - 1) / 2) & 1 ? -1.0 : 1.0;
        Q0 += s * t0;
        Q1 += s * t1;
      } else {
        const double s = (k / 2) & 1 ? -1.0 : 1.0;
        P0 += s * t0;
        P1 += s * t1;
      }
      if (fabs(t0) < 1e-18 && fabs(t1) < 1e-18) break;
    }
    double s, c;
    sincos(x, &s, &c);
    const double r2 = 0.70710678118654752440;
    const double c0 = (c + s) * r2, s0 = (s - c) * r2;     // chi = x - pi/4
    const double c1 = (s - c) * r2, s1 = -(s + c) * r2;    // chi = x - 3 pi/4
    const double amp = sqrt(2.0 / (PI * x));
    *j0 = amp * (P0 * c0 - Q0 * s0);
    *y0 = amp * (P0 * s0 + Q0 * c0);
    *j1 = amp * (P1 * c1 - Q1 * s1);
    *y1 = amp * (P1 * s1 + Q1 * c1);
    return;
  }
  const int N = 2 * ((int)x + 20);  // even, >= x + 40
  double fp = 0.0, fc = 1.0;        // f_{k+1}, f_k with k = N
  double S = 2.0 * fc;              // J0 + 2 sum J_2k (N even)
  double sy0 = (((N / 2) & 1) ? -1.0 : 1.0) * fc / (N / 2);
  double sy1 = 0.0;
  double fodd = 0.0;                // f_{m+2} for odd m (f_{N+1} = 0)
  double f1 = 0.0;
  for (int k = N; k >= 1; --k) {
    const double fm = (2.0 * k / x) * fc - fp;
    fp = fc;
    fc = fm;
    const int m = k - 1;
    if (m & 1) {
      const int kk = (m + 1) / 2;
      sy1 += ((kk & 1) ? -1.0 : 1.0) * (fc - fodd) / kk;
      fodd = fc;
      if (m == 1) f1 = fc;
    } else if (m >= 2) {
      S += 2.0 * fc;
      sy0 += (((m / 2) & 1) ? -1.0 : 1.0) * fc / (m / 2);
    } else {
      S += fc;
    }
    if (fabs(fc) > 1e250) {
      const double sc = 1e-250;
      fc *= sc; fp *= sc; fodd *= sc; f1 *= sc; S *= sc; sy0 *= sc; sy1 *= sc;
    }
  }
  const double J0 = fc / S, J1 = f1 / S;
  const double lg = log(0.5 * x) + EULER;
  *j0 = J0;
  *j1 = J1;
  *y0 = (2.0 / PI) * lg * J0 - (4.0 / PI) * sy0 / S;
  *y1 = (2.0 / PI) * (lg * J1 - J0 / x) + (2.0 / PI) * sy1 / S;
}

}  // namespace fwi
