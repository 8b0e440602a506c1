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

// The same functions of a complex argument z (|arg z| < pi/2; the lossy 2D
// background has k r just above the real axis), by the same two methods with
// complex arithmetic: Hankel's expansion for |z| >= 25, Miller's backward
// recurrence with the same normalisation and Neumann's series (principal
// logarithm) below. Outputs are (re, im) pairs.
struct cz {
  double re, im;
};
__host__ __device__ inline cz czm(double a, double b) { return cz{a, b}; }
__host__ __device__ inline cz operator+(cz a, cz b) { return cz{a.re + b.re, a.im + b.im}; }
__host__ __device__ inline cz operator-(cz a, cz b) { return cz{a.re - b.re, a.im - b.im}; }
__host__ __device__ inline cz operator*(cz a, cz b) { return cz{a.re * b.re - a.im * b.im, a.re * b.im + a.im * b.re}; }
__host__ __device__ inline cz operator*(double s, cz a) { return cz{s * a.re, s * a.im}; }
__host__ __device__ inline cz czdiv(cz a, cz b) {
  // scaled division (Smith's method)
  if (fabs(b.re) >= fabs(b.im)) {
    const double r = b.im / b.re, d = b.re + r * b.im;
    return cz{(a.re + r * a.im) / d, (a.im - r * a.re) / d};
  }
  const double r = b.re / b.im, d = b.im + r * b.re;
  return cz{(r * a.re + a.im) / d, (r * a.im - a.re) / d};
}
__host__ __device__ inline double czabs(cz a) { return hypot(a.re, a.im); }
__host__ __device__ inline cz czsqrt(cz a) {
  const double m = czabs(a);
  const double re = sqrt(0.5 * (m + a.re)), im = sqrt(0.5 * (m - a.re));
  return cz{re, a.im < 0.0 ? -im : im};
}
__host__ __device__ inline cz czlog(cz a) { return cz{log(czabs(a)), atan2(a.im, a.re)}; }

__host__ __device__ inline void cbessel01(cz z, cz* j0, cz* j1, cz* y0, cz* y1) {
  const double PI = 3.14159265358979323846;
  const double EULER = 0.57721566490153286061;
  const double az = czabs(z);
  if (az >= 25.0) {
    const cz iz = czdiv(czm(1.0, 0.0), z);
    cz P0 = czm(1.0, 0.0), Q0 = czm(0.0, 0.0), P1 = czm(1.0, 0.0), Q1 = czm(0.0, 0.0);
    cz t0 = czm(1.0, 0.0), t1 = czm(1.0, 0.0);
    for (int k = 1; k <= 60; ++k) {
      const double f = (double)(2 * k - 1) * (double)(2 * k - 1);
      t0 = ((0.0 - f) / (8.0 * k)) * (t0 * iz);
      t1 = ((4.0 - f) / (8.0 * k)) * (t1 * iz);
      if (k & 1) {
        const double s = ((k - 1) / 2) & 1 ? -1.0 : 1.0;
        Q0 = Q0 + s * t0;
        Q1 = Q1 + s * t1;
      } else {
        const double s = (k / 2) & 1 ? -1.0 : 1.0;
        P0 = P0 + s * t0;
        P1 = P1 + s * t1;
      }
      if (czabs(t0) < 1e-18 && czabs(t1) < 1e-18) break;
    }
    // cos z, sin z of the complex argument
    double s, c;
    sincos(z.re, &s, &c);
    const double ch = cosh(z.im), sh = sinh(z.im);
    const cz cs = czm(c * ch, -s * sh), sn = czm(s * ch, c * sh);
    const double r2 = 0.70710678118654752440;
    const cz c0 = r2 * (cs + sn), s0 = r2 * (sn - cs);                  // chi = z - pi/4
    const cz c1 = r2 * (sn - cs), s1 = (-r2) * (sn + cs);               // chi = z - 3 pi/4
    const cz amp = czsqrt(czdiv(czm(2.0 / PI, 0.0), z));
    *j0 = amp * (P0 * c0 - Q0 * s0);
    *y0 = amp * (P0 * s0 + Q0 * c0);
    *j1 = amp * (P1 * c1 - Q1 * s1);
    *y1 = amp * (P1 * s1 + Q1 * c1);
    return;
  }
  const cz iz = czdiv(czm(1.0, 0.0), z);
  const int N = 2 * ((int)az + 20);
  cz fp = czm(0.0, 0.0), fc = czm(1.0, 0.0);
  cz S = czm(2.0, 0.0);
  cz sy0 = ((((N / 2) & 1) ? -1.0 : 1.0) / (N / 2)) * fc;
  cz sy1 = czm(0.0, 0.0), fodd = czm(0.0, 0.0), f1 = czm(0.0, 0.0);
  for (int k = N; k >= 1; --k) {
    const cz fm = (2.0 * k) * (iz * fc) - fp;
    fp = fc;
    fc = fm;
    const int m = k - 1;
    if (m & 1) {
      const int kk = (m + 1) / 2;
      sy1 = sy1 + (((kk & 1) ? -1.0 : 1.0) / kk) * (fc - fodd);
      fodd = fc;
      if (m == 1) f1 = fc;
    } else if (m >= 2) {
      S = S + 2.0 * fc;
      sy0 = sy0 + ((((m / 2) & 1) ? -1.0 : 1.0) / (m / 2)) * fc;
    } else {
      S = S + fc;
    }
    if (czabs(fc) > 1e250) {
      const double sc = 1e-250;
      fc = sc * fc; fp = sc * fp; fodd = sc * fodd; f1 = sc * f1; S = sc * S; sy0 = sc * sy0; sy1 = sc * sy1;
    }
  }
  const cz J0 = czdiv(fc, S), J1 = czdiv(f1, S);
  const cz lg = czlog(0.5 * z) + czm(EULER, 0.0);
  *j0 = J0;
  *j1 = J1;
  *y0 = (2.0 / PI) * (lg * J0) - (4.0 / PI) * czdiv(sy0, S);
  *y1 = (2.0 / PI) * (lg * J1 - J0 * iz) + (2.0 / PI) * czdiv(sy1, S);
}

// H0^(1)(z) = J0 + i Y0, the 2D Green's function's Hankel function, for a
// complex argument: for |z| >= 25 straight from Hankel's expansion,
// sqrt(2/(pi z)) (P0 + i Q0) e^{i (z - pi/4)} (no cancellation between J0 and
// Y0, which both grow like e^{Im z}; from |z| >= 15 when Im z >= 1); below
// from cbessel01.
__host__ __device__ inline cz chankel0(cz z) {
  const double PI = 3.14159265358979323846;
  const double az = czabs(z);
  // J0 + i Y0 loses e^{2 Im z} to cancellation: the expansion (error about
  // e^{-2|z|}) takes over from |z| = 15 once Im z >= 1
  if (az < 15.0 || (az < 25.0 && z.im < 1.0)) {
    cz j0, j1, y0, y1;
    cbessel01(z, &j0, &j1, &y0, &y1);
    return cz{j0.re - y0.im, j0.im + y0.re};
  }
  const cz iz = czdiv(czm(1.0, 0.0), z);
  cz P = czm(1.0, 0.0), Q = czm(0.0, 0.0), t = czm(1.0, 0.0);
  for (int k = 1; k <= 60; ++k) {
    const double f = (double)(2 * k - 1) * (double)(2 * k - 1);
    t = (-f / (8.0 * k)) * (t * iz);
    if (k & 1) Q = Q + ((((k - 1) / 2) & 1) ? -1.0 : 1.0) * t;
    else P = P + (((k / 2) & 1) ? -1.0 : 1.0) * t;
    if (czabs(t) < 1e-18) break;
  }
  double s, c;
  sincos(z.re - 0.25 * PI, &s, &c);
  const double d = exp(-z.im);
  const cz e = czm(d * c, d * s);
  const cz amp = czsqrt(czdiv(czm(2.0 / PI, 0.0), z));
  return amp * ((P + czm(-Q.im, Q.re)) * e);
}

}  // namespace fwi
