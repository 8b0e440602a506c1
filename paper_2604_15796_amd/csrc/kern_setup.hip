// Set-up kernels: contrast (Eq. 1-3), the circulant Green table of the
// discrete volume integral operator (Eq. 5, Sec. IV-A) and the incident fields
// of point elements (Sec. II). All evaluated in FP64.
#include <algorithm>
#include <complex>

#include "bessel.hpp"
#include "internal.hpp"

namespace fwi {

constexpr double PI = 3.14159265358979323846;

// m = kappa/kappa0 - 1 with kappa rho0 = 1/c^2 - alpha^2/(2 pi)^2 + i alpha/(pi c)
// (e^{-i omega t}) and the background kappa0 rho0 from (c0, alpha0).
__global__ void k_contrast(long n, double c0, double a0, const double* __restrict__ c,
                           const double* __restrict__ alpha, c128* __restrict__ m64, c64* __restrict__ m32) {
  const long i = (long)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  const double cc = c[i], a = alpha ? alpha[i] : 0.0;
  double re, im;
  if (a0 == 0.0) {
    // c0^2/c^2 - 1 as (c0 - c)(c0 + c)/c^2: no cancellation near the
    // background, and exactly zero where c = c0
    re = (c0 - cc) * (c0 + cc) / (cc * cc) - c0 * c0 * (a * a / (4.0 * PI * PI));
    im = c0 * c0 * a / (PI * cc);
  } else {
    // (kappa rho - kappa0 rho0) / (kappa0 rho0), the difference formed term by
    // term (exactly zero on the background)
    const double nr = (c0 - cc) * (c0 + cc) / (cc * cc * c0 * c0) - (a - a0) * (a + a0) / (4.0 * PI * PI);
    const double ni = a / (PI * cc) - a0 / (PI * c0);
    const double dr = 1.0 / (c0 * c0) - a0 * a0 / (4.0 * PI * PI), di = a0 / (PI * c0);
    const double d2 = dr * dr + di * di;
    re = (nr * dr + ni * di) / d2;
    im = (ni * dr - nr * di) / d2;
  }
  m64[i] = mk(re, im);
  if (m32) m32[i] = mk((float)re, (float)im);
}

void launch_contrast(long n, double c0, double alpha0, const double* c, const double* alpha, c128* m64, c64* m32,
                     hipStream_t st) {
  if (n == 0) return;
  hipLaunchKernelGGL(k_contrast, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, st, n, c0, alpha0, c, alpha, m64,
                     m32);
  FWI_LAUNCH_CHECK();
}

// Inverse of the contrast formula: kappa rho = (m + 1) kappa0 rho0 = A + i B
// with A = 1/c^2 - alpha^2/(4 pi^2) and B = alpha/(pi c), so c^2 is the
// positive root of (B^2/4) x^2 + A x - 1 = 0, written without cancellation as
// x = 2 / (A + sqrt(A^2 + B^2)); then alpha = pi c B. No positive root: NaN.
__global__ void k_sos_from_contrast(long n, c128 k0r, const c128* __restrict__ m, double* __restrict__ c,
                                    double* __restrict__ alpha) {
  const long i = (long)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  const c128 kr = mk(m[i].x + 1.0, m[i].y) * k0r;
  const double A = kr.x, B = kr.y;
  const double den = A + sqrt(A * A + B * B);
  const double cc = den > 0.0 ? sqrt(2.0 / den) : nan("");
  if (c) c[i] = cc;
  if (alpha) alpha[i] = PI * cc * B;
}

void launch_sos_from_contrast(long n, c128 k0r, const c128* m, double* c, double* alpha, hipStream_t st) {
  if (n == 0) return;
  hipLaunchKernelGGL(k_sos_from_contrast, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, st, n, k0r, m, c, alpha);
  FWI_LAUNCH_CHECK();
}

// Cell weight constants (Richmond: equal-area disk / equal-volume ball of radius a).
//  2D: W(r>0) = (i/4)(2 pi a/k) J1(ka) H0(kr),  W(0) = (i pi a/(2k)) H1(ka) - 1/k^2
//  3D: W(r>0) = (4 pi/k^3)(sin ka - ka cos ka) e^{ikr}/(4 pi r),
//      W(0)  = ((1 - i ka) e^{ika} - 1)/k^2
// k is complex for a lossy background.
struct WeightConsts {
  c128 fac;          // factor multiplying G(r) for r > 0 (2D: (2 pi a/k) J1(ka); 3D: (4 pi/k^3)(...))
  c128 self;         // W(0)
};

static WeightConsts weight_consts(int dim, c128 kc, double dx) {
  WeightConsts w{};
  if (dim == 2 && kc.y == 0.0) {
    const double k = kc.x;
    const double a = dx / std::sqrt(PI), ka = k * a;
    double j0, j1, y0, y1;
    bessel01(ka, &j0, &j1, &y0, &y1);
    w.fac = mk((2.0 * PI * a / k) * j1, 0.0);
    // (i pi a/(2k)) (J1 + i Y1) - 1/k^2
    const double s = PI * a / (2.0 * k);
    w.self = mk(-s * y1 - 1.0 / (k * k), s * j1);
  } else if (dim == 2) {
    using cd = std::complex<double>;
    const cd k(kc.x, kc.y), I(0.0, 1.0);
    const double a = dx / std::sqrt(PI);
    const cd ka = k * a;
    cz j0, j1, y0, y1;
    cbessel01(cz{ka.real(), ka.imag()}, &j0, &j1, &y0, &y1);
    const cd J1(j1.re, j1.im), H1(j1.re - y1.im, j1.im + y1.re);
    const cd fac = (2.0 * PI * a / k) * J1;
    const cd self = (I * PI * a / (2.0 * k)) * H1 - 1.0 / (k * k);
    w.fac = mk(fac.real(), fac.imag());
    w.self = mk(self.real(), self.imag());
  } else {
    using cd = std::complex<double>;
    const cd k(kc.x, kc.y), I(0.0, 1.0);
    const double a = dx * std::cbrt(3.0 / (4.0 * PI));
    const cd ka = k * a;
    const cd fac = 4.0 * PI / (k * k * k) * (std::sin(ka) - ka * std::cos(ka));
    const cd self = ((1.0 - I * ka) * std::exp(I * ka) - 1.0) / (k * k);
    w.fac = mk(fac.real(), fac.imag());
    w.self = mk(self.real(), self.imag());
  }
  return w;
}

// e^{i k r} for complex k (Im k >= 0: decaying)
__device__ __forceinline__ c128 expikr(c128 k, double r) {
  double s, c;
  sincos(k.x * r, &s, &c);
  const double d = k.y != 0.0 ? exp(-k.y * r) : 1.0;
  return mk(d * c, d * s);
}

// T[iz][iy][ix] = k^2 W(dx |Delta|) / (Lz Ly Lx) on the circulant grid: offset
// i for i < n, i - L for i > L - n, and zero elsewhere (never reached by the
// linear convolution of an n-point axis).
__global__ void k_green_table(int dim, int nx, int ny, int nz, int Lx, int Ly, int Lz, double dx, c128 k,
                              c128 fac, c128 self, double scale, c128* __restrict__ T) {
  const long i = (long)blockIdx.x * blockDim.x + threadIdx.x;
  const long total = (long)Lx * Ly * Lz;
  if (i >= total) return;
  const int ix = (int)(i % Lx);
  const int iy = (int)((i / Lx) % Ly);
  const int iz = (int)(i / ((long)Lx * Ly));
  auto off = [](int idx, int n, int L, bool& ok) -> int {
    if (idx < n) return idx;
    if (idx > L - n) return idx - L;
    ok = false;
    return 0;
  };
  bool ok = true;
  const int dxi = off(ix, nx, Lx, ok);
  const int dyi = dim == 3 ? off(iy, ny, Ly, ok) : 0;
  const int dzi = off(iz, nz, Lz, ok);
  c128 v = mk(0.0, 0.0);
  if (ok) {
    const double r = dx * sqrt((double)dxi * dxi + (double)dyi * dyi + (double)dzi * dzi);
    if (r == 0.0) {
      v = self;
    } else if (dim == 2 && k.y == 0.0) {
      double j0, j1, y0, y1;
      bessel01(k.x * r, &j0, &j1, &y0, &y1);
      // (i/4) H0 = (i/4)(J0 + i Y0) = (-Y0/4, J0/4)
      v = mk(-0.25 * fac.x * y0, 0.25 * fac.x * j0);
    } else if (dim == 2) {
      const cz h = chankel0(cz{k.x * r, k.y * r});
      v = fac * mk(-0.25 * h.im, 0.25 * h.re);  // (i/4) H0 times the weight factor
    } else {
      v = (1.0 / (4.0 * PI * r)) * (fac * expikr(k, r));
    }
    v = (scale * (k * k)) * v;
  }
  T[i] = v;
}

void launch_green_table(const Geo& g, c128 k, c128* table, hipStream_t st) {
  const WeightConsts w = weight_consts(g.dim, k, g.dx);
  const long total = g.npad();
  hipLaunchKernelGGL(k_green_table, dim3((unsigned)((total + 255) / 256)), dim3(256), 0, st, g.dim, g.nx, g.ny, g.nz,
                     g.Lx, g.Ly, g.Lz, g.dx, k, w.fac, w.self, 1.0 / (double)total, table);
  FWI_LAUNCH_CHECK();
}

// P0[e][n] = G(k |x_n - x_e|): 2D (i/4) H0^(1), 3D e^{ikr}/(4 pi r); with an
// aperture, the average of G over the element's rectangle on the top face
// (product Gauss-Legendre rule: sub-point x_e + (hw xi_a, hh xi_b, 0) with
// weight w_a w_b / 4, one point in a direction of zero extent).
__global__ void k_incident(int dim, int nx, int ny, int nz, double dx, c128 k, int ne,
                           const double* __restrict__ exyz, Aperture ap, c128* __restrict__ P0) {
  const long n = (long)nx * ny * nz;
  const long i = (long)blockIdx.x * blockDim.x + threadIdx.x;
  const int e = blockIdx.y;
  if (i >= n) return;
  const int ix = (int)(i % nx);
  const int iy = (int)((i / nx) % ny);
  const int iz = (int)(i / ((long)nx * ny));
  const int qa = ap.hw > 0.0 ? ap.rule.q : 1, qb = ap.hh > 0.0 ? ap.rule.q : 1;
  c128 v = mk(0.0, 0.0);
  for (int a = 0; a < qa; ++a) {
    const double sx = ap.hw > 0.0 ? ap.hw * ap.rule.x[a] : 0.0;
    const double wa = ap.hw > 0.0 ? 0.5 * ap.rule.w[a] : 1.0;
    for (int b = 0; b < qb; ++b) {
      const double sy = ap.hh > 0.0 ? ap.hh * ap.rule.x[b] : 0.0;
      const double wb = ap.hh > 0.0 ? 0.5 * ap.rule.w[b] : 1.0;
      const double px = (ix + 0.5) * dx - (exyz[3 * e + 0] + sx);
      const double py = (dim == 3 ? (iy + 0.5) * dx : 0.0) - (exyz[3 * e + 1] + sy);
      const double pz = (iz + 0.5) * dx - exyz[3 * e + 2];
      const double r = sqrt(px * px + py * py + pz * pz);
      c128 gv;
      if (dim == 2 && k.y == 0.0) {
        double j0, j1, y0, y1;
        bessel01(k.x * r, &j0, &j1, &y0, &y1);
        gv = mk(-0.25 * y0, 0.25 * j0);
      } else if (dim == 2) {
        const cz h = chankel0(cz{k.x * r, k.y * r});
        gv = mk(-0.25 * h.im, 0.25 * h.re);
      } else {
        gv = (1.0 / (4.0 * PI * r)) * expikr(k, r);
      }
      v = v + (wa * wb) * gv;
    }
  }
  P0[(long)e * n + i] = v;
}

void launch_incident(const Geo& g, c128 k, int ne, const double* exyz, const Aperture& ap, c128* P0,
                     hipStream_t st) {
  const long n = g.n();
  if (n == 0 || ne == 0) return;
  hipLaunchKernelGGL(k_incident, dim3((unsigned)((n + 255) / 256), ne), dim3(256), 0, st, g.dim, g.nx, g.ny, g.nz, g.dx,
                     k, ne, exyz, ap, P0);
  FWI_LAUNCH_CHECK();
}

// Gauss-Legendre nodes (roots of P_q) by Newton's method from the classical
// starting values cos(pi (i + 3/4) / (q + 1/2)), P_q and P_q' by the
// three-term recurrence; weights 2 / ((1 - x^2) P_q'(x)^2).
GaussRule gauss_legendre(int q) {
  GaussRule r{};
  r.q = q;
  for (int i = 0; i < q; ++i) {
    double x = std::cos(PI * (i + 0.75) / (q + 0.5)), dp = 1.0;
    for (int it = 0; it < 100; ++it) {
      double p0 = 1.0, p1 = x;
      for (int j = 2; j <= q; ++j) {
        const double p2 = ((2.0 * j - 1.0) * x * p1 - (j - 1.0) * p0) / j;
        p0 = p1;
        p1 = p2;
      }
      dp = q * (x * p1 - p0) / (x * x - 1.0);
      const double step = p1 / dp;
      x -= step;
      if (std::fabs(step) < 1e-16) break;
    }
    double p0 = 1.0, p1 = x;
    for (int j = 2; j <= q; ++j) {
      const double p2 = ((2.0 * j - 1.0) * x * p1 - (j - 1.0) * p0) / j;
      p0 = p1;
      p1 = p2;
    }
    dp = q * (x * p1 - p0) / (x * x - 1.0);
    r.x[i] = x;
    r.w[i] = 2.0 / ((1.0 - x * x) * dp * dp);
  }
  return r;
}

__global__ void k_cast_64_32(long count, const c128* __restrict__ in, c64* __restrict__ out) {
  const long i = (long)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < count) out[i] = cvt<float>(in[i]);
}
void launch_cast_64_32(long count, const c128* in, c64* out, hipStream_t st) {
  if (count == 0) return;
  hipLaunchKernelGGL(k_cast_64_32, dim3((unsigned)((count + 255) / 256)), dim3(256), 0, st, count, in, out);
  FWI_LAUNCH_CHECK();
}

// The complex64 kernel spectrum of a geometry with fused lateral-elevation
// passes: cast, with the (ky, kx) frequencies of every z-plane stored
// class-major (kx = 4k + c at column c Lx/4 + k, ky = 2m + d at row
// d Ly/2 + m), the order of the padded spectra those passes write.
__global__ void k_cast_xy_64_32(long count, int Lx, int Ly, const c128* __restrict__ in, c64* __restrict__ out) {
  const long i = (long)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= count) return;
  const long plane = (long)Lx * Ly;
  const long z = i / plane;
  const int r = (int)(i - z * plane), ky = r / Lx, kx = r - ky * Lx;
  const int row = (ky & 1) * (Ly / 2) + (ky >> 1), col = (kx & 3) * (Lx / 4) + (kx >> 2);
  out[z * plane + (long)row * Lx + col] = cvt<float>(in[i]);
}
void launch_cast_xy_64_32(const Geo& g, const c128* in, c64* out, hipStream_t st) {
  if (g.Lx % 4 || g.Ly % 2) throw Error(-6, "class-major spectrum needs Lx % 4 == 0 and Ly % 2 == 0");
  const long count = g.npad();
  hipLaunchKernelGGL(k_cast_xy_64_32, dim3((unsigned)((count + 255) / 256)), dim3(256), 0, st, count, g.Lx, g.Ly, in,
                     out);
  FWI_LAUNCH_CHECK();
}

__global__ void k_scale_c128(long count, double s, c128* x) {
  const long i = (long)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < count) x[i] = s * x[i];
}
void launch_scale_c128(long count, double s, c128* x, hipStream_t st) {
  if (count == 0) return;
  hipLaunchKernelGGL(k_scale_c128, dim3((unsigned)((count + 255) / 256)), dim3(256), 0, st, count, s, x);
  FWI_LAUNCH_CHECK();
}

}  // namespace fwi

// Host evaluation of the same Bessel routine the kernels use (for CPU checks).
extern "C" void fwi_host_bessel01(double x, double* out4) {
  fwi::bessel01(x, &out4[0], &out4[1], &out4[2], &out4[3]);
}

// Host evaluation of the complex-argument routine (for CPU checks):
// out = J0, J1, Y0, Y1 as (re, im) pairs.
extern "C" void fwi_host_cbessel01(double re, double im, double* out8) {
  fwi::cz j0, j1, y0, y1;
  fwi::cbessel01(fwi::cz{re, im}, &j0, &j1, &y0, &y1);
  const fwi::cz v[4] = {j0, j1, y0, y1};
  for (int i = 0; i < 4; ++i) {
    out8[2 * i] = v[i].re;
    out8[2 * i + 1] = v[i].im;
  }
}

extern "C" void fwi_host_chankel0(double re, double im, double* out2) {
  const fwi::cz h = fwi::chankel0(fwi::cz{re, im});
  out2[0] = h.re;
  out2[1] = h.im;
}

// The aperture rule the kernels receive (for CPU checks).
extern "C" int fwi_host_gauss_legendre(int q, double* x, double* w) {
  if (q < 1 || q > fwi::kMaxGaussPoints || !x || !w) return -1;
  const fwi::GaussRule r = fwi::gauss_legendre(q);
  for (int i = 0; i < q; ++i) {
    x[i] = r.x[i];
    w[i] = r.w[i];
  }
  return 0;
}

namespace fwi {

// Input checks: out[0] = #(c <= 0 or non-finite), out[1] = #(alpha < 0 or
// non-finite) (k_check_sos), out[0] = #non-finite complex entries
// (k_check_complex). Counts are summed per workgroup and added to out[] with
// integer atomics (exact in any order); k_check_clear zeroes out[] in the same
// stream first. Grid-stride loops over up to 2048 workgroups.
__global__ void k_check_clear(int* __restrict__ out) {
  if (threadIdx.x < 2) out[threadIdx.x] = 0;
}

__global__ void __launch_bounds__(256) k_check_sos(long n, const double* __restrict__ c,
                                                   const double* __restrict__ alpha, int* __restrict__ out) {
  __shared__ double red[4];
  double bc = 0.0, ba = 0.0;
  const long stride = (long)gridDim.x * 256;
  for (long i = (long)blockIdx.x * 256 + threadIdx.x; i < n; i += stride) {
    const double v = c[i];
    if (!(v > 0.0) || !isfinite(v)) bc += 1.0;
    if (alpha) {
      const double a = alpha[i];
      if (!(a >= 0.0) || !isfinite(a)) ba += 1.0;
    }
  }
  const double sc = block_sum<256>(bc, red);
  const double sa = block_sum<256>(ba, red);
  if (threadIdx.x == 0) {
    if (sc > 0.0) atomicAdd(out, (int)sc);
    if (sa > 0.0) atomicAdd(out + 1, (int)sa);
  }
}

__global__ void __launch_bounds__(256) k_check_complex(long n, const c128* __restrict__ x, int* __restrict__ out) {
  __shared__ double red[4];
  double b = 0.0;
  const long stride = (long)gridDim.x * 256;
  for (long i = (long)blockIdx.x * 256 + threadIdx.x; i < n; i += stride) {
    const c128 v = x[i];
    if (!isfinite(v.x) || !isfinite(v.y)) b += 1.0;
  }
  const double s = block_sum<256>(b, red);
  if (threadIdx.x == 0 && s > 0.0) atomicAdd(out, (int)s);
}

static unsigned check_blocks(long n) { return (unsigned)std::max<long>(1, std::min<long>((n + 255) / 256, 2048)); }

void launch_check_sos(long n, const double* c, const double* alpha, int* out, hipStream_t st) {
  hipLaunchKernelGGL(k_check_clear, dim3(1), dim3(64), 0, st, out);
  FWI_LAUNCH_CHECK();
  hipLaunchKernelGGL(k_check_sos, dim3(check_blocks(n)), dim3(256), 0, st, n, c, alpha, out);
  FWI_LAUNCH_CHECK();
}
void launch_check_complex(long n, const c128* x, int* out, hipStream_t st) {
  hipLaunchKernelGGL(k_check_clear, dim3(1), dim3(64), 0, st, out);
  FWI_LAUNCH_CHECK();
  hipLaunchKernelGGL(k_check_complex, dim3(check_blocks(n)), dim3(256), 0, st, n, x, out);
  FWI_LAUNCH_CHECK();
}

}  // namespace fwi
