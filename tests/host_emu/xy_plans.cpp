// CPU check of the fused lateral-elevation passes (xy_passes.hpp): one
// workgroup runs as host threads on one z-plane of random data, and
//  - the forward body's class-major padded spectrum is compared with a
//    direct 2D DFT of the zero-padded operand (m times the plane),
//  - the inverse body's plane is compared with the unnormalised inverse 2D
//    DFT of a random natural-order spectrum, cropped,
//  - the Gram-Schmidt and start operands and their per-row norms, and the
//    operator epilogue y = s (x - conv), are compared with direct sums.
// Arrays are sized exactly, so an address sanitizer build also checks every
// access. Prints one line per check, ending in "ok" or "FAIL".
#include <complex>
#include <cstdio>
#include <random>
#include <thread>
#include <vector>

#include "hip/hip_runtime.h"
thread_local EmuIdx threadIdx, blockIdx;
std::barrier<>* emu_bar;
#include "fft.hpp"

namespace fwi {
enum RowInKind { RI_PLAIN = 0, RI_UPD32 = 1, RI_UPD64 = 2, RI_ORTH = 3, RI_ORTH_ONLY = 4, RI_START = 5 };
enum Epilogue { EPI_VIE = 0, EPI_RESID = 1, EPI_COPY = 2, EPI_RESID32 = 3, EPI_VIE_DOT = 4 };
constexpr int kMaxDotVec = 33;
}  // namespace fwi
#define FWI_XY_BODIES_ONLY
#include "xy_passes.hpp"

using namespace fwi;
using cld = std::complex<long double>;
static const long double kPi = 3.14159265358979323846264338327950288L;

template <typename T>
std::vector<cplx<T>> twiddle_table(int L) {
  std::vector<cplx<T>> t(L);
  for (int m = 0; m < L; ++m) t[m] = mk((T)cosl(-2 * kPi * m / L), (T)sinl(-2 * kPi * m / L));
  return t;
}
template <int NT, class Body>
void run_workgroup(Body body) {
  std::barrier<> bar(NT);
  emu_bar = &bar;
  std::vector<std::thread> th;
  for (int i = 0; i < NT; ++i) th.emplace_back([&, i] { threadIdx.x = (unsigned)i; body(); });
  for (auto& t : th) t.join();
}
// separable 2D DFT of A[Ly][Lx] (sgn -1 forward, +1 inverse, unnormalised)
std::vector<cld> dft2(const std::vector<cld>& A, int Ly, int Lx, int sgn) {
  std::vector<cld> B(A.size()), C(A.size());
  for (int y = 0; y < Ly; ++y)
    for (int k = 0; k < Lx; ++k) {
      cld s = 0;
      for (int x = 0; x < Lx; ++x) {
        const long double a = sgn * 2 * kPi * (long double)((long)x * k % Lx) / Lx;
        s += A[(long)y * Lx + x] * cld(cosl(a), sinl(a));
      }
      B[(long)y * Lx + k] = s;
    }
  for (int k = 0; k < Lx; ++k)
    for (int m = 0; m < Ly; ++m) {
      cld s = 0;
      for (int y = 0; y < Ly; ++y) {
        const long double a = sgn * 2 * kPi * (long double)((long)y * m % Ly) / Ly;
        s += B[(long)y * Lx + k] * cld(cosl(a), sinl(a));
      }
      C[(long)m * Lx + k] = s;
    }
  return C;
}
template <typename T>
cld L(cplx<T> v) {
  return cld(v.x, v.y);
}
double rel(long double e, long double n) { return (double)std::sqrt(e / (n > 0 ? n : 1)); }
int g_fail = 0;
void report(const char* what, int MX, int HY, double err, double tol) {
  const bool ok = err < tol;
  if (!ok) g_fail = 1;
  std::printf("%-10s MX=%3d HY=%3d err %.2e %s\n", what, MX, HY, err, ok ? "ok" : "FAIL");
}

template <int MX, int HY>
void run(unsigned seed) {
  using T = float;
  using Q = XyCfg<T, MX, HY>;
  constexpr int NT = Q::NTX;
  const int Lx = 4 * MX, Ly = 2 * HY;
  const int nx = 2 * MX - 3, ny = HY - 5, nz = 3, B = 2;  // ragged plane, several planes and RHS
  const long n = (long)nx * ny * nz, npl = (long)Ly * Lx;
  const int z = 1, b = 1;  // the plane the workgroup does
  std::mt19937 g(seed);
  std::normal_distribution<double> nd;
  auto rnd = [&]() { return mk((T)nd(g), (T)nd(g)); };
  const auto twx = twiddle_table<T>(Lx), twy = twiddle_table<T>(Ly), twm = twiddle_table<T>(MX),
             twh = twiddle_table<T>(HY);
  const int nvec = 3, cstride = 5;
  std::vector<cplx<T>> x(B * n), m(n), basis(nvec * B * n), xout(B * n, mk((T)0, (T)0)), U2(B * nz * npl),
      y(B * n, mk((T)0, (T)0)), scale(B);
  std::vector<c128> coef(B * cstride), src(B * n);
  std::vector<double> rowpart((long)B * nz * ny, -1.0);
  for (auto& v : x) v = rnd();
  for (auto& v : m) v = rnd();
  for (auto& v : basis) v = rnd();
  for (auto& v : U2) v = rnd();
  for (auto& v : scale) v = rnd();
  for (auto& v : coef) v = mk(nd(g), nd(g));
  for (auto& v : src) v = mk(nd(g), nd(g));
  XyArgs<T> a{};
  a.nx = nx;
  a.ny = ny;
  a.nz = nz;
  a.Lx = Lx;
  a.Ly = Ly;
  a.B = B;
  a.twx = twx.data();
  a.twy = twy.data();
  a.twm = twm.data();
  a.twh = twh.data();
  a.U2 = U2.data();
  a.x = x.data();
  a.m = m.data();
  a.basis = basis.data();
  a.vs = B * n;
  a.nvec = nvec;
  a.coef = coef.data();
  a.cstride = cstride;
  a.xout = xout.data();
  a.rowpart = rowpart.data();
  a.src = src.data();
  a.scale = scale.data();
  a.y = y.data();
  std::vector<cplx<T>> sh(Q::LDS);
  const long pb = (long)b * n + (long)z * ny * nx, mb = (long)z * ny * nx;
  auto U2at = [&](int ky, int kx) {
    const int row = (ky % 2) * HY + ky / 2, col = (kx % 4) * MX + kx / 4;
    return U2[((long)b * nz + z) * npl + (long)row * Lx + col];
  };
  // forward of the operand formed as K does, against the direct DFT
  auto fwd_check = [&](auto kind, const char* name) {
    constexpr int K = decltype(kind)::value;
    for (auto& v : rowpart) v = -1.0;
    run_workgroup<NT>([&] { xy_fwd_body<T, MX, HY, K>(a, z, b, sh.data()); });
    std::vector<cld> op(npl, 0);
    long double eo = 0, no = 0, er = 0, nr = 0;
    for (int yy = 0; yy < ny; ++yy) {
      long double rs = 0;
      for (int xx = 0; xx < nx; ++xx) {
        const long e = (long)yy * nx + xx;
        cld v;
        if (K == RI_START) {
          v = cld((float)src[pb + e].x, (float)src[pb + e].y);
          rs += std::norm(cld(src[pb + e].x, src[pb + e].y));
        } else {
          v = L(x[pb + e]);
          if (K == RI_ORTH)
            for (int j = 0; j < nvec; ++j)
              v += cld(coef[b * cstride + j].x, coef[b * cstride + j].y) * L(basis[(long)j * B * n + pb + e]);
          rs += std::norm(v);
        }
        if (K != RI_PLAIN) {
          eo += std::norm(L(xout[pb + e]) - v);
          no += std::norm(v);
        }
        op[(long)yy * Lx + xx] = v * L(m[mb + e]);
      }
      if (K != RI_PLAIN) {
        const long double got = rowpart[(long)b * nz * ny + (long)z * ny + yy];
        er += (got - rs) * (got - rs);
        nr += rs * rs;
      }
    }
    const auto X = dft2(op, Ly, Lx, -1);
    long double e = 0, nn = 0;
    for (int ky = 0; ky < Ly; ++ky)
      for (int kx = 0; kx < Lx; ++kx) {
        e += std::norm(L(U2at(ky, kx)) - X[(long)ky * Lx + kx]);
        nn += std::norm(X[(long)ky * Lx + kx]);
      }
    report(name, MX, HY, rel(e, nn), 3e-6);
    if (K != RI_PLAIN) {
      report("  operand", MX, HY, rel(eo, no), 1e-6);
      report("  row norm", MX, HY, rel(er, nr), 1e-6);
    }
  };
  fwd_check(std::integral_constant<int, RI_PLAIN>{}, "fwd");
  fwd_check(std::integral_constant<int, RI_ORTH>{}, "fwd orth");
  fwd_check(std::integral_constant<int, RI_START>{}, "fwd start");
  // inverse of a random class-major spectrum, against the direct inverse DFT
  for (auto& v : U2) v = rnd();
  std::vector<cld> S(npl);
  for (int ky = 0; ky < Ly; ++ky)
    for (int kx = 0; kx < Lx; ++kx) S[(long)ky * Lx + kx] = L(U2at(ky, kx));
  const auto want = dft2(S, Ly, Lx, +1);
  auto inv_check = [&](auto epi, const char* name) {
    constexpr int E = decltype(epi)::value;
    std::vector<double> red(2 * kMaxDotVec * (NT / 64 > 0 ? NT / 64 : 1));
    run_workgroup<NT>([&] { xy_inv_body<T, MX, HY, E>(a, z, b, sh.data(), red.data()); });
    long double e = 0, nn = 0;
    for (int yy = 0; yy < ny; ++yy)
      for (int xx = 0; xx < nx; ++xx) {
        const long ei = (long)yy * nx + xx;
        cld w = want[(long)yy * Lx + xx];
        if (E != EPI_COPY) w = (L(x[pb + ei]) - w) * L(scale[b]);
        e += std::norm(L(y[pb + ei]) - w);
        nn += std::norm(w);
      }
    report(name, MX, HY, rel(e, nn), 3e-6);
  };
  inv_check(std::integral_constant<int, EPI_COPY>{}, "inv");
  inv_check(std::integral_constant<int, EPI_VIE>{}, "inv vie");
  // with the inner products (their wave sums are not emulated: y is checked,
  // and the accesses of the dot loop run under the sanitizer)
  std::vector<cplx<T>> vscale((nvec + 1) * B);
  for (auto& v : vscale) v = rnd();
  std::vector<c128> dotp((long)B * nz * (nvec + 1), mk(0.0, 0.0));
  a.dbasis = basis.data();
  a.dvs = B * n;
  a.dnvec = nvec;
  a.vscale = vscale.data();
  a.dotp = dotp.data();
  a.dstride = nvec + 1;
  inv_check(std::integral_constant<int, EPI_VIE_DOT>{}, "inv dots");
  // the plane's outputs only: y of the other plane and RHS untouched
  long bad = 0;
  for (long i = 0; i < B * n; ++i)
    if ((i < pb || i >= pb + (long)ny * nx) && (y[i].x != 0 || y[i].y != 0)) ++bad;
  report("confined", MX, HY, (double)bad, 0.5);
}

// FWI_XY_PART 0 / 1 selects one of the two shapes (the test builds and runs
// them in parallel); undefined: both.
int main() {
#if !defined(FWI_XY_PART) || FWI_XY_PART == 0
  run<32, 64>(11);
#endif
#if !defined(FWI_XY_PART) || FWI_XY_PART == 1
  run<64, 128>(12);
#endif
  return g_fail;
}
