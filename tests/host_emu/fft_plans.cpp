// CPU check of the line-FFT device code (Stockham stages, radix-16/32 plans,
// zero-padded first stage, cropped last stage, fused convolution middle
// stage): one workgroup runs as NT host threads on random lines, and the
// results are compared with a direct DFT in long double. Prints one line per
// configuration, ending in "ok" or "FAIL".
#include <complex>
#include <cstdio>
#include <random>
#include <thread>
#include <vector>

#include "hip/hip_runtime.h"
thread_local EmuIdx threadIdx, blockIdx;
std::barrier<>* emu_bar;
#include "fft.hpp"

using namespace fwi;
using cld = std::complex<long double>;
static const long double kPi = 3.14159265358979323846264338327950288L;

template <typename T>
std::vector<cplx<T>> twiddle_table(int L) {
  std::vector<cplx<T>> t(L);
  for (int m = 0; m < L; ++m) t[m] = mk((T)cosl(-2 * kPi * m / L), (T)sinl(-2 * kPi * m / L));
  return t;
}
std::vector<cld> direct_dft(const std::vector<cld>& x, int sgn) {
  const int L = (int)x.size();
  std::vector<cld> X(L);
  for (int q = 0; q < L; ++q) {
    cld s = 0;
    for (int r = 0; r < L; ++r) {
      const long double a = sgn * 2 * kPi * (long double)((long)r * q % L) / L;
      s += x[r] * cld(cosl(a), sinl(a));
    }
    X[q] = s;
  }
  return X;
}
template <int NT, class Body>
void run_workgroup(Body body) {
  std::barrier<> bar(NT);
  emu_bar = &bar;
  std::vector<std::thread> th;
  for (int i = 0; i < NT; ++i) th.emplace_back([&, i] { threadIdx.x = (unsigned)i; body(); });
  for (auto& t : th) t.join();
}

// MODE 0: forward over a zero-padded line, 1: inverse cropped to half, 2: convolution,
// 3: convolution with the twiddle powers from a power table (plans with radices up to 16)
template <typename T, int L, int NL, int NT, bool LF, int MODE>
double check(unsigned seed) {
  using C = LineCfg<T, L, NL, NT, LF>;
  std::mt19937 g(seed);
  std::normal_distribution<double> nd;
  const int lin = MODE == 1 ? L : L / 2 - (int)(seed % 3);   // ragged padding
  const int lout = MODE == 0 ? L : L / 2 - (int)(seed % 2);  // ragged crop
  const cplx<T> fill = mk((T)-7, (T)-7);
  std::vector<cplx<T>> in(NL * L), out(NL * L, fill), gh(NL * L), sh(C::LDS_ELEMS);
  std::vector<cplx<T>> tab(MODE == 3 ? pow_table_size<C>() : 1, fill);  // the workgroup's LDS table
  for (auto& v : in) v = mk((T)nd(g), (T)nd(g));
  for (auto& v : gh) v = mk((T)nd(g), (T)nd(g));
  const auto tw = twiddle_table<T>(L);
  auto src = [&](int line, int pb, int ro) -> cplx<T> {
    const int p = pb + ro;
    return p < lin ? in[line * L + p] : mk((T)0, (T)0);
  };
  auto snk = [&](int line, int pb, int ro, cplx<T> v) {
    const int p = pb + ro;
    if (p < lout) out[line * L + p] = v;
  };
  run_workgroup<NT>([&] {
    if constexpr (MODE == 0) {
      fft_line_transform<C, 0, true, false>(tw.data(), sh.data(), src, snk);
    } else if constexpr (MODE == 1) {
      fft_line_transform<C, 1, false, true>(tw.data(), sh.data(), src, snk);
    } else {
      using Map = ConvMidMap<C>;
      cplx<T> gpre[Map::TT][Map::R];
      for (int t = 0; t < Map::TT; ++t)
        for (int r = 0; r < Map::R; ++r) {
          int line, p;
          if (Map::at(t, r, line, p)) gpre[t][r] = gh[line * L + p];
        }
      auto ghf = [&](int t, int r, int, int) { return gpre[t][r]; };
      if constexpr (MODE == 3) fft_line_convolve<C, true>(tw.data(), sh.data(), src, ghf, snk, tab.data());
      else fft_line_convolve<C>(tw.data(), sh.data(), src, ghf, snk);
    }
  });
  double err = 0, nrm = 0;
  for (int l : {0, NL / 2, NL - 1}) {
    std::vector<cld> x(L);
    for (int p = 0; p < L; ++p) x[p] = p < lin ? cld(in[l * L + p].x, in[l * L + p].y) : cld(0);
    std::vector<cld> y;
    if (MODE == 0) {
      y = direct_dft(x, -1);
    } else if (MODE == 1) {
      y = direct_dft(x, +1);
    } else {  // MODE 2, 3
      auto X = direct_dft(x, -1);
      for (int p = 0; p < L; ++p) X[p] *= cld(gh[l * L + p].x, gh[l * L + p].y);
      y = direct_dft(X, +1);
    }
    for (int p = 0; p < lout; ++p) {
      err += std::norm(cld(out[l * L + p].x, out[l * L + p].y) - y[p]);
      nrm += std::norm(y[p]);
    }
  }
  for (int i = 0; i < NL * L; ++i)  // cropped points are never written
    if (i % L >= lout && (out[i].x != fill.x || out[i].y != fill.y)) return 1e30;
  return std::sqrt(err / nrm);
}

template <typename T, int L, int NL, int NT, bool LF>
void all_modes(const char* name) {
  using C = LineCfg<T, L, NL, NT, LF>;
  const double e0 = check<T, L, NL, NT, LF, 0>(L + NL), e1 = check<T, L, NL, NT, LF, 1>(L + 2 * NL),
               e2 = check<T, L, NL, NT, LF, 2>(L + 3 * NL);
  double e3 = 0;
  if constexpr (plan_max_radix<L, C::BIG>() <= 16) e3 = check<T, L, NL, NT, LF, 3>(L + 5 * NL);
  const double tol = sizeof(T) == 4 ? 2e-6 : 1e-14;
  const bool ok = e0 < tol && e1 < tol && e2 < tol && e3 < tol;
  std::printf("%-6s L=%4d NL=%2d NT=%3d LF=%d BIG=%d fwd %.2e inv %.2e conv %.2e table %.2e %s\n", name, L, NL, NT,
              (int)LF, (int)C::BIG, e0, e1, e2, e3, ok ? "ok" : "FAIL");
}

#define FWI_EMU_LENGTHS(T, NL, NT, LF)                                                                      \
  all_modes<T, 32, NL, NT, LF>(#T), all_modes<T, 48, NL, NT, LF>(#T), all_modes<T, 64, NL, NT, LF>(#T),     \
      all_modes<T, 96, NL, NT, LF>(#T), all_modes<T, 128, NL, NT, LF>(#T), all_modes<T, 192, NL, NT, LF>(#T), \
      all_modes<T, 256, NL, NT, LF>(#T), all_modes<T, 384, NL, NT, LF>(#T), all_modes<T, 512, NL, NT, LF>(#T), \
      all_modes<T, 768, NL, NT, LF>(#T), all_modes<T, 1024, NL, NT, LF>(#T)

// FWI_EMU_PART 0 .. 3 selects a quarter of the configurations (the test
// builds and runs the quarters in parallel); undefined: all of them.
#if defined(FWI_EMU_PART)
#define FWI_EMU_IN(k) (FWI_EMU_PART == (k))
#else
#define FWI_EMU_IN(k) 1
#endif
int main() {
#if FWI_EMU_IN(0)
  FWI_EMU_LENGTHS(float, 16, 256, true);   // strided passes, radix-16/32 plans from 256 up
#endif
#if FWI_EMU_IN(1)
  FWI_EMU_LENGTHS(double, 8, 256, true);   // complex128 strided passes
#endif
#if FWI_EMU_IN(2)
  FWI_EMU_LENGTHS(float, 4, 256, false);   // row passes
#endif
#if FWI_EMU_IN(3)
  all_modes<float, 512, 16, 256, false>("float");   // row pass, radix-16/32 plan
  all_modes<float, 128, 32, 256, false>("float");   // radix 16 x 8
  all_modes<float, 768, 8, 256, false>("float");    // radix 8/8/12, butterflies not a divisor of NT
  all_modes<double, 512, 4, 256, true>("double");   // narrow strided tiles
  all_modes<double, 1024, 4, 256, true>("double");
  all_modes<float, 512, 4, 256, true>("float");
  all_modes<float, 96, 4, 256, true>("float");
  all_modes<double, 192, 16, 256, true>("double");  // radix 16 x 12 in complex128
  all_modes<float, 256, 32, 256, true>("float");    // 32-column strided tiles of length 256
  all_modes<float, 256, 32, 512, true>("float");
#endif
  return 0;
}
