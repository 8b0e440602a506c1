// Stand-ins for the library's kernel launchers (kern_*.hip, fft_passes.hpp)
// for the host build of the C ABI. Each one reads and writes exactly the
// ranges that the launcher's contract names (so the sanitizers check every
// extent that the host code plans) and computes only what the host code
// reads back: active counts and iteration counts of the Krylov solver (a RHS
// "converges" after a set number of iterations), misfits, validity flags.
#include <algorithm>
#include <cmath>
#include <cstring>

#include "data.hpp"
#include "emu.hpp"
#include "internal.hpp"
#include "krylov.hpp"

namespace fwi {

using emu::rd;
using emu::wr;

static int need_iters(int b) { return emu::iters_base + b % std::max(1, emu::iters_spread); }
template <typename T>
static size_t es() {
  return sizeof(cplx<T>);
}

// ------------------------------------------------------------- krylov ---
int krylov_nblk(long n) {
  long nb = (n + 16 * 256 - 1) / (16 * 256);
  return (int)(nb < 1 ? 1 : nb);
}

template <typename T>
void krylov_rows_norm(const KrylovState<T>& s, const double* rowpart, int rows, hipStream_t st) {
  const KrylovState<T> k = s;
  emu::submit(st, "rows_norm", [=] {
    rd(rowpart, sizeof(double) * k.B * rows);
    wr(k.nrmp, sizeof(double) * k.B * k.nblk);
  });
}

template <typename T>
void krylov_cycle_init(const KrylovState<T>& s, int first, double, double, hipStream_t st) {
  const KrylovState<T> k = s;
  emu::submit(st, "cycle_init", [=] {
    rd(k.nrmp, sizeof(double) * k.B * k.nblk);
    rd(k.iters, sizeof(int) * k.B);
    if (!first) rd(k.bnorm, sizeof(double) * k.B);
    wr(k.rnorm, sizeof(double) * k.B);
    if (first) wr(k.bnorm, sizeof(double) * k.B);
    wr(k.ncol, sizeof(int) * k.B);
    wr(k.gv, sizeof(c128) * k.B * (k.JM + 1));
    int act = 0;
    for (int b = 0; b < k.B; ++b) {
      k.active[b] = k.iters[b] < need_iters(b);
      if (k.active[b]) {
        ++act;
        k.target[b] = 0.5;
        k.rscale[b] = 1.0;
        k.vscale[b] = mk((T)1, (T)0);
      }
    }
    k.counters[0] = act;
    k.counters[1] = act;
    k.maxrel[0] = act ? 1e-3 : 1e-9;
  });
}

template <typename T>
void krylov_dots(const KrylovState<T>& s, int j, hipStream_t st) {
  const KrylovState<T> k = s;
  emu::submit(st, "dots", [=] {
    for (int i = 0; i <= j + 1; ++i) rd(k.V + (long)i * k.vstride(), es<T>() * k.vstride());
    rd(k.active, sizeof(int) * k.B);
    rd(k.vscale, es<T>() * k.B * (j + 1));
    wr(k.dotp, sizeof(c128) * k.B * k.nblk * (k.JM + 1));
  });
}

template <typename T>
void krylov_hsum(const KrylovState<T>& s, int j, int ndot, hipStream_t st) {
  const KrylovState<T> k = s;
  emu::submit(st, "hsum", [=] {
    rd(k.active, sizeof(int) * k.B);
    rd(k.vscale, es<T>() * k.B * (j + 1));
    rd(k.dotp, sizeof(c128) * k.B * ndot * (k.JM + 1));
    rd(k.H, sizeof(c128) * k.B * (k.JM + 1) * k.JM);
    wr(k.hcoef, sizeof(c128) * k.B * (k.JM + 1));
    k.counters[0] = 0;
  });
}

template <typename T>
void krylov_givens(const KrylovState<T>& s, int j, const double* rowpart, int rows, hipStream_t st) {
  const KrylovState<T> k = s;
  emu::submit(st, "givens", [=] {
    rd(rowpart, sizeof(double) * k.B * rows);
    rd(k.H, sizeof(c128) * k.B * (k.JM + 1) * k.JM);
    rd(k.cs, sizeof(double) * k.B * k.JM);
    rd(k.sn, sizeof(c128) * k.B * k.JM);
    rd(k.gv, sizeof(c128) * k.B * (k.JM + 1));
    rd(k.target, sizeof(double) * k.B);
    int act = 0;
    for (int b = 0; b < k.B; ++b) {
      if (!k.active[b]) continue;
      k.ncol[b] = j + 1;
      k.iters[b] += 1;
      if (k.iters[b] >= need_iters(b)) {
        k.active[b] = 0;
      } else {
        k.vscale[(long)(j + 1) * k.B + b] = mk((T)1, (T)0);
        ++act;
      }
    }
    k.counters[0] = act;
  });
}

template <typename T>
void krylov_backsolve(const KrylovState<T>& s, hipStream_t st) {
  const KrylovState<T> k = s;
  emu::submit(st, "backsolve", [=] {
    rd(k.ncol, sizeof(int) * k.B);
    rd(k.H, sizeof(c128) * k.B * (k.JM + 1) * k.JM);
    rd(k.gv, sizeof(c128) * k.B * (k.JM + 1));
    rd(k.rnorm, sizeof(double) * k.B);
    rd(k.vscale, es<T>() * k.B * (k.JM + 1));
    wr(k.y, sizeof(c128) * k.B * k.JM);
  });
}

template <typename T>
void krylov_xupdate(const KrylovState<T>& s, c128* x, int first, hipStream_t st) {
  const KrylovState<T> k = s;
  emu::submit(st, "xupdate", [=] {
    int kmax = 0;
    for (int b = 0; b < k.B; ++b) kmax = std::max(kmax, k.ncol[b]);
    for (int i = 0; i < kmax; ++i) rd(k.V + (long)i * k.vstride(), es<T>() * k.vstride());
    rd(k.y, sizeof(c128) * k.B * k.JM);
    if (!first) rd(x, sizeof(c128) * k.vstride());
    wr(x, sizeof(c128) * k.vstride());
  });
}

template <typename T>
void krylov_finish_cycle(const KrylovState<T>& s, c128* x, int first, hipStream_t st) {
  krylov_backsolve(s, st);
  krylov_xupdate(s, x, first, st);
}

template <typename T>
void krylov_reset_iters(const KrylovState<T>& s, hipStream_t st) {
  const KrylovState<T> k = s;
  emu::submit(st, "reset_iters", [=] { std::memset(k.iters, 0, sizeof(int) * k.B); });
}

#define FWI_INST(T)                                                                            \
  template void krylov_rows_norm<T>(const KrylovState<T>&, const double*, int, hipStream_t);   \
  template void krylov_cycle_init<T>(const KrylovState<T>&, int, double, double, hipStream_t); \
  template void krylov_dots<T>(const KrylovState<T>&, int, hipStream_t);                        \
  template void krylov_hsum<T>(const KrylovState<T>&, int, int, hipStream_t);                   \
  template void krylov_givens<T>(const KrylovState<T>&, int, const double*, int, hipStream_t);  \
  template void krylov_backsolve<T>(const KrylovState<T>&, hipStream_t);                       \
  template void krylov_xupdate<T>(const KrylovState<T>&, c128*, int, hipStream_t);             \
  template void krylov_finish_cycle<T>(const KrylovState<T>&, c128*, int, hipStream_t);        \
  template void krylov_reset_iters<T>(const KrylovState<T>&, hipStream_t);
FWI_INST(float)
FWI_INST(double)
#undef FWI_INST

void launch_fill_zero_c128(long count, c128* p, hipStream_t st) {
  if (count == 0) return;
  emu::submit(st, "fill_zero", [=] { wr(p, sizeof(c128) * count); });
}
void launch_iter_stats(int B, const int* iters, unsigned long long* out, hipStream_t st) {
  emu::submit(st, "iter_stats", [=] {
    for (int b = 0; b < B; ++b) {
      out[0] = std::max<unsigned long long>(out[0], (unsigned long long)iters[b]);
      out[1] += (unsigned long long)iters[b];
    }
  });
}
void launch_zero_u64(int count, unsigned long long* p, hipStream_t st) {
  emu::submit(st, "zero_u64", [=] { wr(p, sizeof(unsigned long long) * count); });
}
void launch_copy_c128(long count, const c128* in, c128* out, hipStream_t st) {
  if (count == 0) return;
  emu::submit(st, "copy_c128", [=] {
    rd(in, sizeof(c128) * count);
    std::memmove(out, in, sizeof(c128) * count);
  });
}

// ------------------------------------------------------------ operator ---
// Rows per workgroup of the inverse row pass (the launcher fuses the Arnoldi
// inner products only when a workgroup's rows belong to one RHS).
template <typename T>
static int row_inv_rows(int L) {
  const int v = tune_variant(PK_ROW_INV, sizeof(T) == 8, L);
  const int pts = v == 0 ? 2048 : v == 1 ? 4096 : 8192;
  int nl = std::max(pts / L, 1);
  if (nl * (L + L / 8) * (int)sizeof(cplx<T>) > 160 * 1024 - 4096) nl = std::max(nl / 2, 1);
  return nl;
}

template <typename T>
void launch_vie_rows(const Geo& g, const Twiddles& tw, int B, const cplx<T>* x, const int* active, const cplx<T>* m,
                     cplx<T>* U1, hipStream_t st, const XUpdate* xu, const OrthIn* orth, const StartIn* start,
                     cplx<T>* U2) {
  (void)tw.get<T>(g.Lx);
  if ((xu != nullptr) + (orth != nullptr) + (start != nullptr) > 1) throw Error(-6, "one combined input per pass");
  const long n = g.n(), rows = (long)g.nz * g.ny, u1 = g.u1();
  const size_t e = es<T>();
  const XUpdate xv = xu ? *xu : XUpdate{};
  const OrthIn ov = orth ? *orth : OrthIn{};
  const StartIn sv = start ? *start : StartIn{};
  const bool has_xu = xu, has_orth = orth, has_start = start;
  // the fused lateral-elevation pass writes the padded spectrum U2 instead of U1
  const bool xy = sizeof(T) == 4 && g.xy && !(orth && !orth->transform);
  if (xy) {
    (void)tw.get<T>(g.Ly);
    (void)tw.get<T>(g.Lx / 4);
    (void)tw.get<T>(g.Ly / 2);
    if (!U2) throw Error(-6, "the fused lateral-elevation pass needs the y-pass buffer");
  }
  const long u2 = g.u2();
  if (has_xu && (sizeof(T) != 8 || active)) throw Error(-6, "the fused solution update is for complex128 residuals");
  if (has_start && (!m || active)) throw Error(-6, "the start pass needs the contrast and every RHS");
  emu::submit(st, "row_fwd", [=] {
    if (active) rd(active, sizeof(int) * B);
    bool transform = true;
    if (has_xu) {
      rd(xv.ncol, sizeof(int) * B);
      int kmax = 0;
      for (int b = 0; b < B; ++b) kmax = std::max(kmax, xv.ncol[b]);
      const size_t eb = xv.fp32 ? 8 : 16;
      for (int i = 0; i < kmax; ++i) rd((const char*)xv.basis + (size_t)i * xv.vs * eb, eb * B * n);
      rd(xv.coef, sizeof(c128) * B * xv.cstride);
      if (!xv.first) rd(x, e * B * n);
      wr(const_cast<cplx<T>*>(x), e * B * n);
    } else if (has_orth) {
      for (int i = 0; i < ov.nvec; ++i) rd((const char*)ov.basis + (size_t)i * ov.vs * e, e * B * n);
      rd(ov.coef, sizeof(c128) * B * ov.cstride);
      rd(x, e * B * n);
      wr(const_cast<cplx<T>*>(x), e * B * n);
      wr(ov.rowpart, sizeof(double) * B * rows);
      transform = ov.transform;
    } else if (has_start) {
      rd(sv.b, sizeof(c128) * B * n);
      wr(const_cast<cplx<T>*>(x), e * B * n);
      wr(sv.rowpart, sizeof(double) * B * rows);
    } else {
      rd(x, e * B * n);
    }
    if (transform) {
      rd(m, e * n);
      if (xy) wr(U2, e * B * u2);
      else wr(U1, e * B * u1);
    }
  });
}

template <typename T>
void launch_vie_tail(const Geo& g, const Twiddles& tw, int B, const cplx<T>* x, const cplx<T>* scale,
                     const int* active, const cplx<T>* ghat, const int* rhs_freq, cplx<T>* U1, cplx<T>* U2,
                     cplx<T>* y, const cplx<T>* rhs, int epi, hipStream_t st, c64* y32, double* rowpart,
                     VieDots* dots) {
  (void)tw.get<T>(g.Lx);
  (void)tw.get<T>(g.Lz);
  if (g.dim == 3) (void)tw.get<T>(g.Ly);
  const long n = g.n(), rows = (long)g.nz * g.ny, u1 = g.u1(), u2 = g.u2(), np = g.npad();
  const size_t e = es<T>();
  VieDots dv{};
  const bool xy = sizeof(T) == 4 && g.xy;
  if (xy) {
    (void)tw.get<T>(g.Lx / 4);
    (void)tw.get<T>(g.Ly / 2);
    if (epi != EPI_VIE && epi != EPI_COPY) throw Error(-6, "the fused lateral-elevation pass has no residual epilogue");
  }
  if (dots) {
    dots->nparts = 0;
    const int nl = row_inv_rows<T>(g.Lx);
    if (xy) {
      if (epi == EPI_VIE && g.nz <= kMaxDotParts && dots->nvec <= 33) {
        dots->nparts = g.nz;
        dv = *dots;
      }
    } else if (epi == EPI_VIE && rows % nl == 0 && rows / nl <= kMaxDotParts && dots->nvec <= 33) {
      dots->nparts = (int)(rows / nl);
      dv = *dots;
    }
  }
  const bool fused = dv.nparts > 0;
  emu::submit(st, "vie_tail", [=] {
    if (active) rd(active, sizeof(int) * B);
    rd(rhs_freq, sizeof(int) * B);
    for (int b = 0; b < B; ++b) rd(ghat + (long)rhs_freq[b] * np, e * np);
    if (xy) {
      rd(U2, e * B * u2);
      wr(U2, e * B * u2);
      rd(U2, e * B * u2);
    } else {
      rd(U1, e * B * u1);
      if (g.dim == 3) {
        wr(U2, e * B * u2);
        rd(U2, e * B * u2);
      }
      wr(U1, e * B * u1);
    }
    if (scale) rd(scale, e * B);
    rd(x, e * B * n);
    if (epi == EPI_VIE) {
      wr(y, e * B * n);
      if (fused) {
        for (int i = 0; i < dv.nvec; ++i) rd((const char*)dv.basis + (size_t)i * dv.vs * e, e * B * n);
        rd(dv.vscale, e * B * dv.nvec);
        wr(dv.dotp, sizeof(c128) * B * dv.nparts * dv.dstride);
      }
    } else if (epi == EPI_RESID) {
      rd(rhs, e * B * n);
      wr(y, e * B * n);
      wr(rowpart, sizeof(double) * B * rows);
    } else if (epi == EPI_RESID32) {
      rd(rhs, e * B * n);
      wr(y32, sizeof(c64) * B * n);
      wr(rowpart, sizeof(double) * B * rows);
    }
  });
}

template <typename T>
void launch_vie(const Geo& g, const Twiddles& tw, int B, const cplx<T>* x, const cplx<T>* scale, const int* active,
                const cplx<T>* m, const cplx<T>* ghat, const int* rhs_freq, cplx<T>* U1, cplx<T>* U2, cplx<T>* y,
                const cplx<T>* rhs, int epi, hipStream_t st, c64* y32, double* rowpart, VieDots* dots,
                const XUpdate* xu) {
  launch_vie_rows<T>(g, tw, B, x, active, m, U1, st, xu, nullptr, nullptr, U2);
  launch_vie_tail<T>(g, tw, B, x, scale, active, ghat, rhs_freq, U1, U2, y, rhs, epi, st, y32, rowpart, dots);
}

void launch_fft_full(const Geo& g, const Twiddles& tw, const c128* in, c128* work, c128* out, hipStream_t st) {
  (void)tw.get<double>(g.Lx);
  const long np = g.npad();
  emu::submit(st, "fft_full", [=] {
    rd(in, 16 * np);
    wr(work, 16 * np);
    wr(out, 16 * np);
  });
}

template <typename T>
void launch_fft_padded(const Geo& g, const Twiddles& tw, const cplx<T>* in, cplx<T>* U1, cplx<T>* out,
                       hipStream_t st) {
  (void)tw.get<T>(g.Lx);
  const long n = g.n(), np = g.npad(), u1 = g.u1();
  emu::submit(st, "fft_padded", [=] {
    rd(in, es<T>() * n);
    wr(U1, es<T>() * u1);
    wr(out, es<T>() * np);
  });
}

#define FWI_INST(T)                                                                                                  \
  template void launch_vie<T>(const Geo&, const Twiddles&, int, const cplx<T>*, const cplx<T>*, const int*,          \
                              const cplx<T>*, const cplx<T>*, const int*, cplx<T>*, cplx<T>*, cplx<T>*,              \
                              const cplx<T>*, int, hipStream_t, c64*, double*, VieDots*, const XUpdate*);            \
  template void launch_vie_rows<T>(const Geo&, const Twiddles&, int, const cplx<T>*, const int*, const cplx<T>*,     \
                                   cplx<T>*, hipStream_t, const XUpdate*, const OrthIn*, const StartIn*, cplx<T>*);  \
  template void launch_vie_tail<T>(const Geo&, const Twiddles&, int, const cplx<T>*, const cplx<T>*, const int*,     \
                                   const cplx<T>*, const int*, cplx<T>*, cplx<T>*, cplx<T>*, const cplx<T>*, int,    \
                                   hipStream_t, c64*, double*, VieDots*);                                            \
  template void launch_fft_padded<T>(const Geo&, const Twiddles&, const cplx<T>*, cplx<T>*, cplx<T>*, hipStream_t);
FWI_INST(float)
FWI_INST(double)
#undef FWI_INST

// -------------------------------------------------------------- set-up ---
void launch_contrast(long n, double, double, const double* c, const double* alpha, c128* m64, c64* m32,
                     hipStream_t st) {
  emu::submit(st, "contrast", [=] {
    rd(c, 8 * n);
    if (alpha) rd(alpha, 8 * n);
    wr(m64, 16 * n);
    wr(m32, 8 * n);
  });
}
void launch_sos_from_contrast(long n, c128, const c128* m, double* c, double* alpha, hipStream_t st) {
  emu::submit(st, "sos", [=] {
    rd(m, 16 * n);
    if (c) wr(c, 8 * n);
    if (alpha) wr(alpha, 8 * n);
  });
}
void launch_green_table(const Geo& g, c128, c128* table, hipStream_t st) {
  const long np = g.npad();
  emu::submit(st, "green_table", [=] { wr(table, 16 * np); });
}
GaussRule gauss_legendre(int q) {
  GaussRule r{};
  r.q = q;
  for (int i = 0; i < q; ++i) {
    r.x[i] = -1.0 + (2.0 * i + 1.0) / q;
    r.w[i] = 2.0 / q;
  }
  return r;
}
void launch_incident(const Geo& g, c128, int ne, const double* exyz, const Aperture&, c128* P0, hipStream_t st) {
  const long n = g.n();
  emu::submit(st, "incident", [=] {
    rd(exyz, 24 * ne);
    wr(P0, 16 * n * ne);
  });
}
void launch_cast_64_32(long count, const c128* in, c64* out, hipStream_t st) {
  if (count == 0) return;
  emu::submit(st, "cast", [=] {
    rd(in, 16 * count);
    wr(out, 8 * count);
  });
}
void launch_cast_xy_64_32(const Geo& g, const c128* in, c64* out, hipStream_t st) {
  if (g.Lx % 4 || g.Ly % 2) throw Error(-6, "class-major spectrum needs Lx % 4 == 0 and Ly % 2 == 0");
  const long count = g.npad();
  emu::submit(st, "cast_xy", [=] {
    rd(in, 16 * count);
    wr(out, 8 * count);
  });
}
void launch_scale_c128(long count, double, c128* x, hipStream_t st) {
  emu::submit(st, "scale", [=] {
    rd(x, 16 * count);
    wr(x, 16 * count);
  });
}
void launch_check_sos(long n, const double* c, const double* alpha, int* out, hipStream_t st) {
  emu::submit(st, "check_sos", [=] {
    rd(c, 8 * n);
    if (alpha) rd(alpha, 8 * n);
    out[0] = out[1] = 0;
  });
}
void launch_check_complex(long n, const c128* x, int* out, hipStream_t st) {
  emu::submit(st, "check_complex", [=] {
    rd(x, 16 * n);
    out[0] = 0;
  });
}

// ---------------------------------------------------------------- data ---
void launch_gemm_nt(int nf, const c128* A, long a_ls, int ni, const c128* w, const c128* Bm, long b_ls, int nj, long n,
                    const c128* coef, c128* part, int nks, c128* C, hipStream_t st) {
  emu::submit(st, "gemm_nt", [=] {
    rd(A, 16 * ((nf - 1) * a_ls + (long)ni * n));
    rd(w, 16 * n);
    rd(Bm, 16 * ((nf - 1) * b_ls + (long)nj * n));
    rd(coef, 16 * nf);
    wr(part, 16 * (long)nks * nf * ni * nj);
    wr(C, 16 * (long)nf * ni * nj);
  });
}
void launch_gemm_cn(int nf, const c128* M, int ni, int nj, const c128* P, long p_ls, long n, c128* S, long s_ls,
                    hipStream_t st) {
  emu::submit(st, "gemm_cn", [=] {
    rd(M, 16 * (long)nf * ni * nj);
    rd(P, 16 * ((nf - 1) * p_ls + (long)nj * n));
    wr(S, 16 * ((nf - 1) * s_ls + (long)ni * n));
  });
}
int gemm_cn_grad_segments(int nf, int ni) { return nf * ((ni + 63) / 64); }
void launch_gemm_cn_grad(int nf, const c128* M, int ni, int nj, const c128* P, long p_ls, long n, const c128* T,
                         long t_ls, const c128* k2, c128* part, hipStream_t st) {
  emu::submit(st, "gemm_cn_grad", [=] {
    rd(M, 16 * (long)nf * ni * nj);
    rd(P, 16 * ((nf - 1) * p_ls + (long)nj * n));
    rd(T, 16 * ((nf - 1) * t_ls + (long)ni * n));
    rd(k2, 16 * nf);
    wr(part, 16 * (long)gemm_cn_grad_segments(nf, ni) * n);
  });
}
void launch_grad_sum(long n, const c128* part, int nseg, int first, c128* acc, hipStream_t st) {
  emu::submit(st, "grad_sum", [=] {
    rd(part, 16 * nseg * n);
    if (!first) rd(acc, 16 * n);
    wr(acc, 16 * n);
  });
}
void launch_residual(long count, const c128* data, const c128* dobs, c128* r, double* misfit, hipStream_t st) {
  emu::submit(st, "residual", [=] {
    double s = 0.0;
    for (long i = 0; i < count; ++i) {
      const c128 v = dobs ? data[i] - dobs[i] : data[i];
      r[i] = v;
      s += v.x * v.x + v.y * v.y;
    }
    misfit[0] = 0.5 * s;
  });
}
void launch_gradient_accum(long n, int nf, int ni, const c128* p, const c128* lam, const c128* k2, c128* part,
                           int nseg, int first, c128* acc, hipStream_t st) {
  emu::submit(st, "gradient_accum", [=] {
    rd(p, 16 * (long)nf * ni * n);
    rd(lam, 16 * (long)nf * ni * n);
    rd(k2, 16 * nf);
    wr(part, 16 * (long)nseg * n);
    if (!first) rd(acc, 16 * n);
    wr(acc, 16 * n);
  });
}
void launch_grad_chain(long n, const c128* acc, double, c128, const double* c, const double* alpha, c128* g,
                       double* gc, double* ga, hipStream_t st) {
  emu::submit(st, "grad_chain", [=] {
    rd(acc, 16 * n);
    if (c) rd(c, 8 * n);
    if (alpha) rd(alpha, 8 * n);
    if (g) wr(g, 16 * n);
    if (gc) wr(gc, 8 * n);
    if (ga) wr(ga, 8 * n);
  });
}
void launch_tv_grad(const Geo& g, const c128* m, c128* out, hipStream_t st) {
  const long n = g.n();
  const int d = g.dim;
  emu::submit(st, "tv_grad", [=] {
    rd(m, 16 * n);
    wr(out, 16 * d * n);
  });
}
void launch_tv_gradT(const Geo& g, const c128* a, double, double, c128* out, hipStream_t st) {
  const long n = g.n();
  const int d = g.dim;
  emu::submit(st, "tv_gradT", [=] {
    rd(a, 16 * d * n);
    wr(out, 16 * n);
  });
}
int launch_tv_shrink_dual(const Geo& g, const c128* gm, double, double, c128* gout, c128* u, double* tvp,
                          hipStream_t st) {
  const long n = g.n();
  const int d = g.dim;
  const int nb = (int)((n + 255) / 256);
  emu::submit(st, "shrink_dual", [=] {
    rd(gm, 16 * d * n);
    rd(u, 16 * d * n);
    wr(gout, 16 * d * n);
    wr(u, 16 * d * n);
    wr(tvp, 8 * nb);
  });
  return nb;
}
void launch_lincomb(long n, double, const c128* x, double, const c128* y, double, const c128* z, c128* out,
                    hipStream_t st) {
  emu::submit(st, "lincomb", [=] {
    rd(x, 16 * n);
    rd(y, 16 * n);
    if (z) rd(z, 16 * n);
    wr(out, 16 * n);
  });
}
int dot_blocks(long n) {
  long b = (n + 255) / 256;
  return (int)(b > 512 ? 512 : (b < 1 ? 1 : b));
}
void launch_dot_re(long n, const c128* x, const c128* y, double* part, double* out, hipStream_t st) {
  const int nb = dot_blocks(n);
  emu::submit(st, "dot_re", [=] {
    rd(x, 16 * n);
    rd(y, 16 * n);
    wr(part, 8 * nb);
    out[0] = 1.0;
  });
}
void launch_sum(int nb, const double* part, double* out, hipStream_t st) {
  emu::submit(st, "sum", [=] {
    rd(part, 8 * nb);
    out[0] = 1.0;
  });
}
void launch_cg_step1(long n, const double* sc, c128* x, c128* r, const c128* p, const c128* Ap, hipStream_t st) {
  emu::submit(st, "cg1", [=] {
    rd(sc, 8 * 2);
    rd(p, 16 * n);
    rd(Ap, 16 * n);
    wr(x, 16 * n);
    wr(r, 16 * n);
  });
}
void launch_cg_step2(long n, const double* sc, const c128* r, c128* p, hipStream_t st) {
  emu::submit(st, "cg2", [=] {
    rd(sc, 8 * 3);
    rd(r, 16 * n);
    wr(p, 16 * n);
  });
}
void launch_copy_scalar(const double* in, double* out, hipStream_t st) {
  emu::submit(st, "copy_scalar", [=] { out[0] = in[0]; });
}
void launch_prolong(const Geo& g, int r, const c128* mc, c128* mf, hipStream_t st) {
  const long n = g.n();
  const long nc = (long)((g.nx + r - 1) / r) * (g.dim == 3 ? (g.ny + r - 1) / r : 1) * ((g.nz + r - 1) / r);
  emu::submit(st, "prolong", [=] {
    rd(mc, 16 * nc);
    wr(mf, 16 * n);
  });
}
void launch_restrict(const Geo& g, int r, const c128* gf, c128* gcv, hipStream_t st) {
  const long n = g.n();
  const long nc = (long)((g.nx + r - 1) / r) * (g.dim == 3 ? (g.ny + r - 1) / r : 1) * ((g.nz + r - 1) / r);
  emu::submit(st, "restrict", [=] {
    rd(gf, 16 * n);
    wr(gcv, 16 * nc);
  });
}
void launch_conj_c128(long count, const c128* in, c128* out, hipStream_t st) {
  if (count == 0) return;
  emu::submit(st, "conj", [=] {
    rd(in, 16 * count);
    wr(out, 16 * count);
  });
}
void launch_fill_rfreq(int B, int per, int l0, int* rf, hipStream_t st) {
  if (B == 0) return;
  emu::submit(st, "fill_rfreq", [=] {
    for (int b = 0; b < B; ++b) rf[b] = l0 + b / per;
  });
}

}  // namespace fwi
