// Internal host-side interfaces between the C-ABI, the solver driver and the
// kernel launchers. Not part of the public ABI.
#pragma once

#include <hip/hip_ext.h>
#include <hip/hip_runtime.h>
#include <cstddef>
#include <cstdint>
#include <stdexcept>
#include <string>

#include "common.hpp"

namespace fwi {

// Error carrying a public FWI_E_* code.
struct Error : std::runtime_error {
  int code;
  Error(int c, const std::string& m) : std::runtime_error(m), code(c) {}
};

#define FWI_HIP(call)                                                                    \
  do {                                                                                   \
    hipError_t e_ = (call);                                                              \
    if (e_ != hipSuccess)                                                                \
      throw ::fwi::Error(-5, std::string("HIP error: ") + hipGetErrorString(e_) + " at " + \
                                 __FILE__ + ":" + std::to_string(__LINE__));             \
  } while (0)

#define FWI_LAUNCH_CHECK() FWI_HIP(hipGetLastError())

// Kernel classes that can be timed with HIP events (fwi_profile).
enum KernelClass { KC_ROW_FWD = 0, KC_CONV, KC_ROW_INV, KC_Y_FWD, KC_Y_INV, KC_DOTS, KC_ORTH, KC_ORTH_FWD, KC_COUNT };
// Per-thread hooks set by the entry points: launch sites report each launch of
// a class with its algorithmic HBM bytes; active-RHS and frequency-count hints
// let them compute those bytes for masked batches.
// A launch moves per_rhs bytes for each RHS it processes plus fixed bytes; a
// masked launch processes the RHS still active (tl_active when it is enqueued,
// corrected by set_active once the solver has read the true count), an
// unmasked one all B.
struct LaunchProfiler {
  virtual void begin(int cls, hipStream_t st) = 0;
  virtual void end(int cls, hipStream_t st, double per_rhs, double fixed, bool masked, long B) = 0;
  virtual size_t mark() const = 0;                  // index of the next record
  virtual void set_active(size_t from, long act) = 0;  // masked records from `from` on
  virtual ~LaunchProfiler() = default;
};
extern thread_local LaunchProfiler* tl_prof;
// Events of the launch being profiled (null otherwise): the kernel launch
// itself records them (hipExtLaunchKernel), so timing adds no packets to the
// stream; every profiled region launches exactly one kernel.
extern thread_local hipEvent_t tl_ev_start, tl_ev_stop;
extern thread_local bool tl_ev_used;  // the events were handed to a launch
#define FWI_TIMED_LAUNCH(kernel, grid, block, shmem, st, ...)                                          \
  do {                                                                                                 \
    if (::fwi::tl_ev_start) {                                                                          \
      hipExtLaunchKernelGGL(kernel, grid, block, shmem, st, ::fwi::tl_ev_start, ::fwi::tl_ev_stop, 0, \
                            __VA_ARGS__);                                                              \
      ::fwi::tl_ev_used = true;                                                                        \
    } else {                                                                                           \
      hipLaunchKernelGGL(kernel, grid, block, shmem, st, __VA_ARGS__);                                 \
    }                                                                                                  \
  } while (0)
extern thread_local long tl_active;  // RHS that the next launches actually process (0: all)
extern thread_local int tl_nfreq;    // distinct frequencies in the batch (Ghat reads)
inline void prof_begin(int cls, hipStream_t st) {
  if (tl_prof) tl_prof->begin(cls, st);
}
inline void prof_end(int cls, hipStream_t st, double per_rhs, double fixed, bool masked, long B) {
  if (tl_prof) tl_prof->end(cls, st, per_rhs, fixed, masked, B);
}

// Supported FFT lengths (padded axis sizes): 2^a 3^b from 32 to 1024.
constexpr int kNumLengths = 11;
constexpr int kLengths[kNumLengths] = {32, 48, 64, 96, 128, 192, 256, 384, 512, 768, 1024};
int length_index(int L);          // -1 if unsupported

// Tile variants of the FFT passes, chosen per (pass, precision, length).
enum PassKind { PK_ROW_FWD = 0, PK_ROW_INV, PK_CONV, PK_STRIDED, PK_COUNT };
constexpr int kNumVariants = 3;
struct FftTuning {
  signed char v[PK_COUNT][2][kNumLengths];  // -1: built-in default
  FftTuning() {
    for (auto& a : v)
      for (auto& b : a)
        for (auto& c : b) c = -1;
  }
};
extern thread_local const FftTuning* tl_tune;
extern thread_local int tl_force_variant;  // >= 0: every pass uses this variant
extern thread_local int tl_force_wide;     // 1: strided passes use 64-bit addressing
extern thread_local int tl_xy_off;         // 1: no fused lateral-elevation passes (separate x and y passes)
// (Lx / 4, Ly / 2) of the grids built with fused lateral-elevation passes
__host__ __device__ constexpr bool xy_shape(int MX, int HY) { return (MX == 64 && HY == 128) || (MX == 32 && HY == 64); }
int default_variant(int pass, bool dbl, int L);
int tune_variant(int pass, bool dbl, int L);
int padded_length(int n);         // smallest supported L >= 2n, 0 if none

// Twiddle tables tw[m] = exp(-2 pi i m / L) for every supported L.
struct Twiddles {
  const c128* d64[kNumLengths] = {};
  const c64* d32[kNumLengths] = {};
  template <typename T>
  const cplx<T>* get(int L) const;
};

template <>
const c128* Twiddles::get<double>(int L) const;
template <>
const c64* Twiddles::get<float>(int L) const;

// Grid geometry of one problem: cells and padded FFT extents.
struct Geo {
  int dim = 2, nx = 0, ny = 1, nz = 0;
  int Lx = 0, Ly = 1, Lz = 0;
  double dx = 0, c0 = 0;
  double alpha0 = 0;  // background attenuation [Np/m/Hz] (3D only)
  // 3D complex64 operator with fused lateral-elevation passes (xy_passes.hpp):
  // its padded spectra, and the complex64 kernel spectrum, are class-major
  int xy = 0;
  long n() const { return (long)nx * ny * nz; }
  long npad() const { return (long)Lx * Ly * Lz; }
  // per-RHS intermediate sizes (elements): after the x pass / after the y pass
  long u1() const { return (long)nz * ny * Lx; }
  long u2() const { return dim == 3 ? (long)nz * Ly * Lx : 0; }
};
inline int xy_applies(const Geo& g) {
  return g.dim == 3 && !tl_xy_off && g.Lx % 4 == 0 && g.Ly % 2 == 0 && 2 * g.nx <= g.Lx && 2 * g.ny <= g.Ly &&
         xy_shape(g.Lx / 4, g.Ly / 2);
}

enum Epilogue { EPI_VIE = 0, EPI_RESID = 1, EPI_COPY = 2, EPI_RESID32 = 3, EPI_VIE_DOT = 4 };

// Arnoldi inner products fused into the last pass of an EPI_VIE operator:
// dotp[b][part][i] = vscale_i,b * sum over the part's rows of conj(V_i) . y,
// i < nvec, one part per workgroup of the inverse row pass. Done only when
// every workgroup's rows belong to one RHS and there are at most kMaxDotParts
// parts per RHS; launch_vie reports whether it did them (and `nparts`).
constexpr int kMaxDotParts = 2048;
struct VieDots {
  const void* basis = nullptr;   // V_0 [B][n] (cplx<T>), vector i at basis + i*vs
  long vs = 0;
  int nvec = 0;                  // j + 1
  const void* vscale = nullptr;  // [JM+1][B] cplx<T>
  c128* dotp = nullptr;          // [B][nparts][dstride]
  int dstride = 0;               // JM + 1
  int nparts = 0;                // out: parts per RHS
};

// Solution update of a refinement cycle fused into the first pass of the
// next FP64 residual: before its row transform, every RHS forms
// x_b = (first ? 0 : x_b) + sum_{i < ncol_b} coef[b][i] V_i,b (FP64), stores it
// back into x and transforms it (the residual is then that of the new x).
struct XUpdate {
  const void* basis = nullptr;  // V_0 [B][n] of complex64 (fp32) or complex128, vector i at basis + i*vs
  bool fp32 = true;
  long vs = 0;
  const int* ncol = nullptr;    // [B] vectors per RHS
  const c128* coef = nullptr;   // [B][cstride]
  int cstride = 0;
  int first = 0;
  int kmax = 0;                 // bound on ncol (profiled bytes only)
};

// Arnoldi orthogonalisation fused into the first pass of the next matvec:
// the new vector w (stored in place of V_nvec) becomes
// v = w + sum_{i < nvec} coef[b][i] V_i (FP64, coef = -h_i times the stored
// vector's scale), is rounded and stored back, |v|^2 is summed per grid row
// into rowpart, and v (unscaled) is row-transformed unless !transform.
struct OrthIn {
  const void* basis = nullptr;  // V_0 [B][n] (cplx<T>), vector i at basis + i*vs
  long vs = 0;
  int nvec = 0;
  const c128* coef = nullptr;   // [B][cstride]
  int cstride = 0;
  double* rowpart = nullptr;    // [B * rows per RHS]
  bool transform = true;
};

// First cycle (x_0 = 0, r = b) fused into the first pass: V_0 = b rounded to
// the basis precision, |b|^2 summed per grid row into rowpart (FP64), V_0
// (unscaled) row-transformed, for every RHS.
struct StartIn {
  const c128* b = nullptr;      // [B][n]
  double* rowpart = nullptr;    // [B * rows per RHS]
};

// y = A x for B right-hand sides (Eq. 5 discretised):
//   EPI_VIE  : y_b = s_b (x_b - conv(m * x_b)) = s_b x_b - conv(m * s_b x_b)
//   EPI_RESID: y_b = rhs_b - (x_b - conv(m * x_b))        (scale ignored), and
//              rowpart[row] = sum over the row of |y_b|^2 (rows of nx points)
//   EPI_RESID32: the same residual rounded to complex64 into y32 (y unused)
// x, y, rhs: [B][n]; scale: [B] or null; active: [B] or null (inactive RHS are
// skipped and their y left untouched); ghat: [nf][npad] spectra with k^2 and
// 1/npad folded in; rhs_freq: [B] frequency index per RHS; U1 [B][u1],
// U2 [B][u2] (3D) scratch. xu (FP64 residuals only): x is first updated in
// place as described for XUpdate.
template <typename T>
void launch_vie(const Geo& g, const Twiddles& tw, int B, const cplx<T>* x, const cplx<T>* scale, const int* active,
                const cplx<T>* m, const cplx<T>* ghat, const int* rhs_freq, cplx<T>* U1, cplx<T>* U2, cplx<T>* y,
                const cplx<T>* rhs, int epi, hipStream_t st, c64* y32 = nullptr, double* rowpart = nullptr,
                VieDots* dots = nullptr,  // returns through dots->nparts (0: not fused)
                const XUpdate* xu = nullptr);
// The same operator in two launches groups: the first pass (rows of x, or of
// the combined input of xu / orth, transformed into U1, or into U2 when the
// lateral and elevation passes are fused) and the rest.
template <typename T>
void launch_vie_rows(const Geo& g, const Twiddles& tw, int B, const cplx<T>* x, const int* active, const cplx<T>* m,
                     cplx<T>* U1, hipStream_t st, const XUpdate* xu = nullptr, const OrthIn* orth = nullptr,
                     const StartIn* start = nullptr,
                     cplx<T>* U2 = nullptr);  // written instead of U1 by a fused lateral-elevation pass (g.xy)
template <typename T>
void launch_vie_tail(const Geo& g, const Twiddles& tw, int B, const cplx<T>* x, const cplx<T>* scale,
                     const int* active, const cplx<T>* ghat, const int* rhs_freq, cplx<T>* U1, cplx<T>* U2,
                     cplx<T>* y, const cplx<T>* rhs, int epi, hipStream_t st, c64* y32 = nullptr,
                     double* rowpart = nullptr, VieDots* dots = nullptr);

// Forward FFT of a full padded grid [Lz][Ly][Lx] (no padding, no crop), in place
// through `work` of the same size: out = FFT(in). Used for the Green spectrum.
void launch_fft_full(const Geo& g, const Twiddles& tw, const c128* in, c128* work, c128* out, hipStream_t st);

// Zero-padded forward FFT of [nz][ny][nx] data into [Lz][Ly][Lx] (diagnostics).
template <typename T>
void launch_fft_padded(const Geo& g, const Twiddles& tw, const cplx<T>* in, cplx<T>* U1, cplx<T>* out,
                       hipStream_t st);

// ---------------------------------------------------------- setup kernels ---
// kappa_0 rho_0 of the background: 1/c0^2 - alpha0^2/(4 pi^2) + i alpha0/(pi c0)
inline c128 kappa0_rho(double c0, double alpha0) {
  const double pi = 3.14159265358979323846;
  return mk(1.0 / (c0 * c0) - alpha0 * alpha0 / (4.0 * pi * pi), alpha0 / (pi * c0));
}
void launch_contrast(long n, double c0, double alpha0, const double* c, const double* alpha, c128* m64, c64* m32,
                     hipStream_t st);
void launch_sos_from_contrast(long n, c128 k0r, const c128* m, double* c, double* alpha, hipStream_t st);
void launch_green_table(const Geo& g, c128 k, c128* table, hipStream_t st);
// Gauss-Legendre rule on [-1, 1] for the element apertures.
constexpr int kMaxGaussPoints = 16;
struct GaussRule {
  int q;
  double x[kMaxGaussPoints], w[kMaxGaussPoints];
};
GaussRule gauss_legendre(int q);
// Element aperture: half width (x) and half height (y) [m] and the rule used
// in each direction with a nonzero extent.
struct Aperture {
  double hw, hh;
  GaussRule rule;
};
void launch_incident(const Geo& g, c128 k, int ne, const double* elem_xyz_dev, const Aperture& ap, c128* P0,
                     hipStream_t st);
void launch_cast_64_32(long count, const c128* in, c64* out, hipStream_t st);
void launch_cast_xy_64_32(const Geo& g, const c128* in, c64* out, hipStream_t st);  // class-major (g.xy)
void launch_scale_c128(long count, double s, c128* x, hipStream_t st);

}  // namespace fwi

namespace fwi {
void launch_check_sos(long n, const double* c, const double* alpha, int* out, hipStream_t st);
void launch_check_complex(long n, const c128* x, int* out, hipStream_t st);
}  // namespace fwi
