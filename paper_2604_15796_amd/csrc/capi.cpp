// C ABI of the FWI hot path (include/fwi.h): argument validation, the
// per-problem caches (Green spectra, incident fields), the workspace arena,
// the batched Krylov driver and the entry points of Sec. II-IV.
#include "../../include/fwi.h"

#include <chrono>
#include <complex>
#include <cmath>
#include <cstring>
#include <limits>
#include <map>
#include <set>
#include <sstream>
#include <string>
#include <type_traits>
#include <utility>
#include <vector>

#include "data.hpp"
#include "internal.hpp"
#include "krylov.hpp"

#ifdef FWI_WORKSPACE_GUARD
#include <sanitizer/asan_interface.h>
#endif

using namespace fwi;

namespace fwi {

thread_local LaunchProfiler* tl_prof = nullptr;
thread_local long tl_active = 0;
thread_local hipEvent_t tl_ev_start = nullptr, tl_ev_stop = nullptr;
thread_local bool tl_ev_used = false;
thread_local int tl_nfreq = 0;
thread_local const FftTuning* tl_tune = nullptr;
thread_local int tl_force_variant = -1;
thread_local int tl_force_wide = 0;
thread_local int tl_xy_off = 0;

int default_variant(int pass, bool dbl, int L) {
  if (pass == PK_ROW_FWD || pass == PK_ROW_INV) return 0;  // 2048 points per workgroup
  if (pass == PK_CONV && L == 192) return 1;                 // (16, 256): the radix 16 x 12 plan
  if (pass == PK_CONV && !dbl) return 2;                     // (16, 512) columns, threads
  return dbl ? 0 : 1;                                        // (8, 256) / (16, 256)
}

// Fastest variant by measured time; another variant replaces the default only
// if it is at least 2% faster (timing noise does not flip the choice).
int pick_variant(const double* t, int dflt) {
  int best = dflt;
  for (int v = 0; v < kNumVariants; ++v)
    if (v != best && t[v] > 0.0 && t[v] < 0.98 * t[best]) best = v;
  return best;
}

int tune_variant(int pass, bool dbl, int L) {
  if (tl_force_variant >= 0) return tl_force_variant;
  const int li = length_index(L);
  if (tl_tune && li >= 0) {
    const int v = tl_tune->v[pass][dbl ? 1 : 0][li];
    if (v >= 0 && v < kNumVariants) return v;
  }
  return default_variant(pass, dbl, L);
}

int length_index(int L) {
  for (int i = 0; i < kNumLengths; ++i)
    if (kLengths[i] == L) return i;
  return -1;
}
int padded_length(int n) {
  if (n < 1) return 0;
  for (int i = 0; i < kNumLengths; ++i)
    if (kLengths[i] >= 2 * n) return kLengths[i];
  return 0;
}
template <>
const c128* Twiddles::get<double>(int L) const {
  const int i = length_index(L);
  if (i < 0) throw Error(FWI_E_UNSUPPORTED, "no twiddles for length " + std::to_string(L));
  return d64[i];
}
template <>
const c64* Twiddles::get<float>(int L) const {
  const int i = length_index(L);
  if (i < 0) throw Error(FWI_E_UNSUPPORTED, "no twiddles for length " + std::to_string(L));
  return d32[i];
}

}  // namespace fwi

namespace {

// --------------------------------------------------------------- arena ---
// Host sanitizer builds of this file (FWI_WORKSPACE_GUARD, tests only) leave
// a poisoned gap after every workspace buffer, so that an access past a
// planned extent is reported; the library build has no gap.
#ifdef FWI_WORKSPACE_GUARD
constexpr size_t kArenaGuard = 256;
inline void guard_poison(char* p, size_t n) { ASAN_POISON_MEMORY_REGION(p, n); }
inline void guard_clear(char* p, size_t n) { ASAN_UNPOISON_MEMORY_REGION(p, n); }
#else
constexpr size_t kArenaGuard = 0;
inline void guard_poison(char*, size_t) {}
inline void guard_clear(char*, size_t) {}
#endif

struct Arena {
  char* base = nullptr;
  size_t cap = 0, used = 0;
  bool dry = true;
  template <typename T>
  T* take(size_t count) {
    const size_t bytes = (count * sizeof(T) + 255) & ~size_t(255);
    const size_t off = used;
    used += bytes + kArenaGuard;
    if (dry) return nullptr;
    if (used > cap) throw Error(FWI_E_NOMEM, "workspace exhausted");
    guard_poison(base + off + count * sizeof(T), bytes - count * sizeof(T) + kArenaGuard);
    return reinterpret_cast<T*>(base + off);
  }
  // plan again from the start of the bound workspace
  void rewind() {
    used = 0;
    if (base) guard_clear(base, cap);
  }
};

// ------------------------------------------------------- problem cache ---
struct ProblemCache {
  std::string key;
  Geo g;
  int nf = 0, ne = 0;
  std::vector<c128> k;  // background wavenumbers (complex for a lossy background)
  c128* ghat64 = nullptr;   // [nf][npad]
  c64* ghat32 = nullptr;    // [nf][npad]
  c128* P0 = nullptr;       // [nf][ne][n]
  c128* k2 = nullptr;       // [nf]  k_l^2
  c128* coef = nullptr;     // [nf]  k_l^2 dV
  int* rhs_freq = nullptr;  // [nf*ne]
  double* elems = nullptr;  // [ne][3]
  void release() {
    void* ps[] = {ghat64, ghat32, P0, k2, coef, rhs_freq, elems};
    for (void* p : ps)
      if (p) (void)hipFree(p);
    ghat64 = nullptr;
    ghat32 = nullptr;
    P0 = nullptr;
    k2 = coef = nullptr;
    rhs_freq = nullptr;
    elems = nullptr;
    key.clear();
  }
};

// HIP-event timing of selected kernel classes, on the stream they run on.
struct EventProfiler : LaunchProfiler {
  unsigned mask = 0;
  std::vector<hipEvent_t> pool;
  size_t used = 0;
  struct Rec {
    int cls;
    hipEvent_t a, b;
    double per_rhs, fixed;
    bool masked;
    long B, act;
  };
  std::vector<Rec> recs;
  double tot_ms[2 * KC_COUNT] = {};
  long long cnt[2 * KC_COUNT] = {};
  double byt[2 * KC_COUNT] = {};
  hipEvent_t get() {
    if (used == pool.size()) {
      // timing-only events: no system-scope fence, so a recorded event does
      // not hold back the next launch
      hipEvent_t e;
      FWI_HIP(hipEventCreateWithFlags(&e, hipEventDisableSystemFence));
      pool.push_back(e);
    }
    return pool[used++];
  }
  // the region's single kernel launch records the two events
  void begin(int cls, hipStream_t) override {
    if (!((mask >> cls) & 1u)) return;
    tl_ev_start = get();
    tl_ev_stop = get();
    tl_ev_used = false;
  }
  void end(int cls, hipStream_t, double per_rhs, double fixed, bool masked, long B) override {
    if (!((mask >> cls) & 1u)) return;
    const long act = masked && tl_active > 0 && tl_active < B ? tl_active : B;
    if (tl_ev_used) recs.push_back({cls, tl_ev_start, tl_ev_stop, per_rhs, fixed, masked, B, act});
    tl_ev_start = tl_ev_stop = nullptr;
    tl_ev_used = false;
  }
  size_t mark() const override { return recs.size(); }
  void set_active(size_t from, long act) override {
    for (size_t k = from; k < recs.size(); ++k)
      if (recs[k].masked) recs[k].act = act < recs[k].B ? act : recs[k].B;
  }
  void flush() {
    for (const Rec& r : recs) {
      FWI_HIP(hipEventSynchronize(r.b));
      float ms = 0.f;
      FWI_HIP(hipEventElapsedTime(&ms, r.a, r.b));
      tot_ms[r.cls] += ms;
      cnt[r.cls] += 1;
      byt[r.cls] += r.per_rhs * (double)r.act + r.fixed;
    }
    recs.clear();
    used = 0;
  }
  void reset() {
    recs.clear();
    used = 0;
    for (int k = 0; k < 2 * KC_COUNT; ++k) {
      tot_ms[k] = 0.0;
      cnt[k] = 0;
      byt[k] = 0.0;
    }
  }
  ~EventProfiler() override {
    for (hipEvent_t e : pool) (void)hipEventDestroy(e);
  }
};

double now_ms() {
  using namespace std::chrono;
  return duration<double, std::milli>(steady_clock::now().time_since_epoch()).count();
}

// Scratch of fwi_apply_operator_noalloc (for callers that cannot allocate):
// a file-scope device array, one copy per GPU the library runs on, held until
// the process ends. Host code never uses its name as an address: each context
// looks up its device's copy once (hipGetSymbolAddress at fwi_create, with
// that device current) and passes that pointer on.
constexpr size_t kStaticScratchBytes = size_t(64) << 20;
static __device__ __align__(256) char scratch[kStaticScratchBytes];

}  // namespace

struct fwi_ctx {
  int device = 0;
  int force_wide = 0;          // fwi_set_addressing
  int xy_off = 1;              // fused lateral-elevation passes off unless fwi_set_plane_fusion(ctx, 1)
  hipStream_t stream = nullptr;
  std::string err;
  Twiddles tw;
  std::vector<void*> tw_allocs;
  char* ws_ext = nullptr;
  size_t ws_ext_bytes = 0;
  char* ws_int = nullptr;
  size_t ws_int_bytes = 0;
  ProblemCache pc;
  int* h_int = nullptr;        // pinned host scratch
  double* h_dbl = nullptr;
  int* d_int = nullptr;        // device scratch for checks
  EventProfiler prof;
  FftTuning tune;
  std::map<std::string, ProblemCache> bcache;  // caches of the batched entry point
  hipStream_t cap_stream = nullptr;            // capture stream of the batched entry point
  std::vector<hipStream_t> branch;             // one per instance of a wave (default priority)
  std::vector<hipEvent_t> branch_ev;
  hipEvent_t fork_ev = nullptr;
  hipEvent_t count_ev = nullptr;               // active-count copy of the solver loop
  unsigned long long* d_itstat = nullptr;      // iteration max / sum of the current call's solves
  char* scratch_dev = nullptr;                 // this device's copy of `scratch`
  ~fwi_ctx() {
    if (count_ev) (void)hipEventDestroy(count_ev);
    for (auto& kv : bcache) kv.second.release();
    for (hipStream_t st : branch) (void)hipStreamDestroy(st);
    for (hipEvent_t e : branch_ev) (void)hipEventDestroy(e);
    if (fork_ev) (void)hipEventDestroy(fork_ev);
    if (cap_stream) (void)hipStreamDestroy(cap_stream);
  }
};

namespace {

int fail(fwi_ctx* ctx, int code, const std::string& msg) {
  if (ctx) ctx->err = msg;
  return code;
}

// ---------------------------------------------------------- validation ---
int validate_problem(const fwi_problem* p, std::string& msg) {
  if (!p) return msg = "problem is NULL", FWI_E_INVAL;
  if (p->dim != 2 && p->dim != 3) return msg = "dim must be 2 or 3", FWI_E_UNSUPPORTED;
  if (p->nx < 1 || p->nz < 1 || p->ny < 1) return msg = "grid extents must be >= 1", FWI_E_INVAL;
  if (p->dim == 2 && p->ny != 1) return msg = "ny must be 1 in 2D", FWI_E_INVAL;
  if (!padded_length(p->nx) || !padded_length(p->nz) || (p->dim == 3 && !padded_length(p->ny)))
    return msg = "grid extent above 512 cells per axis", FWI_E_UNSUPPORTED;
  if (!(p->dx > 0.0) || !std::isfinite(p->dx)) return msg = "dx must be finite and > 0", FWI_E_INVAL;
  if (!(p->c0 > 0.0) || !std::isfinite(p->c0)) return msg = "c0 must be finite and > 0", FWI_E_INVAL;
  if (p->nf < 1 || !p->freq_hz) return msg = "need nf >= 1 frequencies", FWI_E_INVAL;
  for (int l = 0; l < p->nf; ++l)
    if (!(p->freq_hz[l] > 0.0) || !std::isfinite(p->freq_hz[l])) return msg = "frequencies must be > 0", FWI_E_INVAL;
  if (p->ne < 1 || !p->elem_xyz) return msg = "need ne >= 1 elements", FWI_E_INVAL;
  if (p->ne > 256) return msg = "more than 256 elements", FWI_E_UNSUPPORTED;
  const double wx = p->nx * p->dx, wy = p->ny * p->dx;
  std::set<std::pair<double, double>> seen;
  for (int e = 0; e < p->ne; ++e) {
    const double x = p->elem_xyz[3 * e], y = p->elem_xyz[3 * e + 1], z = p->elem_xyz[3 * e + 2];
    if (!std::isfinite(x) || !std::isfinite(y) || !std::isfinite(z)) return msg = "non-finite element position", FWI_E_INVAL;
    if (z != 0.0) return msg = "elements must lie on the top face z = 0", FWI_E_UNSUPPORTED;
    if (x < 0.0 || x > wx) return msg = "element outside the lateral extent", FWI_E_INVAL;
    if (p->dim == 3 && (y < 0.0 || y > wy)) return msg = "element outside the elevation extent", FWI_E_INVAL;
    if (p->dim == 2 && y != 0.0) return msg = "2D elements must have y = 0", FWI_E_INVAL;
    if (!seen.insert({x, y}).second) return msg = "duplicate element position", FWI_E_INVAL;
  }
  if (!(p->elem_width >= 0.0) || !std::isfinite(p->elem_width) || !(p->elem_height >= 0.0) ||
      !std::isfinite(p->elem_height))
    return msg = "element aperture must be finite and >= 0", FWI_E_INVAL;
  if (p->dim == 2 && p->elem_height != 0.0) return msg = "2D elements have no height", FWI_E_INVAL;
  if ((p->elem_width > 0.0 || p->elem_height > 0.0) && (p->elem_quad < 1 || p->elem_quad > kMaxGaussPoints))
    return msg = "elem_quad must be in 1..16", FWI_E_INVAL;
  if (!(p->alpha0 >= 0.0) || !std::isfinite(p->alpha0)) return msg = "alpha0 must be finite and >= 0", FWI_E_INVAL;
  return FWI_OK;
}

int validate_opts(const fwi_solve_opts* o, std::string& msg) {
  if (!o) return msg = "opts is NULL", FWI_E_INVAL;
  if (o->precision != FWI_FP64 && o->precision != FWI_FP32_REFINE) return msg = "bad precision", FWI_E_INVAL;
  if (!(o->rtol > 0.0 && o->rtol < 1.0)) return msg = "rtol must be in (0, 1)", FWI_E_INVAL;
  if (o->restart != 8 && o->restart != 16 && o->restart != 32) return msg = "restart must be 8, 16 or 32", FWI_E_UNSUPPORTED;
  if (o->max_iter < 1) return msg = "max_iter must be >= 1", FWI_E_INVAL;
  if (o->precision == FWI_FP32_REFINE) {
    if (o->max_refine < 1) return msg = "max_refine must be >= 1", FWI_E_INVAL;
    if (!(o->inner_rtol > 0.0 && o->inner_rtol < 1.0)) return msg = "inner_rtol must be in (0, 1)", FWI_E_INVAL;
  }
  if (o->max_rhs < 0) return msg = "max_rhs must be >= 0", FWI_E_INVAL;
  if (o->check_every < 1) return msg = "check_every must be >= 1", FWI_E_INVAL;
  if (o->tx_chunk < 0) return msg = "tx_chunk must be >= 0", FWI_E_INVAL;
  if (o->fields_c64 != 0 && o->fields_c64 != 1) return msg = "fields_c64 must be 0 or 1", FWI_E_INVAL;
  return FWI_OK;
}

Geo make_geo(const fwi_problem* p) {
  Geo g;
  g.dim = p->dim;
  g.nx = p->nx;
  g.ny = p->dim == 3 ? p->ny : 1;
  g.nz = p->nz;
  g.Lx = padded_length(g.nx);
  g.Ly = p->dim == 3 ? padded_length(g.ny) : 1;
  g.Lz = padded_length(g.nz);
  g.dx = p->dx;
  g.c0 = p->c0;
  g.alpha0 = p->alpha0;
  g.xy = xy_applies(g);
  return g;
}

// 1 / (kappa0 rho0) of a problem's background (c0^2 when lossless)
c128 inv_kappa0(const Geo& g) {
  if (g.alpha0 == 0.0) return mk(g.c0 * g.c0, 0.0);
  const c128 k = kappa0_rho(g.c0, g.alpha0);
  const double d = k.x * k.x + k.y * k.y;
  return mk(k.x / d, -k.y / d);
}

// Cache key of a problem: the raw bytes of everything the cached data depend
// on (exact comparison, no formatting cost).
std::string problem_key(const fwi_problem* p) {
  std::string k;
  auto put = [&k](const void* src, size_t bytes) { k.append(static_cast<const char*>(src), bytes); };
  const int ints[5] = {p->dim, p->nx, p->ny, p->nz, p->nf};
  put(ints, sizeof(ints));
  put(&p->dx, sizeof(double));
  put(&p->c0, sizeof(double));
  put(p->freq_hz, sizeof(double) * p->nf);
  put(&p->ne, sizeof(int));
  put(p->elem_xyz, sizeof(double) * 3 * p->ne);
  const bool ap = p->elem_width > 0.0 || p->elem_height > 0.0;
  const double aw = p->elem_width, ah = p->elem_height;
  const int q = ap ? p->elem_quad : 0;
  put(&aw, sizeof(double));
  put(&ah, sizeof(double));
  put(&q, sizeof(int));
  put(&p->alpha0, sizeof(double));
  // the layout of the cached complex64 kernel spectrum
  const int xy = tl_xy_off;
  put(&xy, sizeof(int));
  return k;
}

// ------------------------------------------------------------ twiddles ---
void make_twiddles(fwi_ctx* c) {
  for (int li = 0; li < kNumLengths; ++li) {
    const int L = kLengths[li];
    std::vector<c128> h64(L);
    std::vector<c64> h32(L);
    for (int m = 0; m < L; ++m) {
      const long double ang = -2.0L * 3.141592653589793238462643383279502884L * (long double)m / (long double)L;
      h64[m] = mk((double)cosl(ang), (double)sinl(ang));
      h32[m] = mk((float)cosl(ang), (float)sinl(ang));
    }
    void *p64 = nullptr, *p32 = nullptr;
    FWI_HIP(hipMalloc(&p64, sizeof(c128) * L));
    c->tw_allocs.push_back(p64);
    FWI_HIP(hipMalloc(&p32, sizeof(c64) * L));
    c->tw_allocs.push_back(p32);
    FWI_HIP(hipMemcpy(p64, h64.data(), sizeof(c128) * L, hipMemcpyHostToDevice));
    FWI_HIP(hipMemcpy(p32, h32.data(), sizeof(c64) * L, hipMemcpyHostToDevice));
    c->tw.d64[li] = (const c128*)p64;
    c->tw.d32[li] = (const c64*)p32;
  }
}

// --------------------------------------------------------- cache build ---
// Green spectra (FP64 FFT of the circulant table, cast to FP32 as well) and
// incident fields of every frequency, built into `pc`.
double build_cache(fwi_ctx* c, const fwi_problem* p, ProblemCache& pc, const std::string& key) {
  const double t0 = now_ms();
  pc.release();
  pc.g = make_geo(p);
  pc.nf = p->nf;
  pc.ne = p->ne;
  const Geo& g = pc.g;
  const long n = g.n(), np = g.npad();
  hipStream_t st = c->stream;
  FWI_HIP(hipMalloc((void**)&pc.ghat64, sizeof(c128) * np * pc.nf));
  FWI_HIP(hipMalloc((void**)&pc.ghat32, sizeof(c64) * np * pc.nf));
  FWI_HIP(hipMalloc((void**)&pc.P0, sizeof(c128) * n * pc.ne * pc.nf));
  FWI_HIP(hipMalloc((void**)&pc.k2, sizeof(c128) * pc.nf));
  FWI_HIP(hipMalloc((void**)&pc.coef, sizeof(c128) * pc.nf));
  FWI_HIP(hipMalloc((void**)&pc.rhs_freq, sizeof(int) * pc.nf * pc.ne));
  FWI_HIP(hipMalloc((void**)&pc.elems, sizeof(double) * 3 * pc.ne));
  FWI_HIP(hipMemcpyAsync(pc.elems, p->elem_xyz, sizeof(double) * 3 * pc.ne, hipMemcpyHostToDevice, st));
  std::vector<c128> hk2(pc.nf), hcoef(pc.nf);
  std::vector<int> hrf((size_t)pc.nf * pc.ne);
  const double dV = std::pow(g.dx, g.dim);
  pc.k.resize(pc.nf);
  c128 *table = nullptr, *work = nullptr;
  FWI_HIP(hipMalloc((void**)&table, sizeof(c128) * np));
  FWI_HIP(hipMalloc((void**)&work, sizeof(c128) * np));
  Aperture ap{};
  ap.hw = 0.5 * p->elem_width;
  ap.hh = 0.5 * p->elem_height;
  ap.rule = gauss_legendre(ap.hw > 0.0 || ap.hh > 0.0 ? p->elem_quad : 1);
  for (int l = 0; l < pc.nf; ++l) {
    // k = omega sqrt(kappa0 rho0), the root with Im k >= 0 (decaying)
    const double w = 2.0 * 3.14159265358979323846 * p->freq_hz[l];
    c128 k = mk(w / p->c0, 0.0);
    if (p->alpha0 > 0.0) {
      const c128 k0r = kappa0_rho(p->c0, p->alpha0);
      const std::complex<double> s = std::sqrt(std::complex<double>(k0r.x, k0r.y));
      k = mk(w * s.real(), w * s.imag());
    }
    pc.k[l] = k;
    hk2[l] = k * k;
    hcoef[l] = dV * (k * k);
    for (int e = 0; e < pc.ne; ++e) hrf[(size_t)l * pc.ne + e] = l;
    launch_green_table(g, k, table, st);
    launch_fft_full(g, c->tw, table, work, pc.ghat64 + (long)l * np, st);
    if (g.xy) launch_cast_xy_64_32(g, pc.ghat64 + (long)l * np, pc.ghat32 + (long)l * np, st);
    else launch_cast_64_32(np, pc.ghat64 + (long)l * np, pc.ghat32 + (long)l * np, st);
    launch_incident(g, k, pc.ne, pc.elems, ap, pc.P0 + (long)l * pc.ne * n, st);
  }
  FWI_HIP(hipMemcpyAsync(pc.k2, hk2.data(), sizeof(c128) * pc.nf, hipMemcpyHostToDevice, st));
  FWI_HIP(hipMemcpyAsync(pc.coef, hcoef.data(), sizeof(c128) * pc.nf, hipMemcpyHostToDevice, st));
  FWI_HIP(hipMemcpyAsync(pc.rhs_freq, hrf.data(), sizeof(int) * hrf.size(), hipMemcpyHostToDevice, st));
  FWI_HIP(hipStreamSynchronize(st));
  FWI_HIP(hipFree(table));
  FWI_HIP(hipFree(work));
  pc.key = key;
  return now_ms() - t0;
}

// The single-problem cache used by the per-problem entry points.
double ensure_cache(fwi_ctx* c, const fwi_problem* p) {
  const std::string key = problem_key(p);
  if (key == c->pc.key) return 0.0;
  return build_cache(c, p, c->pc, key);
}

// ----------------------------------------------------------- workspace ---
void bind_workspace(fwi_ctx* c, Arena& a, size_t need) {
  a.dry = false;
  a.used = 0;
  if (c->ws_ext) {
    if (need > c->ws_ext_bytes)
      throw Error(FWI_E_NOMEM, "caller workspace too small: need " + std::to_string(need) + " bytes");
    a.base = c->ws_ext;
    a.cap = c->ws_ext_bytes;
    a.rewind();
    return;
  }
  if (need > c->ws_int_bytes) {
    if (c->ws_int) FWI_HIP(hipFree(c->ws_int));
    c->ws_int = nullptr;
    c->ws_int_bytes = 0;
    if (hipMalloc((void**)&c->ws_int, need) != hipSuccess) {
      (void)hipGetLastError();
      throw Error(FWI_E_NOMEM, "cannot allocate " + std::to_string(need) + " bytes of workspace");
    }
    c->ws_int_bytes = need;
  }
  a.base = c->ws_int;
  a.cap = c->ws_int_bytes;
  a.rewind();
}

// ------------------------------------------------------- solve buffers ---
template <typename T>
struct SolveBufs {
  KrylovState<T> ks;
  double* rowpart = nullptr;  // [B][nz*ny] residual norm partials
  cplx<T>* U1 = nullptr;
  cplx<T>* U2 = nullptr;
  c128* U1_64 = nullptr;
  c128* U2_64 = nullptr;
};

// Inner-product partials per RHS: the k_dots blocks, or one per workgroup of
// the inverse row pass when the products are fused into it (its smallest
// tile holds 2048 points, max(2048 / Lx, 1) rows; at most kMaxDotParts).
int dot_parts(const Geo& g, int nblk) {
  const long rows = (long)g.nz * g.ny;
  const long nl0 = std::max(2048 / g.Lx, 1);
  const long fused = std::min<long>(kMaxDotParts, (rows + nl0 - 1) / nl0);
  return (int)std::max<long>(nblk, fused);
}

template <typename T>
void plan_solve(Arena& a, const Geo& g, int B, int JM, SolveBufs<T>& s) {
  KrylovState<T>& k = s.ks;
  const long n = g.n();
  k.B = B;
  k.JM = JM;
  k.n = n;
  k.nblk = krylov_nblk(n);
  k.chunk = (int)((n + k.nblk - 1) / k.nblk);
  k.V = a.take<cplx<T>>((size_t)(JM + 1) * B * n);
  k.H = a.take<c128>((size_t)B * (JM + 1) * JM);
  k.cs = a.take<double>((size_t)B * JM);
  k.sn = a.take<c128>((size_t)B * JM);
  k.gv = a.take<c128>((size_t)B * (JM + 1));
  k.y = a.take<c128>((size_t)B * JM);
  k.dotp = a.take<c128>((size_t)B * dot_parts(g, k.nblk) * (JM + 1));
  k.hcoef = a.take<c128>((size_t)B * (JM + 1));
  k.nrmp = a.take<double>((size_t)B * k.nblk);
  k.rnorm = a.take<double>(B);
  k.bnorm = a.take<double>(B);
  k.target = a.take<double>(B);
  k.rscale = a.take<double>(B);
  k.vscale = a.take<cplx<T>>((size_t)(JM + 1) * B);
  k.active = a.take<int>(B);
  k.ncol = a.take<int>(B);
  k.iters = a.take<int>(B);
  k.counters = a.take<int>(4);  // active counts, then the max relative residual: one copy reads both
  k.maxrel = k.counters ? reinterpret_cast<double*>(k.counters + 2) : nullptr;
  s.rowpart = a.take<double>((size_t)B * g.nz * g.ny);
  s.U1 = a.take<cplx<T>>((size_t)B * g.u1());
  s.U2 = g.dim == 3 ? a.take<cplx<T>>((size_t)B * g.u2()) : nullptr;
  if (std::is_same<T, float>::value) {
    s.U1_64 = a.take<c128>((size_t)B * g.u1());
    s.U2_64 = g.dim == 3 ? a.take<c128>((size_t)B * g.u2()) : nullptr;
  } else {
    s.U1_64 = reinterpret_cast<c128*>(s.U1);
    s.U2_64 = reinterpret_cast<c128*>(s.U2);
  }
}

struct SolveTotals {
  int iters_max = 0, cycles = 0, unconverged = 0;
  double maxrel = 0.0;
  long long solves = 0, matvecs = 0;
  double t_solve = 0.0;
  void merge(const SolveTotals& o) {
    iters_max = std::max(iters_max, o.iters_max);
    cycles = std::max(cycles, o.cycles);
    unconverged += o.unconverged;
    maxrel = std::max(maxrel, o.maxrel);
    solves += o.solves;
    matvecs += o.matvecs;
    t_solve += o.t_solve;
  }
};

// Batched solve A_{f_b} x_b = b_b for B right-hand sides (restarted GMRES in
// FP64, or FP32 GMRES cycles inside FP64-residual iterative refinement).
// Each cycle starts from the true FP64 residual r = b - A x, normalises it,
// runs at most `restart` Arnoldi steps per RHS (stopping each RHS at its
// target) and adds the correction to the FP64 solution x.
// Inner products of Arnoldi step j, to be fused into the operator's last pass.
template <typename T>
VieDots arnoldi_dots(const KrylovState<T>& ks, int j) {
  VieDots d;
  d.basis = ks.V;
  d.vs = ks.vstride();
  d.nvec = j + 1;
  d.vscale = ks.vscale;
  d.dotp = ks.dotp;
  d.dstride = ks.JM + 1;
  return d;
}

// Orthogonalisation of the matvec result of step j (stored in V_{j+1}),
// fused into the first pass of step j + 1 (or done alone after the last step).
template <typename T>
OrthIn arnoldi_orth(const KrylovState<T>& ks, int j, double* rowpart, bool transform) {
  OrthIn o;
  o.basis = ks.V;
  o.vs = ks.vstride();
  o.nvec = j + 1;
  o.coef = ks.hcoef;
  o.cstride = ks.JM + 1;
  o.rowpart = rowpart;
  o.transform = transform;
  return o;
}

// Arnoldi steps of one cycle, in launch order. Step j: the tail of the
// matvec (convolution, last pass with the inner products of w = A v_j
// against V_0..V_j) writes w into V_{j+1}; then column j of H is summed and
// the first pass of the next matvec orthogonalises w into v_{j+1}, stores it,
// sums |v_{j+1}|^2 per row and row-transforms it (only orthogonalises after
// the last step); then the Givens kernel finishes column j and sets the scale
// of v_{j+1}, so the next tail runs on the RHS still active.
template <typename T>
struct ArnoldiDriver {
  const Geo& g;
  const Twiddles& tw;
  KrylovState<T>& ks;
  SolveBufs<T>& s;
  const cplx<T>* mT;
  const cplx<T>* ghatT;
  const int* rhs_freq;
  hipStream_t st;
  int B;
  // first pass of step 0 on V_0 (scaled by vscale_0 in the last pass)
  void first_rows() {
    launch_vie_rows<T>(g, tw, B, ks.V, ks.active, mT, s.U1, st, nullptr, nullptr, nullptr, s.U2);
  }
  // rest of step j: w into V_{j+1}, inner products, column j of H
  void tail(int j) {
    const long vs = ks.vstride();
    VieDots dots = arnoldi_dots(ks, j);
    launch_vie_tail<T>(g, tw, B, ks.V + (long)j * vs, ks.vscale + (long)j * ks.B, ks.active, ghatT, rhs_freq, s.U1,
                       s.U2, ks.V + (long)(j + 1) * vs, nullptr, EPI_VIE, st, nullptr, nullptr, &dots);
    int ndot = dots.nparts;
    if (ndot == 0) {
      krylov_dots(ks, j, st);
      ndot = ks.nblk;
    }
    krylov_hsum(ks, j, ndot, st);
  }
  // orthogonalise w_{j+1} (and transform it unless this was the last step),
  // then the rotations of column j
  void orth_givens(int j, bool transform) {
    const OrthIn o = arnoldi_orth(ks, j, s.rowpart, transform);
    launch_vie_rows<T>(g, tw, B, ks.V + (long)(j + 1) * ks.vstride(), ks.active, mT, s.U1, st, nullptr, &o,
                       nullptr, s.U2);
    krylov_givens(ks, j, s.rowpart, g.nz * g.ny, st);
  }
};

// r = b - A x in FP64 for every RHS; the epilogue stores r into V_0 of the
// basis (rounded to the basis precision) and one |r|^2 partial per grid row.
template <typename T>
void launch_residual_basis(const Geo& g, const Twiddles& tw, int B, const c128* x64, const c128* m64,
                           const c128* ghat64, const int* rhs_freq, SolveBufs<T>& s, const c128* b64,
                           hipStream_t st, const XUpdate* xu = nullptr) {
  if (std::is_same<T, float>::value)
    launch_vie<double>(g, tw, B, x64, nullptr, nullptr, m64, ghat64, rhs_freq, s.U1_64, s.U2_64, nullptr, b64,
                       EPI_RESID32, st, reinterpret_cast<c64*>(s.ks.V), s.rowpart, nullptr, xu);
  else
    launch_vie<double>(g, tw, B, x64, nullptr, nullptr, m64, ghat64, rhs_freq, s.U1_64, s.U2_64,
                       reinterpret_cast<c128*>(s.ks.V), b64, EPI_RESID, st, nullptr, s.rowpart, nullptr, xu);
}

// The correction of a finished cycle, applied by the next residual's first pass.
template <typename T>
XUpdate cycle_update(const KrylovState<T>& ks, int first, int steps) {
  XUpdate u;
  u.basis = ks.V;
  u.fp32 = std::is_same<T, float>::value;
  u.vs = ks.vstride();
  u.ncol = ks.ncol;
  u.coef = ks.y;
  u.cstride = ks.JM;
  u.first = first;
  u.kmax = steps;
  return u;
}

template <typename T>
SolveTotals run_solve(fwi_ctx* c, const Geo& g, const c128* m64, const cplx<T>* mT, const c128* ghat64,
                      const cplx<T>* ghatT, int B, const c128* b64, const int* rhs_freq, c128* x64,
                      const fwi_solve_opts& o, SolveBufs<T>& s, int nfreq) {
  tl_nfreq = nfreq;
  hipStream_t st = c->stream;
  KrylovState<T>& ks = s.ks;
  const bool fp32 = std::is_same<T, float>::value;
  const double inner = fp32 ? o.inner_rtol : 0.0;
  const int max_cycles = fp32 ? o.max_refine : (o.max_iter + o.restart - 1) / o.restart + 1;
  const double t0 = now_ms();
  SolveTotals res;
  res.solves = B;
  krylov_reset_iters(ks, st);
  int total = 0, cyc = 0;
  bool x_written = false;
  XUpdate pending_x;  // correction of the last cycle, not yet added to x
  ArnoldiDriver<T> drv{g, c->tw, ks, s, mT, ghatT, rhs_freq, st, B};
  for (;; ++cyc) {
    if (cyc == 0) {
      // x_0 = 0, r = b: the first pass casts b into V_0, sums |b|^2 per row
      // and transforms V_0 (every RHS; masks come with the cycle start)
      const StartIn si{b64, s.rowpart};
      launch_vie_rows<T>(g, c->tw, B, ks.V, nullptr, mT, s.U1, st, nullptr, nullptr, &si, s.U2);
      krylov_rows_norm(ks, s.rowpart, g.nz * g.ny, st);
    } else {
      // FP64 residual of x plus the last cycle's correction (added to x by
      // its first pass); its epilogue writes V_0 (unscaled) and per-row norms
      tl_active = B;
      launch_residual_basis(g, c->tw, B, x64, m64, ghat64, rhs_freq, s, b64, st, &pending_x);
      x_written = true;
      krylov_rows_norm(ks, s.rowpart, g.nz * g.ny, st);
      res.matvecs += B;
    }
    krylov_cycle_init(ks, cyc == 0, o.rtol, inner, st);
    FWI_HIP(hipMemcpyAsync(c->h_int, ks.counters, 2 * sizeof(int) + sizeof(double), hipMemcpyDeviceToHost, st));
    FWI_HIP(hipEventRecord(c->count_ev, st));
    FWI_HIP(hipEventSynchronize(c->count_ev));
    std::memcpy(&res.maxrel, c->h_int + 2, sizeof(double));
    if (!std::isfinite(res.maxrel)) throw Error(FWI_E_NONFINITE, "non-finite residual in the Krylov solve");
    const int nact = c->h_int[0];
    tl_active = nact;
    if (nact == 0) break;
    if (cyc >= max_cycles || total >= o.max_iter) {
      res.unconverged = nact;
      break;
    }
    // The active count after step j-1 is copied asynchronously and read only
    // once step j is enqueued, so the device does not wait for the host
    // between steps; a step enqueued after every RHS stopped runs fully masked.
    // Once at most half the RHS are left, the host waits for each count
    // before enqueueing the next step instead (a wait costs less than a
    // masked step).
    bool pending = false;
    int known = nact;  // latest active count read
    int steps = 0;     // Arnoldi steps of this cycle
    if (cyc > 0) drv.first_rows();
    for (int j = 0;; ++j) {
      const size_t mark = tl_prof ? tl_prof->mark() : 0;
      drv.tail(j);
      ++total;
      ++steps;
      const bool last = j + 1 == ks.JM || total >= o.max_iter;
      drv.orth_givens(j, !last);
      if (pending) {
        pending = false;
        FWI_HIP(hipEventSynchronize(c->count_ev));
        known = c->h_int[8];  // RHS that step j processed
        tl_active = known;
        if (tl_prof) tl_prof->set_active(mark, known);
        if (known == 0) {
          --total;
          --steps;
          break;
        }
      }
      if (last) break;
      if ((j + 1) % o.check_every == 0) {
        FWI_HIP(hipMemcpyAsync(c->h_int + 8, ks.counters, sizeof(int), hipMemcpyDeviceToHost, st));
        FWI_HIP(hipEventRecord(c->count_ev, st));
        if (2 * known <= B) {
          FWI_HIP(hipEventSynchronize(c->count_ev));
          known = c->h_int[8];
          tl_active = known;
          if (known == 0) break;
        } else {
          pending = true;
        }
      }
    }
    krylov_backsolve(ks, st);
    pending_x = cycle_update(ks, cyc == 0, steps);
  }
  if (!x_written) launch_fill_zero_c128((long)B * ks.n, x64, st);  // nothing to solve: x = 0
  res.cycles = cyc;
  // iteration counts stay on the device until the call collects them
  launch_iter_stats(B, ks.iters, c->d_itstat, st);
  res.t_solve = now_ms() - t0;  // the last cycle start was waited for: the solve's work is done
  return res;
}

// Transmits per solved batch when `per` transmits share a frequency: all of
// them, or chunks of tx_chunk (one frequency at a time).
int chunk_of(const fwi_solve_opts& o, int per) { return o.tx_chunk > 0 && o.tx_chunk < per ? o.tx_chunk : per; }
int chunks_of(const fwi_solve_opts& o, int per) {
  const int cs = chunk_of(o, per);
  return (per + cs - 1) / cs;
}

// Groups of whole frequencies solved together: at most max_rhs RHS per batch
// (one frequency per group when the transmits are chunked).
int freqs_per_group(const fwi_problem* p, const fwi_solve_opts& o) {
  if (chunk_of(o, p->ne) < p->ne) return 1;
  if (o.max_rhs <= 0) return p->nf;
  const int f = o.max_rhs / p->ne;
  return f < 1 ? 1 : (f > p->nf ? p->nf : f);
}

// Per-call device buffers of the model and of one frequency group.
struct CallBufs {
  c128* m64 = nullptr;
  c64* m32 = nullptr;
  c128* fields = nullptr;   // [B][n]  (group fields, or all fields for ADMM)
  c128* S = nullptr;        // [B][n]  adjoint sources
  c128* lam = nullptr;      // [B][n]  adjoint fields
  c128* data = nullptr;     // [nf][ne][ne]
  c128* r = nullptr;        // [nf][ne][ne]
  c128* gpart = nullptr;    // [nks][nfg][ne][ne] or [nseg][n]
  long gpart_len = 0;       // elements of gpart
  c128* gacc = nullptr;     // [n]
  double* misfits = nullptr;  // [ngroups * chunks]
  int* rfreq = nullptr;     // [B]
  c128* wtx = nullptr;      // [nf][nt][ne] conjugated transmit weights (nt <= ne; gradient plans)
  // ADMM
  c128 *cg_x = nullptr, *cg_r = nullptr, *cg_p = nullptr, *cg_Ap = nullptr, *vec = nullptr;
  c128 *gm = nullptr, *tmpd = nullptr, *Jp = nullptr;
  c128* fine = nullptr;     // [n] forward-mesh vector of a coarse inversion mesh
  double *dpart = nullptr, *sc = nullptr;
};

constexpr int kGradSeg = 16;

// K-splits of the sampling / Jacobian GEMM over the n grid points: one split
// per 1024 points, at most 64 while the output tiles and frequencies already
// give >= 1024 workgroups, more (up to 512) when they do not (a 3D grid with
// one frequency and 64 x 64 outputs is one tile). gemm_splits_max bounds every
// launch's count (buffer plans).
int gemm_splits_max(long n) {
  const long s = (n + 1023) / 1024;
  return (int)(s < 1 ? 1 : (s > 512 ? 512 : s));
}
int gemm_splits(long n, int nf, int ni, int nj) {
  const long units = (long)nf * ((ni + 63) / 64) * ((nj + 63) / 64);
  const long want = std::max<long>(64, (1024 + units - 1) / units);
  return (int)std::min<long>(gemm_splits_max(n), want);
}

// Plans every buffer of an entry point; `entry` as in fwi_workspace_size.
template <typename T>
void plan_call(Arena& a, const fwi_problem* p, const fwi_solve_opts& o, int entry, CallBufs& cb, SolveBufs<T>& sb,
               int B_override = 0) {
  const Geo g = make_geo(p);
  const long n = g.n();
  const int nfg = freqs_per_group(p, o);
  const int B = B_override > 0 ? B_override : nfg * chunk_of(o, p->ne);
  const int ngroups = (p->nf + nfg - 1) / nfg;
  const long ndata = (long)p->nf * p->ne * p->ne;
  cb.m64 = a.take<c128>(n);
  cb.m32 = a.take<c64>(n);
  cb.rfreq = a.take<int>(B);
  cb.data = a.take<c128>(ndata);
  cb.r = a.take<c128>(ndata);
  cb.misfits = a.take<double>((size_t)ngroups * chunks_of(o, p->ne) + 2);
  const long gp = std::max((long)gemm_splits_max(n) * nfg * p->ne * p->ne, (long)kGradSeg * n);
  cb.gpart_len = std::max(gp, (long)gemm_splits_max(n) * p->nf * p->ne * p->ne);
  cb.gpart = a.take<c128>(cb.gpart_len);
  cb.gacc = a.take<c128>(n);
  if (entry == FWI_ENTRY_ADMM)
    cb.fields = a.take<c128>((size_t)p->nf * p->ne * n);
  else
    cb.fields = a.take<c128>((size_t)B * n);
  if (entry != FWI_ENTRY_FORWARD) {
    cb.S = a.take<c128>((size_t)B * n);
    cb.lam = a.take<c128>((size_t)B * n);
  }
  if (entry != FWI_ENTRY_FORWARD) cb.wtx = a.take<c128>(ndata);
  if (entry == FWI_ENTRY_ADMM) {
    cb.cg_x = a.take<c128>(n);
    cb.cg_r = a.take<c128>(n);
    cb.cg_p = a.take<c128>(n);
    cb.cg_Ap = a.take<c128>(n);
    cb.vec = a.take<c128>(n);
    cb.gm = a.take<c128>((size_t)g.dim * n);
    cb.tmpd = a.take<c128>((size_t)g.dim * n);
    cb.Jp = a.take<c128>(ndata);
    cb.fine = a.take<c128>(n);
    cb.dpart = a.take<double>(std::max(dot_blocks(n), (int)((n + 255) / 256)) + 8);
    cb.sc = a.take<double>(8);
  }
  plan_solve<T>(a, g, B, o.restart, sb);
}

// ---------------------------------------------------------- pipelines ---
struct Runner {
  fwi_ctx* c;
  const fwi_problem* p;
  fwi_solve_opts o;
  Geo g;
  long n;
  int nfg, ngroups;
  CallBufs cb;
  SolveTotals tot;
  double t_setup = 0.0;

  Runner(fwi_ctx* c_, const fwi_problem* p_, const fwi_solve_opts& o_) : c(c_), p(p_), o(o_) {
    g = make_geo(p);
    n = g.n();
    nfg = freqs_per_group(p, o);
    ngroups = (p->nf + nfg - 1) / nfg;
    launch_zero_u64(2, c->d_itstat, c->stream);  // this call's iteration statistics
  }

  // Solve A_l x = rhs for frequencies [l0, l0 + nf), `per` right-hand sides
  // per frequency (frequency-major), into `out`.
  template <typename T>
  void solve_rhs(SolveBufs<T>& sb, int l0, int nf, int per, const c128* rhs, c128* out) {
    const ProblemCache& pc = c->pc;
    const int B = nf * per;
    const cplx<T>* mT = std::is_same<T, float>::value ? (const cplx<T>*)cb.m32 : (const cplx<T>*)cb.m64;
    const cplx<T>* gT = std::is_same<T, float>::value ? (const cplx<T>*)pc.ghat32 : (const cplx<T>*)pc.ghat64;
    launch_fill_rfreq(B, per, l0, cb.rfreq, c->stream);
    // a short batch reuses the planned buffers with a smaller B
    SolveBufs<T> s = sb;
    s.ks.B = B;
    SolveTotals r = run_solve<T>(c, g, cb.m64, mT, pc.ghat64, gT, B, rhs, cb.rfreq, out, o, s, nf);
    tot.merge(r);
  }

  // Fields of one solved batch into the caller's array: complex128 in place
  // (solved there directly) or rounded to complex64.
  c128* field_target(c128* fields_out, long off) { return fields_out && !o.fields_c64 ? fields_out + off : cb.fields; }
  void field_store(c128* fields_out, long off, long count) {
    if (fields_out && o.fields_c64) launch_cast_64_32(count, cb.fields, reinterpret_cast<c64*>(fields_out) + off, c->stream);
  }

  // Transmits synthesised from the elements (Sec. V: steered plane waves;
  // every element receives): transmit t of frequency l drives element e with
  // weight w[l][t][e], so its incident field is sum_e w P0_l[e] and, the
  // problem being linear, its total field solves A_l p = that field. cb.wtx
  // holds conj(w) (the NN product conjugates its left operand). Data
  // [nf][nt][ne] by the point-receiver rule of Eq. 4. Transmits are solved
  // in chunks of tx_chunk when set (one frequency at a time).
  template <typename T>
  void forward_tx(SolveBufs<T>& sb, int nt, c128* data_out, c128* fields_out) {
    const ProblemCache& pc = c->pc;
    hipStream_t st = c->stream;
    const long nd = (long)nt * p->ne;
    const int cs = chunk_of(o, nt);
    for (int gi = 0; gi < ngroups; ++gi) {
      const int l0 = gi * nfg, nf = std::min(nfg, p->nf - l0);
      const c128* P0g = pc.P0 + (long)l0 * p->ne * n;
      for (int t0 = 0; t0 < nt; t0 += cs) {
        const int ti = std::min(cs, nt - t0);  // nf == 1 unless ti == nt
        const long off = ((long)l0 * nt + t0) * n;
        c128* F = field_target(fields_out, off);
        launch_gemm_cn(nf, cb.wtx + l0 * nd + (long)t0 * p->ne, ti, p->ne, P0g, (long)p->ne * n, n, cb.S,
                       (long)ti * n, st);
        solve_rhs<T>(sb, l0, nf, ti, cb.S, F);
        launch_gemm_nt(nf, F, (long)ti * n, ti, cb.m64, P0g, (long)p->ne * n, p->ne, n, pc.coef + l0, cb.gpart,
                       gemm_splits(n, nf, ti, p->ne), data_out + l0 * nd + (long)t0 * p->ne, st);
        field_store(fields_out, off, (long)nf * ti * n);
      }
    }
  }

  // misfit and J^H r for synthesised transmits by adjoint solves: adjoint
  // sources sum_j conj(r_tj) P0_j (the receivers are the elements), adjoint
  // fields by the same operator, g as for element transmits.
  template <typename T>
  double gradient_tx(SolveBufs<T>& sb, int nt, const c128* dobs, c128* data_out, const double* cc,
                     const double* alpha, c128* gm_out, double* gc, double* ga) {
    const ProblemCache& pc = c->pc;
    hipStream_t st = c->stream;
    const long nd = (long)nt * p->ne;
    const int cs = chunk_of(o, nt);
    int seg = 0;
    for (int gi = 0; gi < ngroups; ++gi) {
      const int l0 = gi * nfg, nf = std::min(nfg, p->nf - l0);
      const c128* P0g = pc.P0 + (long)l0 * p->ne * n;
      for (int t0 = 0; t0 < nt; t0 += cs, ++seg) {
        const int ti = std::min(cs, nt - t0);
        const long rows = l0 * nd + (long)t0 * p->ne;  // first data entry of the chunk
        launch_gemm_cn(nf, cb.wtx + rows, ti, p->ne, P0g, (long)p->ne * n, n, cb.S, (long)ti * n, st);
        solve_rhs<T>(sb, l0, nf, ti, cb.S, cb.fields);
        launch_gemm_nt(nf, cb.fields, (long)ti * n, ti, cb.m64, P0g, (long)p->ne * n, p->ne, n, pc.coef + l0,
                       cb.gpart, gemm_splits(n, nf, ti, p->ne), data_out + rows, st);
        launch_residual((long)nf * ti * p->ne, data_out + rows, dobs + rows, cb.r + rows, cb.misfits + seg, st);
        launch_gemm_cn(nf, cb.r + rows, ti, p->ne, P0g, (long)p->ne * n, n, cb.S, (long)ti * n, st);
        solve_rhs<T>(sb, l0, nf, ti, cb.S, cb.lam);
        launch_gradient_accum(n, nf, ti, cb.fields, cb.lam, pc.k2 + l0, cb.gpart, kGradSeg, seg == 0, cb.gacc, st);
      }
    }
    launch_grad_chain(n, cb.gacc, std::pow(g.dx, g.dim), inv_kappa0(g), cc, alpha, gm_out, gc, ga, st);
    return sum_misfits(seg);
  }

  double sum_misfits(int count) {
    std::vector<double> mf(count);
    FWI_HIP(hipMemcpyAsync(mf.data(), cb.misfits, sizeof(double) * count, hipMemcpyDeviceToHost, c->stream));
    FWI_HIP(hipStreamSynchronize(c->stream));
    double phi = 0.0;
    for (double v : mf) phi += v;
    return phi;
  }

  template <typename T>
  void forward(SolveBufs<T>& sb, c128* data_out, c128* fields_out) {
    const ProblemCache& pc = c->pc;
    hipStream_t st = c->stream;
    const long ne2 = (long)p->ne * p->ne;
    const int cs = chunk_of(o, p->ne);
    for (int gi = 0; gi < ngroups; ++gi) {
      const int l0 = gi * nfg, nf = std::min(nfg, p->nf - l0);
      for (int i0 = 0; i0 < p->ne; i0 += cs) {
        const int ni = std::min(cs, p->ne - i0);  // nf == 1 unless ni == ne
        const long off = ((long)l0 * p->ne + i0) * n;
        c128* F = field_target(fields_out, off);
        solve_rhs<T>(sb, l0, nf, ni, pc.P0 + off, F);
        launch_gemm_nt(nf, F, (long)ni * n, ni, cb.m64, pc.P0 + (long)l0 * p->ne * n, (long)p->ne * n, p->ne, n,
                       pc.coef + l0, cb.gpart, gemm_splits(n, nf, ni, p->ne), data_out + l0 * ne2 + (long)i0 * p->ne,
                       st);
        field_store(fields_out, off, (long)nf * ni * n);
      }
    }
  }

  // misfit and J^H r (or J^H b with upstream b) by adjoint solves; the
  // forward fields are solved (in frequency groups and transmit chunks) or,
  // when fields_in is given ([nf][ne][n], from an earlier forward call at the
  // same model), taken from there.
  template <typename T>
  double gradient(SolveBufs<T>& sb, const c128* dobs, const c128* upstream, c128* data_out, const double* cc,
                  const double* alpha, c128* gm_out, double* gc, double* ga, const c128* fields_in = nullptr) {
    const ProblemCache& pc = c->pc;
    hipStream_t st = c->stream;
    const long ne2 = (long)p->ne * p->ne;
    const int cs = chunk_of(o, p->ne);
    int seg = 0;
    for (int gi = 0; gi < ngroups; ++gi) {
      const int l0 = gi * nfg, nf = std::min(nfg, p->nf - l0);
      const c128* P0g = pc.P0 + (long)l0 * p->ne * n;
      for (int i0 = 0; i0 < p->ne; i0 += cs, ++seg) {
        const int ni = std::min(cs, p->ne - i0);
        const long off = ((long)l0 * p->ne + i0) * n;
        const long rows = l0 * ne2 + (long)i0 * p->ne;  // first data entry of the chunk
        const c128* F = cb.fields;
        if (fields_in) {
          F = fields_in + off;
        } else {
          solve_rhs<T>(sb, l0, nf, ni, P0g + (long)i0 * n, cb.fields);
        }
        const c128* rg;
        if (upstream) {
          rg = upstream + rows;
        } else {
          launch_gemm_nt(nf, F, (long)ni * n, ni, cb.m64, P0g, (long)p->ne * n, p->ne, n, pc.coef + l0, cb.gpart,
                         gemm_splits(n, nf, ni, p->ne), data_out + rows, st);
          launch_residual((long)nf * ni * p->ne, data_out + rows, dobs + rows, cb.r + rows, cb.misfits + seg, st);
          rg = cb.r + rows;
        }
        if (o.reciprocity_adjoint) {  // whole frequencies only (checked by the entry)
          launch_gemm_cn(nf, rg, p->ne, p->ne, F, (long)p->ne * n, n, cb.lam, (long)p->ne * n, st);
        } else {
          launch_gemm_cn(nf, rg, ni, p->ne, P0g, (long)p->ne * n, n, cb.S, (long)ni * n, st);
          solve_rhs<T>(sb, l0, nf, ni, cb.S, cb.lam);
        }
        launch_gradient_accum(n, nf, ni, F, cb.lam, pc.k2 + l0, cb.gpart, kGradSeg, seg == 0, cb.gacc, st);
      }
    }
    launch_grad_chain(n, cb.gacc, std::pow(g.dx, g.dim), inv_kappa0(g), cc, alpha, gm_out, gc, ga, st);
    return upstream ? 0.0 : sum_misfits(seg);
  }
};

// Adds the iteration statistics the call's solves left on the device (waits
// for the stream).
void collect_iters(fwi_ctx* c, SolveTotals& t) {
  FWI_HIP(hipMemcpyAsync(c->h_dbl + 8, c->d_itstat, 2 * sizeof(unsigned long long), hipMemcpyDeviceToHost,
                         c->stream));
  FWI_HIP(hipStreamSynchronize(c->stream));
  unsigned long long v[2];
  std::memcpy(v, c->h_dbl + 8, sizeof(v));
  t.iters_max = std::max(t.iters_max, (int)v[0]);
  t.matvecs += (long long)v[1];
}

void fill_stats(fwi_stats* s, const SolveTotals& t, double t_setup, double t_total) {
  if (!s) return;
  s->iterations = t.iters_max;
  s->cycles = t.cycles;
  s->unconverged = t.unconverged;
  s->max_rel_residual = t.maxrel;
  s->solves = t.solves;
  s->matvecs = t.matvecs;
  s->t_setup_ms = t_setup;
  s->t_solve_ms = t.t_solve;
  s->t_total_ms = t_total;
}

void check_sos(fwi_ctx* c, long n, const double* cc, const double* alpha) {
  launch_check_sos(n, cc, alpha, c->d_int, c->stream);
  FWI_HIP(hipMemcpyAsync(c->h_int, c->d_int, 2 * sizeof(int), hipMemcpyDeviceToHost, c->stream));
  FWI_HIP(hipStreamSynchronize(c->stream));
  if (c->h_int[0] || c->h_int[1])
    throw Error(FWI_E_NONFINITE, "speed of sound must be finite and > 0, attenuation finite and >= 0");
}
void check_complex(fwi_ctx* c, long n, const c128* x, const char* what) {
  launch_check_complex(n, x, c->d_int, c->stream);
  FWI_HIP(hipMemcpyAsync(c->h_int, c->d_int, sizeof(int), hipMemcpyDeviceToHost, c->stream));
  FWI_HIP(hipStreamSynchronize(c->stream));
  if (c->h_int[0]) throw Error(FWI_E_NONFINITE, std::string("non-finite values in ") + what);
}

template <typename F>
int guarded(fwi_ctx* c, F&& body) {
  if (!c) return FWI_E_INVAL;
  struct Scope {
    Scope(fwi_ctx* c) {
      tl_prof = c->prof.mask ? &c->prof : nullptr;
      tl_tune = &c->tune;
      tl_force_variant = -1;
      tl_force_wide = c->force_wide;
      tl_xy_off = c->xy_off;
      tl_active = 0;
      tl_nfreq = 0;
    }
    ~Scope() {
      tl_prof = nullptr;
      tl_ev_start = tl_ev_stop = nullptr;
      tl_ev_used = false;
      tl_tune = nullptr;
      tl_force_variant = -1;
      tl_force_wide = 0;
      tl_xy_off = 0;
    }
  } scope(c);
  try {
    FWI_HIP(hipSetDevice(c->device));
    const int rc = body();
    if (c->prof.mask) c->prof.flush();
    return rc;
  } catch (const Error& e) {
    c->err = e.what();
    c->prof.recs.clear();
    c->prof.used = 0;
    return e.code;
  } catch (const std::exception& e) {
    c->err = e.what();
    c->prof.recs.clear();
    c->prof.used = 0;
    return FWI_E_DEVICE;
  }
}

template <typename T>
size_t plan_bytes(const fwi_problem* p, const fwi_solve_opts& o, int entry) {
  Arena a;
  CallBufs cb;
  SolveBufs<T> sb;
  plan_call<T>(a, p, o, entry, cb, sb);
  return a.used;
}

// Prepare: validate, cache, bind workspace and plan buffers.
template <typename T>
void prepare(fwi_ctx* c, Runner& R, SolveBufs<T>& sb, int entry, int B_override = 0) {
  std::string msg;
  int rc = validate_problem(R.p, msg);
  if (rc) throw Error(rc, msg);
  rc = validate_opts(&R.o, msg);
  if (rc) throw Error(rc, msg);
  R.t_setup += ensure_cache(c, R.p);
  Arena dry;
  CallBufs cbd;
  SolveBufs<T> sbd;
  plan_call<T>(dry, R.p, R.o, entry, cbd, sbd, B_override);
  Arena a;
  bind_workspace(c, a, dry.used);
  plan_call<T>(a, R.p, R.o, entry, R.cb, sb, B_override);
}

int finish_rc(const SolveTotals& t) { return t.unconverged ? FWI_E_NOCONV : FWI_OK; }

// ----------------------------------------------------------- entries ---
template <typename T>
int forward_impl(fwi_ctx* c, const fwi_problem* p, const double* cc, const double* alpha, const void* m_in,
                 const fwi_solve_opts* opts, void* data_out, void* fields_out, fwi_stats* stats) {
  const double t0 = now_ms();
  if (!data_out || (!m_in && !cc)) throw Error(FWI_E_INVAL, "NULL array argument");
  Runner R(c, p, *opts);
  SolveBufs<T> sb;
  prepare<T>(c, R, sb, FWI_ENTRY_FORWARD);
  const double ts = now_ms();
  if (m_in) {
    check_complex(c, R.n, (const c128*)m_in, "m");
    launch_copy_c128(R.n, (const c128*)m_in, R.cb.m64, c->stream);
    launch_cast_64_32(R.n, R.cb.m64, R.cb.m32, c->stream);
  } else {
    check_sos(c, R.n, cc, alpha);
    launch_contrast(R.n, p->c0, p->alpha0, cc, alpha, R.cb.m64, R.cb.m32, c->stream);
  }
  R.t_setup += now_ms() - ts;
  R.forward<T>(sb, (c128*)data_out, (c128*)fields_out);
  FWI_HIP(hipStreamSynchronize(c->stream));
  collect_iters(c, R.tot);
  fill_stats(stats, R.tot, R.t_setup, now_ms() - t0);
  return finish_rc(R.tot);
}

template <typename T>
int gradient_impl(fwi_ctx* c, const fwi_problem* p, const double* cc, const double* alpha, const void* m_in,
                  const void* dobs, const void* upstream, const fwi_solve_opts* opts, double* misfit_out,
                  void* grad_m_out, double* gc, double* ga, fwi_stats* stats, const void* fields_in = nullptr) {
  const double t0 = now_ms();
  if ((!m_in && !cc) || (!dobs && !upstream)) throw Error(FWI_E_INVAL, "NULL array argument");
  if (opts->reciprocity_adjoint && p && chunk_of(*opts, p->ne) < p->ne)
    throw Error(FWI_E_UNSUPPORTED, "the reciprocity adjoint needs whole frequencies (tx_chunk 0 or >= ne)");
  Runner R(c, p, *opts);
  SolveBufs<T> sb;
  prepare<T>(c, R, sb, FWI_ENTRY_GRADIENT);
  const double ts = now_ms();
  if (m_in) {
    check_complex(c, R.n, (const c128*)m_in, "m");
    launch_copy_c128(R.n, (const c128*)m_in, R.cb.m64, c->stream);
    launch_cast_64_32(R.n, R.cb.m64, R.cb.m32, c->stream);
  } else {
    check_sos(c, R.n, cc, alpha);
    launch_contrast(R.n, p->c0, p->alpha0, cc, alpha, R.cb.m64, R.cb.m32, c->stream);
  }
  R.t_setup += now_ms() - ts;
  const double phi = R.gradient<T>(sb, (const c128*)dobs, (const c128*)upstream, R.cb.data, cc, alpha,
                                   (c128*)grad_m_out, gc, ga, (const c128*)fields_in);
  FWI_HIP(hipStreamSynchronize(c->stream));
  if (misfit_out) *misfit_out = phi;
  collect_iters(c, R.tot);
  fill_stats(stats, R.tot, R.t_setup, now_ms() - t0);
  return finish_rc(R.tot);
}

// Synthesised transmits: nt in [1, ne] transmits per frequency with weights
// w [nf][nt][ne] (device); planned as the gradient entry (adjoint-source
// buffer for the synthesised incident fields, room for the weights).
template <typename T>
void prepare_tx(fwi_ctx* c, Runner& R, SolveBufs<T>& sb, int nt, const void* w, const double* cc,
                const double* alpha) {
  if (!cc || !w) throw Error(FWI_E_INVAL, "NULL array argument");
  if (nt < 1 || nt > R.p->ne) throw Error(FWI_E_INVAL, "need 1 <= nt <= ne synthesised transmits");
  prepare<T>(c, R, sb, FWI_ENTRY_GRADIENT);
  const long nw = (long)R.p->nf * nt * R.p->ne;
  check_complex(c, nw, (const c128*)w, "transmit weights");
  launch_conj_c128(nw, (const c128*)w, R.cb.wtx, c->stream);
  const double ts = now_ms();
  check_sos(c, R.n, cc, alpha);
  launch_contrast(R.n, R.p->c0, R.p->alpha0, cc, alpha, R.cb.m64, R.cb.m32, c->stream);
  R.t_setup += now_ms() - ts;
}

template <typename T>
int forward_tx_impl(fwi_ctx* c, const fwi_problem* p, const double* cc, const double* alpha, int nt, const void* w,
                    const fwi_solve_opts* opts, void* data_out, void* fields_out, fwi_stats* stats) {
  const double t0 = now_ms();
  if (!data_out) throw Error(FWI_E_INVAL, "NULL array argument");
  Runner R(c, p, *opts);
  SolveBufs<T> sb;
  prepare_tx<T>(c, R, sb, nt, w, cc, alpha);
  R.forward_tx<T>(sb, nt, (c128*)data_out, (c128*)fields_out);
  FWI_HIP(hipStreamSynchronize(c->stream));
  collect_iters(c, R.tot);
  fill_stats(stats, R.tot, R.t_setup, now_ms() - t0);
  return finish_rc(R.tot);
}

template <typename T>
int gradient_tx_impl(fwi_ctx* c, const fwi_problem* p, const double* cc, const double* alpha, int nt, const void* w,
                     const void* dobs, const fwi_solve_opts* opts, double* misfit_out, void* grad_m_out, double* gc,
                     double* ga, fwi_stats* stats) {
  const double t0 = now_ms();
  if (!dobs) throw Error(FWI_E_INVAL, "NULL array argument");
  if (opts->reciprocity_adjoint)
    throw Error(FWI_E_UNSUPPORTED, "reciprocity adjoint needs transmit set = receive set");
  Runner R(c, p, *opts);
  SolveBufs<T> sb;
  prepare_tx<T>(c, R, sb, nt, w, cc, alpha);
  const double phi = R.gradient_tx<T>(sb, nt, (const c128*)dobs, R.cb.data, cc, alpha, (c128*)grad_m_out, gc, ga);
  if (misfit_out) *misfit_out = phi;
  collect_iters(c, R.tot);
  fill_stats(stats, R.tot, R.t_setup, now_ms() - t0);
  return finish_rc(R.tot);
}

// J^H b over all frequency groups from stored transmit fields tx [nf][nt][n]
// and receiver fields rx [nf][ne][n] (the same array for element transmits,
// nt = ne), b [nf][nt][ne] -> out [n] (times dV)
void jh_apply(fwi_ctx* c, const fwi_problem* p, const Geo& g, CallBufs& cb, int nfg, int nt, const c128* tx,
              const c128* rx, const c128* b, c128* out) {
  const ProblemCache& pc = c->pc;
  const long n = g.n(), nd = (long)nt * p->ne;
  const int ngroups = (p->nf + nfg - 1) / nfg;
  for (int gi = 0; gi < ngroups; ++gi) {
    const int l0 = gi * nfg, nf = std::min(nfg, p->nf - l0);
    const int nseg = gemm_cn_grad_segments(nf, nt);
    if ((long)nseg * n <= cb.gpart_len) {
      // the products with the transmit fields formed in the GEMM's epilogue
      launch_gemm_cn_grad(nf, b + l0 * nd, nt, p->ne, rx + (long)l0 * p->ne * n, (long)p->ne * n, n,
                          tx + (long)l0 * nt * n, (long)nt * n, pc.k2 + l0, cb.gpart, c->stream);
      launch_grad_sum(n, cb.gpart, nseg, gi == 0, cb.gacc, c->stream);
    } else {
      launch_gemm_cn(nf, b + l0 * nd, nt, p->ne, rx + (long)l0 * p->ne * n, (long)p->ne * n, n, cb.lam, (long)nt * n,
                     c->stream);
      launch_gradient_accum(n, nf, nt, tx + (long)l0 * nt * n, cb.lam, pc.k2 + l0, cb.gpart, kGradSeg, gi == 0,
                            cb.gacc, c->stream);
    }
  }
  launch_grad_chain(n, cb.gacc, std::pow(g.dx, g.dim), inv_kappa0(g), nullptr, nullptr, out, nullptr, nullptr, c->stream);
}

// J a from stored transmit and receiver fields -> out [nf][nt][ne]
void j_apply(fwi_ctx* c, const fwi_problem* p, const Geo& g, CallBufs& cb, int nt, const c128* tx, const c128* rx,
             const c128* a, c128* out) {
  const long n = g.n();
  launch_gemm_nt(p->nf, tx, (long)nt * n, nt, a, rx, (long)p->ne * n, p->ne, n, c->pc.coef, cb.gpart,
                 gemm_splits(n, p->nf, nt, p->ne),
                 out, c->stream);
}

// Inversion mesh r times coarser than the forward mesh (ceil per axis).
Geo coarse_geo(const Geo& g, int r) {
  Geo c = g;
  if (r > 1) {
    c.nx = (g.nx + r - 1) / r;
    c.ny = g.dim == 3 ? (g.ny + r - 1) / r : 1;
    c.nz = (g.nz + r - 1) / r;
  }
  return c;
}
// Receiver fields of the Jacobian: the forward fields for element transmits.
inline const c128* rxf_of(const CallBufs& cb, const c128* rx, bool tx) { return tx ? rx : cb.fields; }

// One ADMM iteration. nt = 0: element transmits (the Jacobian from the
// forward fields alone). nt > 0: synthesised transmits with weights w
// [nf][nt][ne] and receiver fields rx [nf][ne][n], recomputed at m_k when
// refresh_rx is set and used as given otherwise (Born reuse, Sec. IV-B).
template <typename T>
int admm_impl(fwi_ctx* c, const fwi_problem* p, const fwi_admm_params* prm, void* m_io, void* g_io, void* u_io,
              const void* m_ref, const void* dobs_v, const fwi_solve_opts* opts, fwi_admm_report* rep,
              fwi_stats* stats, int nt = 0, const void* w = nullptr, c128* rx = nullptr, int refresh_rx = 1,
              double* half_dobs2 = nullptr) {
  const double t0 = now_ms();
  if (!prm || !m_io || !g_io || !u_io || !dobs_v) throw Error(FWI_E_INVAL, "NULL argument");
  if (!(prm->rho > 0.0) || prm->lambda < 0.0 || prm->gamma < 0.0 || prm->n_cg < 0)
    throw Error(FWI_E_INVAL, "ADMM parameters: need rho > 0, lambda >= 0, gamma >= 0, n_cg >= 0");
  const bool tx = nt > 0;
  if (tx && (!w || !rx)) throw Error(FWI_E_INVAL, "NULL transmit weights or receiver fields");
  if (tx && nt > p->ne) throw Error(FWI_E_INVAL, "need 1 <= nt <= ne synthesised transmits");
  Runner R(c, p, *opts);
  R.o.fields_c64 = 0;  // the Jacobian keeps complex128 fields
  SolveBufs<T> sb;
  prepare<T>(c, R, sb, FWI_ENTRY_ADMM);
  hipStream_t st = c->stream;
  const int ntx = tx ? nt : p->ne;
  const long ndata = (long)p->nf * ntx * p->ne;
  const Geo& g = R.g;
  // inversion mesh: the forward mesh, or r times coarser (piecewise-constant
  // model, Jacobian J P, TV on the coarse cells)
  const int rf = prm->inv_factor > 1 ? prm->inv_factor : 1;
  const Geo gc = coarse_geo(g, rf);
  const long n = gc.n();
  CallBufs& cb = R.cb;
  c128* m = (c128*)m_io;
  c128* gg = (c128*)g_io;
  c128* uu = (c128*)u_io;
  const c128* dobs = (const c128*)dobs_v;
  const c128* mref = (const c128*)m_ref;
  const bool use_ref = mref && prm->gamma != 0.0;
  check_complex(c, n, m, "m");
  if (rf > 1) launch_prolong(g, rf, m, cb.m64, st);
  else launch_copy_c128(n, m, cb.m64, st);
  launch_cast_64_32(R.n, cb.m64, cb.m32, st);
  // J^H b and J a on the inversion mesh
  auto jh = [&](const c128* b, c128* out) {
    if (rf > 1) {
      jh_apply(c, p, g, cb, R.nfg, ntx, cb.fields, rxf_of(cb, rx, tx), b, cb.fine);
      launch_restrict(g, rf, cb.fine, out, st);
    } else {
      jh_apply(c, p, g, cb, R.nfg, ntx, cb.fields, rxf_of(cb, rx, tx), b, out);
    }
  };
  auto jv = [&](const c128* a, c128* out) {
    if (rf > 1) {
      launch_prolong(g, rf, a, cb.fine, st);
      a = cb.fine;
    }
    j_apply(c, p, g, cb, ntx, cb.fields, rxf_of(cb, rx, tx), a, out);
  };
  // 1. forward solves at m_k, all fields kept for the Jacobian products
  if (tx) {
    const long nw = (long)p->nf * nt * p->ne;
    check_complex(c, nw, (const c128*)w, "transmit weights");
    launch_conj_c128(nw, (const c128*)w, cb.wtx, st);
    R.forward_tx<T>(sb, nt, cb.data, cb.fields);
    if (refresh_rx) R.forward<T>(sb, cb.Jp, rx);  // receiver fields at m_k (data not used)
  } else {
    R.forward<T>(sb, cb.data, cb.fields);
  }
  // 2. residual d_obs - F and data scale
  launch_residual(ndata, cb.data, dobs, cb.r, cb.sc + 4, st);   // r = F - d_obs, sc[4] = misfit
  launch_residual(ndata, dobs, nullptr, cb.Jp, cb.sc + 5, st);  // sc[5] = |d_obs|^2 / 2
  FWI_HIP(hipMemcpyAsync(c->h_dbl, cb.sc + 4, 2 * sizeof(double), hipMemcpyDeviceToHost, st));
  FWI_HIP(hipStreamSynchronize(st));
  const double misfit = c->h_dbl[0];
  if (half_dobs2) *half_dobs2 = c->h_dbl[1];
  double s = prm->data_scale;
  if (!(s > 0.0)) s = c->h_dbl[1] > 0.0 ? 1.0 / (2.0 * c->h_dbl[1]) : 1.0;
  const double rho = prm->rho, gam = use_ref ? prm->gamma : 0.0;
  const double dual = prm->dual_step;
  // 3. b = -s J^H(F - d) + rho grad^T(g + u - grad m) + gamma (m_ref - m)
  jh(cb.r, cb.vec);
  launch_tv_grad(gc, m, cb.gm, st);
  launch_lincomb((long)gc.dim * n, 1.0, gg, 1.0, uu, -1.0, cb.gm, cb.tmpd, st);
  launch_tv_gradT(gc, cb.tmpd, rho, 0.0, cb.cg_r, st);
  launch_lincomb(n, 1.0, cb.cg_r, -s, cb.vec, 0.0, nullptr, cb.cg_r, st);
  if (use_ref) launch_lincomb(n, 1.0, cb.cg_r, gam, mref, -gam, m, cb.cg_r, st);
  // 4. CG on (s J^H J + rho grad^T grad + gamma I) dm = b from dm = 0
  launch_fill_zero_c128(n, cb.cg_x, st);
  launch_copy_c128(n, cb.cg_r, cb.cg_p, st);
  launch_dot_re(n, cb.cg_r, cb.cg_r, cb.dpart, cb.sc + 0, st);
  for (int it = 0; it < prm->n_cg; ++it) {
    jv(cb.cg_p, cb.Jp);
    jh(cb.Jp, cb.vec);
    launch_tv_grad(gc, cb.cg_p, cb.tmpd, st);
    launch_tv_gradT(gc, cb.tmpd, rho, 0.0, cb.cg_Ap, st);
    launch_lincomb(n, 1.0, cb.cg_Ap, s, cb.vec, gam, use_ref ? cb.cg_p : nullptr, cb.cg_Ap, st);
    launch_dot_re(n, cb.cg_p, cb.cg_Ap, cb.dpart, cb.sc + 1, st);
    launch_cg_step1(n, cb.sc, cb.cg_x, cb.cg_r, cb.cg_p, cb.cg_Ap, st);
    launch_dot_re(n, cb.cg_r, cb.cg_r, cb.dpart, cb.sc + 2, st);
    launch_cg_step2(n, cb.sc, cb.cg_r, cb.cg_p, st);
    launch_copy_scalar(cb.sc + 2, cb.sc + 0, st);
  }
  // 5. m += dm; g = shrink(grad m - u); u += dual (g - grad m)
  launch_lincomb(n, 1.0, m, 1.0, cb.cg_x, 0.0, nullptr, m, st);
  launch_tv_grad(gc, m, cb.gm, st);
  const int nb = launch_tv_shrink_dual(gc, cb.gm, prm->lambda / rho, dual, gg, uu, cb.dpart, st);
  launch_sum(nb, cb.dpart, cb.sc + 6, st);
  launch_dot_re(n, cb.cg_x, cb.cg_x, cb.dpart, cb.sc + 7, st);
  FWI_HIP(hipMemcpyAsync(c->h_dbl, cb.sc + 6, 2 * sizeof(double), hipMemcpyDeviceToHost, st));
  FWI_HIP(hipStreamSynchronize(st));
  if (rep) {
    rep->misfit = misfit;
    rep->tv = c->h_dbl[0];
    rep->dm_norm = std::sqrt(c->h_dbl[1]);
  }
  collect_iters(c, R.tot);
  fill_stats(stats, R.tot, R.t_setup, now_ms() - t0);
  return finish_rc(R.tot);
}


// ------------------------------------------------------- uneven batches ---
// Many independent problems (different grids, element and frequency counts)
// solved together: one refinement cycle of every instance of a wave is
// captured into one hipGraph (one branch per instance, convergence masks
// instead of host checks inside the cycle) and replayed until every RHS of
// every instance has converged. Instances are grouped into waves that fit a
// memory budget.
template <typename T>
struct BatchInst {
  const fwi_problem* p = nullptr;
  Geo g;
  ProblemCache* pc = nullptr;
  int B = 0;
  long n = 0;
  size_t bytes = 0;
  CallBufs cb;
  SolveBufs<T> sb;
  hipStream_t st = nullptr;
  hipEvent_t join = nullptr;
  const double* c = nullptr;
  const double* alpha = nullptr;
  const c128* dobs = nullptr;
  c128* grad = nullptr;
  c128* data_out = nullptr;
};

// Parts of a cycle, captured as separate graphs so that the host can skip
// the second half of the steps once every RHS of the wave has stopped.
enum CyclePart { CP_HEAD = 0, CP_REST = 1, CP_FINISH = 2 };
inline int head_steps(int JM) { return JM / 2; }

// CP_HEAD: cycle start (first-cycle start pass, or FP64 residual), norms,
// cycle init and the first JM/2 Arnoldi steps; CP_REST: the remaining steps
// and the solution update; CP_FINISH: the solution update only.
template <typename T>
void enqueue_cycle(fwi_ctx* c, BatchInst<T>& I, const c128* rhs, c128* x, int cyc, int part, const fwi_solve_opts& o,
                   hipStream_t st) {
  const bool fp32 = std::is_same<T, float>::value;
  KrylovState<T>& ks = I.sb.ks;
  SolveBufs<T>& s = I.sb;
  const ProblemCache& pc = *I.pc;
  const cplx<T>* mT = fp32 ? (const cplx<T>*)I.cb.m32 : (const cplx<T>*)I.cb.m64;
  const cplx<T>* gT = fp32 ? (const cplx<T>*)pc.ghat32 : (const cplx<T>*)pc.ghat64;
  ArnoldiDriver<T> drv{I.g, c->tw, ks, s, mT, gT, pc.rhs_freq, st, ks.B};
  const int s1 = head_steps(ks.JM);
  if (part == CP_HEAD) {
    if (cyc == 0) {
      const StartIn si{rhs, s.rowpart};  // first pass of the first step included
      launch_vie_rows<T>(I.g, c->tw, ks.B, ks.V, nullptr, mT, s.U1, st, nullptr, nullptr, &si, s.U2);
      krylov_rows_norm(ks, s.rowpart, I.g.nz * I.g.ny, st);
    } else {
      launch_residual_basis(I.g, c->tw, ks.B, x, I.cb.m64, pc.ghat64, pc.rhs_freq, s, rhs, st);
      krylov_rows_norm(ks, s.rowpart, I.g.nz * I.g.ny, st);
    }
    krylov_cycle_init(ks, cyc == 0, o.rtol, fp32 ? o.inner_rtol : 0.0, st);
    if (cyc > 0) drv.first_rows();
  }
  // the steps of this part, masked once an RHS has converged
  const int j0 = part == CP_HEAD ? 0 : s1, j1 = part == CP_HEAD ? s1 : part == CP_REST ? ks.JM : s1;
  for (int j = j0; j < j1; ++j) {
    drv.tail(j);
    drv.orth_givens(j, j + 1 < ks.JM);
  }
  if (part != CP_HEAD) krylov_finish_cycle(ks, x, cyc == 0, st);
}

template <typename T, class RhsOf, class XOf>
hipGraphExec_t capture_cycle(fwi_ctx* c, std::vector<BatchInst<T>*>& wave, int cyc, int part,
                             const fwi_solve_opts& o, RhsOf&& rhs_of, XOf&& x_of) {
  hipStream_t main = c->cap_stream;
  FWI_HIP(hipStreamBeginCapture(main, hipStreamCaptureModeThreadLocal));
  try {
    FWI_HIP(hipEventRecord(c->fork_ev, main));
    for (BatchInst<T>* I : wave) {
      FWI_HIP(hipStreamWaitEvent(I->st, c->fork_ev, 0));
      enqueue_cycle<T>(c, *I, rhs_of(*I), x_of(*I), cyc, part, o, I->st);
      FWI_HIP(hipEventRecord(I->join, I->st));
      FWI_HIP(hipStreamWaitEvent(main, I->join, 0));
    }
  } catch (...) {
    hipGraph_t g = nullptr;
    (void)hipStreamEndCapture(main, &g);
    if (g) (void)hipGraphDestroy(g);
    throw;
  }
  hipGraph_t graph = nullptr;
  FWI_HIP(hipStreamEndCapture(main, &graph));
  hipGraphExec_t exec = nullptr;
  const hipError_t e = hipGraphInstantiate(&exec, graph, nullptr, nullptr, 0);
  (void)hipGraphDestroy(graph);
  FWI_HIP(e);
  return exec;
}

struct BatchTotals {
  int graph_launches = 0, iters = 0, unconverged = 0, waves = 0;
  double maxrel = 0.0, t_solve = 0.0;
  long long solves = 0;
};

// Solve every instance of the wave for rhs_of(I) into x_of(I).
template <typename T, class RhsOf, class XOf>
void batch_solve(fwi_ctx* c, std::vector<BatchInst<T>*>& wave, int* ctr_dev, const fwi_solve_opts& o,
                 RhsOf&& rhs_of, XOf&& x_of, BatchTotals& tot) {
  hipStream_t main = c->cap_stream;
  const bool fp32 = std::is_same<T, float>::value;
  const int max_cycles = fp32 ? o.max_refine : (o.max_iter + o.restart - 1) / o.restart + 1;
  const double t0 = now_ms();
  for (BatchInst<T>* I : wave) krylov_reset_iters(I->sb.ks, main);  // x is written by the first cycle
  // graphs per (first cycle or later, part), captured when first needed
  hipGraphExec_t gx[2][3] = {};
  auto graph = [&](int cyc, int part) {
    hipGraphExec_t& e = gx[cyc == 0 ? 0 : 1][part];
    if (!e) e = capture_cycle<T>(c, wave, cyc == 0 ? 0 : 1, part, o, rhs_of, x_of);
    return e;
  };
  auto destroy = [&]() {
    for (auto& row : gx)
      for (hipGraphExec_t& e : row)
        if (e) {
          (void)hipGraphExecDestroy(e);
          e = nullptr;
        }
  };
  try {
    const int W = (int)wave.size();
    std::vector<int> ctr(2 * W);
    for (int cyc = 0;; ++cyc) {
      // cycle start and the first half of the steps, then the host reads the
      // counts at the cycle start and after those steps
      FWI_HIP(hipGraphLaunch(graph(cyc, CP_HEAD), main));
      tot.graph_launches += 1;
      FWI_HIP(hipMemcpyAsync(ctr.data(), ctr_dev, sizeof(int) * 2 * W, hipMemcpyDeviceToHost, main));
      FWI_HIP(hipStreamSynchronize(main));
      int active = 0, still = 0;
      for (int i = 0; i < W; ++i) {
        active += ctr[2 * i + 1];  // RHS active at the start of this cycle
        still += ctr[2 * i];       // RHS active after the first half of the steps
      }
      if (active == 0) break;
      // the rest of the steps only while some RHS is still active
      FWI_HIP(hipGraphLaunch(graph(cyc, still > 0 ? CP_REST : CP_FINISH), main));
      tot.graph_launches += 1;
      if (cyc >= max_cycles) {
        tot.unconverged += active;
        break;
      }
    }
  } catch (...) {
    (void)hipStreamSynchronize(main);  // no graph is destroyed while it may still run
    destroy();
    throw;
  }
  FWI_HIP(hipStreamSynchronize(main));
  destroy();
  for (BatchInst<T>* I : wave) {
    std::vector<int> it(I->B);
    double mr = 0.0;
    FWI_HIP(hipMemcpyAsync(it.data(), I->sb.ks.iters, sizeof(int) * I->B, hipMemcpyDeviceToHost, main));
    FWI_HIP(hipMemcpyAsync(&mr, I->sb.ks.maxrel, sizeof(double), hipMemcpyDeviceToHost, main));
    FWI_HIP(hipStreamSynchronize(main));
    for (int v : it) tot.iters = std::max(tot.iters, v);
    if (!std::isfinite(mr)) throw Error(FWI_E_NONFINITE, "non-finite residual in a batched solve");
    tot.maxrel = std::max(tot.maxrel, mr);
    tot.solves += I->B;
  }
  tot.t_solve += now_ms() - t0;
}

template <typename T>
int batch_impl(fwi_ctx* c, int ninst, const fwi_problem* probs, const double* const* cc, const double* const* alpha,
               const void* const* dobs, const fwi_solve_opts* opts, double* misfit_out, void* const* grad_out,
               void* const* data_out, fwi_batch_stats* stats) {
  const double t0 = now_ms();
  tl_prof = nullptr;  // no event records inside captured graphs
  if (ninst < 1 || !probs || !cc || !opts) throw Error(FWI_E_INVAL, "bad batch arguments");
  const bool gradient = dobs != nullptr;
  if (gradient && !grad_out && !misfit_out) throw Error(FWI_E_INVAL, "no batch outputs");
  if (!gradient && !data_out) throw Error(FWI_E_INVAL, "no batch outputs");
  std::string msg;
  int rc = validate_opts(opts, msg);
  if (rc) throw Error(rc, msg);
  fwi_solve_opts o = *opts;
  o.max_rhs = 0;               // every instance solves all its frequencies at once
  o.reciprocity_adjoint = 0;
  // caches and plans
  double t_setup = 0.0;
  std::vector<BatchInst<T>> inst(ninst);
  std::set<std::string> keys;
  for (int i = 0; i < ninst; ++i) {
    rc = validate_problem(&probs[i], msg);
    if (rc) throw Error(rc, "instance " + std::to_string(i) + ": " + msg);
    if (!cc[i]) throw Error(FWI_E_INVAL, "instance " + std::to_string(i) + ": c is NULL");
    if (gradient && !dobs[i]) throw Error(FWI_E_INVAL, "instance " + std::to_string(i) + ": d_obs is NULL");
    if (!gradient && !data_out[i]) throw Error(FWI_E_INVAL, "instance " + std::to_string(i) + ": no output");
    const std::string key = problem_key(&probs[i]);
    keys.insert(key);
    ProblemCache& pc = c->bcache[key];
    if (pc.key != key) t_setup += build_cache(c, &probs[i], pc, key);
    BatchInst<T>& I = inst[i];
    I.p = &probs[i];
    I.g = make_geo(&probs[i]);
    I.pc = &pc;
    I.B = probs[i].nf * probs[i].ne;
    I.n = I.g.n();
    I.c = cc[i];
    I.alpha = alpha ? alpha[i] : nullptr;
    I.dobs = gradient ? (const c128*)dobs[i] : nullptr;
    I.grad = grad_out ? (c128*)grad_out[i] : nullptr;
    I.data_out = data_out ? (c128*)data_out[i] : nullptr;
    Arena dry;
    plan_call<T>(dry, I.p, o, FWI_ENTRY_GRADIENT, I.cb, I.sb);
    I.bytes = dry.used;
  }
  for (auto it = c->bcache.begin(); it != c->bcache.end();) {  // drop caches of earlier batches
    if (!keys.count(it->first)) {
      it->second.release();
      it = c->bcache.erase(it);
    } else {
      ++it;
    }
  }
  // waves under a memory budget (60% of free device memory after the caches);
  // if the workspace still cannot be allocated, the budget is halved until
  // every wave holds one instance
  size_t free_b = 0, total_b = 0;
  FWI_HIP(hipMemGetInfo(&free_b, &total_b));
  size_t budget = std::max<size_t>((size_t)(0.6 * (double)(free_b + c->ws_int_bytes)), 1);
  std::vector<std::vector<int>> waves;
  size_t maxw = 0, maxn = 0;
  Arena a;
  for (;;) {
    waves.clear();
    size_t cur = 0;
    for (int i = 0; i < ninst; ++i) {
      if (waves.empty() || cur + inst[i].bytes > budget) {
        waves.emplace_back();
        cur = 0;
      }
      waves.back().push_back(i);
      cur += inst[i].bytes;
    }
    maxw = 0;
    maxn = 0;
    for (auto& w : waves) {
      Arena d;  // the wave's counters, then each instance's buffers
      d.take<int>(2 * w.size());
      size_t sum = d.used;
      for (int i : w) sum += inst[i].bytes;
      maxw = std::max(maxw, sum);
      maxn = std::max(maxn, w.size());
    }
    try {
      bind_workspace(c, a, maxw);
      break;
    } catch (const Error& e) {
      if (e.code != FWI_E_NOMEM || c->ws_ext || maxn <= 1) throw;
      budget = maxw / 2;
    }
  }
  // streams and events
  if (!c->cap_stream) FWI_HIP(hipStreamCreateWithFlags(&c->cap_stream, hipStreamNonBlocking));
  if (!c->fork_ev) FWI_HIP(hipEventCreateWithFlags(&c->fork_ev, hipEventDisableTiming));
  while (c->branch.size() < maxn) {
    hipStream_t st;
    hipEvent_t ev;
    FWI_HIP(hipStreamCreateWithFlags(&st, hipStreamNonBlocking));
    FWI_HIP(hipEventCreateWithFlags(&ev, hipEventDisableTiming));
    c->branch.push_back(st);
    c->branch_ev.push_back(ev);
  }
  hipStream_t main = c->cap_stream;
  // order after the caller's earlier work
  FWI_HIP(hipEventRecord(c->fork_ev, c->stream));
  FWI_HIP(hipStreamWaitEvent(main, c->fork_ev, 0));
  BatchTotals tot;
  std::vector<double> misfits(ninst, 0.0);
  for (auto& w : waves) {
    a.rewind();
    int* ctr = a.take<int>(2 * w.size());
    std::vector<BatchInst<T>*> wave;
    for (size_t k = 0; k < w.size(); ++k) {
      BatchInst<T>& I = inst[w[k]];
      plan_call<T>(a, I.p, o, FWI_ENTRY_GRADIENT, I.cb, I.sb);
      I.sb.ks.counters = ctr + 2 * k;
      I.st = c->branch[k];
      I.join = c->branch_ev[k];
      wave.push_back(&I);
    }
    // contrast
    for (BatchInst<T>* I : wave) {
      launch_check_sos(I->n, I->c, I->alpha, c->d_int, main);
      FWI_HIP(hipMemcpyAsync(c->h_int, c->d_int, 2 * sizeof(int), hipMemcpyDeviceToHost, main));
      FWI_HIP(hipStreamSynchronize(main));
      if (c->h_int[0] || c->h_int[1]) throw Error(FWI_E_NONFINITE, "invalid speed of sound / attenuation");
      launch_contrast(I->n, I->p->c0, I->p->alpha0, I->c, I->alpha, I->cb.m64, I->cb.m32, main);
    }
    // forward solves
    batch_solve<T>(c, wave, ctr, o, [](BatchInst<T>& I) -> const c128* { return I.pc->P0; },
                   [](BatchInst<T>& I) -> c128* { return I.cb.fields; }, tot);
    for (BatchInst<T>* I : wave) {
      const int ne = I->p->ne, nf = I->p->nf;
      c128* data = I->data_out ? I->data_out : I->cb.data;
      launch_gemm_nt(nf, I->cb.fields, (long)ne * I->n, ne, I->cb.m64, I->pc->P0, (long)ne * I->n, ne, I->n,
                     I->pc->coef, I->cb.gpart, gemm_splits(I->n, nf, ne, ne), data, main);
      if (gradient) {
        launch_residual((long)nf * ne * ne, data, I->dobs, I->cb.r, I->cb.misfits, main);
        launch_gemm_cn(nf, I->cb.r, ne, ne, I->pc->P0, (long)ne * I->n, I->n, I->cb.S, (long)ne * I->n, main);
      }
    }
    if (gradient) {
      batch_solve<T>(c, wave, ctr, o, [](BatchInst<T>& I) -> const c128* { return I.cb.S; },
                     [](BatchInst<T>& I) -> c128* { return I.cb.lam; }, tot);
      for (size_t k = 0; k < wave.size(); ++k) {
        BatchInst<T>* I = wave[k];
        launch_gradient_accum(I->n, I->p->nf, I->p->ne, I->cb.fields, I->cb.lam, I->pc->k2, I->cb.gpart, kGradSeg,
                              1, I->cb.gacc, main);
        launch_grad_chain(I->n, I->cb.gacc, std::pow(I->g.dx, I->g.dim), inv_kappa0(I->g), nullptr, nullptr, I->grad,
                          nullptr, nullptr, main);
        FWI_HIP(hipMemcpyAsync(&misfits[w[k]], I->cb.misfits, sizeof(double), hipMemcpyDeviceToHost, main));
      }
    }
    FWI_HIP(hipStreamSynchronize(main));
    tot.waves += 1;
  }
  // later work on the caller's stream follows this call
  FWI_HIP(hipEventRecord(c->fork_ev, main));
  FWI_HIP(hipStreamWaitEvent(c->stream, c->fork_ev, 0));
  if (misfit_out)
    for (int i = 0; i < ninst; ++i) misfit_out[i] = misfits[i];
  if (stats) {
    stats->waves = tot.waves;
    stats->graph_launches = tot.graph_launches;
    stats->iterations = tot.iters;
    stats->unconverged = tot.unconverged;
    stats->max_rel_residual = tot.maxrel;
    stats->solves = tot.solves;
    stats->t_setup_ms = t_setup;
    stats->t_solve_ms = tot.t_solve;
    stats->t_total_ms = now_ms() - t0;
  }
  return tot.unconverged ? FWI_E_NOCONV : FWI_OK;
}
// Algorithm 1: g_0 = grad m_0, u_0 = 0, then ADMM iterations until the misfit
// at the iterate falls to tol * 1/2 ||d_obs||^2 (that iteration's update is
// kept) or max_iter iterations have run.
template <typename T>
int invert_impl(fwi_ctx* c, const fwi_problem* p, const fwi_admm_params* prm, int max_iter, double tol, int nt,
                const void* w, void* rx, int born_every, void* m_io, void* g_out, void* u_out, const void* m_ref,
                const void* dobs, const fwi_solve_opts* o, double* hist, int* done, fwi_stats* stats) {
  if (!m_io || !g_out || !u_out || !dobs) throw Error(FWI_E_INVAL, "NULL argument");
  if (max_iter < 0 || !(tol >= 0.0)) throw Error(FWI_E_INVAL, "need max_iter >= 0 and tol >= 0");
  if (nt > 0 && (!w || !rx)) throw Error(FWI_E_INVAL, "NULL transmit weights or receiver fields");
  std::string msg;
  int rc = validate_problem(p, msg);
  if (rc) throw Error(rc, msg);
  const Geo g = coarse_geo(make_geo(p), prm->inv_factor);
  launch_tv_grad(g, (const c128*)m_io, (c128*)g_out, c->stream);
  launch_fill_zero_c128((long)g.dim * g.n(), (c128*)u_out, c->stream);
  if (done) *done = 0;
  fwi_stats tot{};
  int ret = FWI_OK;
  for (int k = 0; k < max_iter; ++k) {
    fwi_admm_report r{};
    fwi_stats s{};
    double half = 0.0;
    const int refresh = nt > 0 && (k == 0 || (born_every > 0 && k % born_every == 0));
    const int rk = admm_impl<T>(c, p, prm, m_io, g_out, u_out, m_ref, dobs, o, &r, &s, nt, w, (c128*)rx, refresh,
                                &half);
    if (rk != FWI_OK) ret = rk;
    if (hist) hist[k] = r.misfit;
    if (done) *done = k + 1;
    tot.iterations = std::max(tot.iterations, s.iterations);
    tot.cycles = std::max(tot.cycles, s.cycles);
    tot.unconverged += s.unconverged;
    tot.max_rel_residual = std::max(tot.max_rel_residual, s.max_rel_residual);
    tot.solves += s.solves;
    tot.matvecs += s.matvecs;
    tot.t_setup_ms += s.t_setup_ms;
    tot.t_solve_ms += s.t_solve_ms;
    tot.t_total_ms += s.t_total_ms;
    if (r.misfit <= tol * half) break;
  }
  if (stats) *stats = tot;
  return ret;
}

// y = A_l x for B vectors (the spectra must be cached), with the scratch
// (frequency indices, cast contrast, pass intermediates) carved from `bound`
// (the static scratch) or, when null, from the context's workspace.
void apply_operator_in(fwi_ctx* c, const fwi_problem* p, int precision, const void* m, int B, const int* freq_index,
                       const void* x, void* y, Arena* bound) {
  const Geo g = make_geo(p);
  const long n = g.n();
  Arena dry;
  auto plan = [&](Arena& a, int*& rf, void*& mT, void*& U1, void*& U2) {
    rf = a.take<int>(B);
    const size_t es = precision == FWI_FP32_REFINE ? sizeof(c64) : sizeof(c128);
    mT = a.take<char>(es * n);
    U1 = a.take<char>(es * B * g.u1());
    U2 = a.take<char>(es * B * std::max(1L, g.u2()));
  };
  int* rf;
  void *mT, *U1, *U2;
  plan(dry, rf, mT, U1, U2);
  Arena a;
  if (bound) {
    if (dry.used > bound->cap)
      throw Error(FWI_E_NOMEM, "the operator needs " + std::to_string(dry.used) + " bytes of scratch; the static "
                               "scratch holds " + std::to_string(bound->cap) + " (use fwi_apply_operator)");
    a = *bound;
    a.rewind();
  } else {
    bind_workspace(c, a, dry.used);
  }
  plan(a, rf, mT, U1, U2);
  hipStream_t st = c->stream;
  FWI_HIP(hipMemcpyAsync(rf, freq_index, sizeof(int) * B, hipMemcpyHostToDevice, st));
  if (precision == FWI_FP32_REFINE) {
    launch_cast_64_32(n, (const c128*)m, (c64*)mT, st);
    launch_vie<float>(g, c->tw, B, (const c64*)x, nullptr, nullptr, (const c64*)mT, c->pc.ghat32, rf, (c64*)U1,
                      (c64*)U2, (c64*)y, nullptr, EPI_VIE, st);
  } else {
    launch_vie<double>(g, c->tw, B, (const c128*)x, nullptr, nullptr, (const c128*)m, c->pc.ghat64, rf, (c128*)U1,
                       (c128*)U2, (c128*)y, nullptr, EPI_VIE, st);
  }
  FWI_HIP(hipStreamSynchronize(st));
}

void check_operator_args(const fwi_problem* p, const void* m, int B, const int* freq_index, const void* x,
                         const void* y) {
  std::string msg;
  int rc = validate_problem(p, msg);
  if (rc) throw Error(rc, msg);
  if (!m || !x || !y || !freq_index || B < 1) throw Error(FWI_E_INVAL, "bad operator arguments");
  for (int b = 0; b < B; ++b)
    if (freq_index[b] < 0 || freq_index[b] >= p->nf) throw Error(FWI_E_INVAL, "frequency index out of range");
}

}  // namespace

// ===================================================================== ABI ===
extern "C" {

void fwi_default_opts(fwi_solve_opts* o) {
  if (!o) return;
  o->precision = FWI_FP64;
  o->rtol = 1e-10;
  o->max_iter = 2000;
  o->restart = 32;
  o->max_refine = 12;
  o->inner_rtol = 1e-3;
  o->max_rhs = 0;
  o->check_every = 1;
  o->reciprocity_adjoint = 0;
  o->fields_c64 = 0;
  o->tx_chunk = 0;
}

int fwi_padded_length(int n) { return padded_length(n); }

int fwi_profile(fwi_ctx* c, unsigned mask) {
  if (!c) return FWI_E_INVAL;
  c->prof.mask = mask & ((1u << (2 * KC_COUNT)) - 1u);
  c->prof.reset();
  return FWI_OK;
}

int fwi_profile_read(const fwi_ctx* c, int cls, double* total_ms, long long* launches, double* bytes) {
  if (!c || cls < 0 || cls >= 2 * KC_COUNT) return FWI_E_INVAL;
  if (total_ms) *total_ms = c->prof.tot_ms[cls];
  if (launches) *launches = c->prof.cnt[cls];
  if (bytes) *bytes = c->prof.byt[cls];
  return FWI_OK;
}

int fwi_validate_problem(const fwi_problem* p) {
  std::string msg;
  return validate_problem(p, msg);
}

int fwi_workspace_size(const fwi_problem* p, const fwi_solve_opts* o, int entry, size_t* bytes) {
  std::string msg;
  int rc = validate_problem(p, msg);
  if (rc) return rc;
  rc = validate_opts(o, msg);
  if (rc) return rc;
  if (!bytes || entry < 0 || entry > 2) return FWI_E_INVAL;
  *bytes = o->precision == FWI_FP32_REFINE ? plan_bytes<float>(p, *o, entry) : plan_bytes<double>(p, *o, entry);
  return FWI_OK;
}

int fwi_create(fwi_ctx** out, int device, void* stream) {
  if (!out) return FWI_E_INVAL;
  *out = nullptr;
  fwi_ctx* c = new (std::nothrow) fwi_ctx();
  if (!c) return FWI_E_NOMEM;
  c->device = device;
  c->stream = (hipStream_t)stream;
  try {
    int count = 0;
    FWI_HIP(hipGetDeviceCount(&count));
    if (device < 0 || device >= count) throw Error(FWI_E_INVAL, "no such HIP device");
    FWI_HIP(hipSetDevice(device));
    make_twiddles(c);
    FWI_HIP(hipHostMalloc((void**)&c->h_int, 64 * sizeof(int), hipHostMallocDefault));
    FWI_HIP(hipHostMalloc((void**)&c->h_dbl, 64 * sizeof(double), hipHostMallocDefault));
    FWI_HIP(hipMalloc((void**)&c->d_int, 64 * sizeof(int)));
    FWI_HIP(hipEventCreateWithFlags(&c->count_ev, hipEventDisableTiming));
    FWI_HIP(hipMalloc((void**)&c->d_itstat, 2 * sizeof(unsigned long long)));
    launch_zero_u64(2, c->d_itstat, c->stream);
    FWI_HIP(hipGetSymbolAddress((void**)&c->scratch_dev, HIP_SYMBOL(scratch)));
  } catch (const Error& e) {
    fwi_destroy(c);
    return e.code;
  }
  *out = c;
  return FWI_OK;
}

void fwi_destroy(fwi_ctx* c) {
  if (!c) return;
  (void)hipSetDevice(c->device);
  c->pc.release();
  for (void* p : c->tw_allocs) (void)hipFree(p);
  if (c->ws_int) (void)hipFree(c->ws_int);
  if (c->h_int) (void)hipHostFree(c->h_int);
  if (c->h_dbl) (void)hipHostFree(c->h_dbl);
  if (c->d_int) (void)hipFree(c->d_int);
  if (c->d_itstat) (void)hipFree(c->d_itstat);
  delete c;
}

const char* fwi_last_error(const fwi_ctx* c) { return c ? c->err.c_str() : "NULL context"; }

int fwi_set_stream(fwi_ctx* c, void* stream) {
  if (!c) return FWI_E_INVAL;
  c->stream = (hipStream_t)stream;
  return FWI_OK;
}

int fwi_set_addressing(fwi_ctx* c, int wide) {
  if (!c || (wide != 0 && wide != 1)) return FWI_E_INVAL;
  c->force_wide = wide;
  return FWI_OK;
}

int fwi_set_plane_fusion(fwi_ctx* c, int on) {
  if (!c || (on != 0 && on != 1)) return FWI_E_INVAL;
  c->xy_off = on ? 0 : 1;  // the problem cache is keyed on it, so a change rebuilds the spectra
  return FWI_OK;
}

int fwi_set_workspace(fwi_ctx* c, void* ptr, size_t bytes) {
  if (!c) return FWI_E_INVAL;
  c->ws_ext = (char*)ptr;
  c->ws_ext_bytes = ptr ? bytes : 0;
  return FWI_OK;
}

int fwi_forward(fwi_ctx* c, const fwi_problem* p, const double* cc, const double* alpha, const fwi_solve_opts* o,
                void* data_out, void* fields_out, fwi_stats* stats) {
  return guarded(c, [&] {
    if (!cc) throw Error(FWI_E_INVAL, "c is NULL");
    if (!o) throw Error(FWI_E_INVAL, "opts is NULL");
    return o->precision == FWI_FP32_REFINE
               ? forward_impl<float>(c, p, cc, alpha, nullptr, o, data_out, fields_out, stats)
               : forward_impl<double>(c, p, cc, alpha, nullptr, o, data_out, fields_out, stats);
  });
}

int fwi_forward_m(fwi_ctx* c, const fwi_problem* p, const void* m, const fwi_solve_opts* o, void* data_out,
                  void* fields_out, fwi_stats* stats) {
  return guarded(c, [&] {
    if (!m) throw Error(FWI_E_INVAL, "m is NULL");
    if (!o) throw Error(FWI_E_INVAL, "opts is NULL");
    return o->precision == FWI_FP32_REFINE ? forward_impl<float>(c, p, nullptr, nullptr, m, o, data_out, fields_out, stats)
                                           : forward_impl<double>(c, p, nullptr, nullptr, m, o, data_out, fields_out, stats);
  });
}

int fwi_adjoint_gradient(fwi_ctx* c, const fwi_problem* p, const double* cc, const double* alpha, const void* dobs,
                         const fwi_solve_opts* o, double* misfit_out, void* grad_m_out, double* gc, double* ga,
                         fwi_stats* stats) {
  return guarded(c, [&] {
    if (!cc || !dobs) throw Error(FWI_E_INVAL, "NULL array argument");
    if (!o) throw Error(FWI_E_INVAL, "opts is NULL");
    return o->precision == FWI_FP32_REFINE
               ? gradient_impl<float>(c, p, cc, alpha, nullptr, dobs, nullptr, o, misfit_out, grad_m_out, gc, ga, stats)
               : gradient_impl<double>(c, p, cc, alpha, nullptr, dobs, nullptr, o, misfit_out, grad_m_out, gc, ga, stats);
  });
}

int fwi_forward_tx(fwi_ctx* c, const fwi_problem* p, const double* cc, const double* alpha, int nt,
                   const void* tx_weights, const fwi_solve_opts* o, void* data_out, void* fields_out, fwi_stats* stats) {
  return guarded(c, [&] {
    if (!o) throw Error(FWI_E_INVAL, "opts is NULL");
    return o->precision == FWI_FP32_REFINE
               ? forward_tx_impl<float>(c, p, cc, alpha, nt, tx_weights, o, data_out, fields_out, stats)
               : forward_tx_impl<double>(c, p, cc, alpha, nt, tx_weights, o, data_out, fields_out, stats);
  });
}

int fwi_adjoint_gradient_tx(fwi_ctx* c, const fwi_problem* p, const double* cc, const double* alpha, int nt,
                            const void* tx_weights, const void* dobs, const fwi_solve_opts* o, double* misfit_out,
                            void* grad_m_out, double* gc, double* ga, fwi_stats* stats) {
  return guarded(c, [&] {
    if (!o) throw Error(FWI_E_INVAL, "opts is NULL");
    return o->precision == FWI_FP32_REFINE
               ? gradient_tx_impl<float>(c, p, cc, alpha, nt, tx_weights, dobs, o, misfit_out, grad_m_out, gc, ga,
                                         stats)
               : gradient_tx_impl<double>(c, p, cc, alpha, nt, tx_weights, dobs, o, misfit_out, grad_m_out, gc, ga,
                                          stats);
  });
}

int fwi_vjp(fwi_ctx* c, const fwi_problem* p, const void* m, const void* grad_data, const fwi_solve_opts* o,
            void* grad_m_out, fwi_stats* stats) {
  return guarded(c, [&] {
    if (!m || !grad_data || !grad_m_out) throw Error(FWI_E_INVAL, "NULL array argument");
    if (!o) throw Error(FWI_E_INVAL, "opts is NULL");
    return o->precision == FWI_FP32_REFINE
               ? gradient_impl<float>(c, p, nullptr, nullptr, m, nullptr, grad_data, o, nullptr, grad_m_out, nullptr,
                                      nullptr, stats)
               : gradient_impl<double>(c, p, nullptr, nullptr, m, nullptr, grad_data, o, nullptr, grad_m_out, nullptr,
                                       nullptr, stats);
  });
}

int fwi_vjp_fields(fwi_ctx* c, const fwi_problem* p, const void* m, const void* fields, const void* grad_data,
                   const fwi_solve_opts* o, void* grad_m_out, fwi_stats* stats) {
  return guarded(c, [&] {
    if (!m || !fields || !grad_data || !grad_m_out) throw Error(FWI_E_INVAL, "NULL array argument");
    if (!o) throw Error(FWI_E_INVAL, "opts is NULL");
    return o->precision == FWI_FP32_REFINE
               ? gradient_impl<float>(c, p, nullptr, nullptr, m, nullptr, grad_data, o, nullptr, grad_m_out, nullptr,
                                      nullptr, stats, fields)
               : gradient_impl<double>(c, p, nullptr, nullptr, m, nullptr, grad_data, o, nullptr, grad_m_out, nullptr,
                                       nullptr, stats, fields);
  });
}

int fwi_tv_admm_step(fwi_ctx* c, const fwi_problem* p, const fwi_admm_params* prm, void* m_io, void* g_io, void* u_io,
                     const void* m_ref, const void* dobs, const fwi_solve_opts* o, fwi_admm_report* rep,
                     fwi_stats* stats) {
  return guarded(c, [&] {
    if (!o) throw Error(FWI_E_INVAL, "opts is NULL");
    return o->precision == FWI_FP32_REFINE ? admm_impl<float>(c, p, prm, m_io, g_io, u_io, m_ref, dobs, o, rep, stats)
                                           : admm_impl<double>(c, p, prm, m_io, g_io, u_io, m_ref, dobs, o, rep, stats);
  });
}

int fwi_tv_admm_step_tx(fwi_ctx* c, const fwi_problem* p, const fwi_admm_params* prm, int nt, const void* tx_weights,
                        void* rx_fields, int refresh_rx, void* m_io, void* g_io, void* u_io, const void* m_ref,
                        const void* dobs, const fwi_solve_opts* o, fwi_admm_report* rep, fwi_stats* stats) {
  return guarded(c, [&] {
    if (!o) throw Error(FWI_E_INVAL, "opts is NULL");
    if (nt < 1) throw Error(FWI_E_INVAL, "need 1 <= nt <= ne synthesised transmits");
    return o->precision == FWI_FP32_REFINE
               ? admm_impl<float>(c, p, prm, m_io, g_io, u_io, m_ref, dobs, o, rep, stats, nt, tx_weights,
                                  (c128*)rx_fields, refresh_rx)
               : admm_impl<double>(c, p, prm, m_io, g_io, u_io, m_ref, dobs, o, rep, stats, nt, tx_weights,
                                   (c128*)rx_fields, refresh_rx);
  });
}

int fwi_invert(fwi_ctx* c, const fwi_problem* p, const fwi_admm_params* prm, int max_iter, double tol, int nt,
               const void* tx_weights, void* rx_fields, int born_every, void* m_inout, void* g_out, void* u_out,
               const void* m_ref, const void* d_obs, const fwi_solve_opts* o, double* misfit_hist, int* iters_done,
               fwi_stats* stats) {
  return guarded(c, [&] {
    if (!o || !prm) throw Error(FWI_E_INVAL, "NULL argument");
    return o->precision == FWI_FP32_REFINE
               ? invert_impl<float>(c, p, prm, max_iter, tol, nt, tx_weights, rx_fields, born_every, m_inout, g_out,
                                    u_out, m_ref, d_obs, o, misfit_hist, iters_done, stats)
               : invert_impl<double>(c, p, prm, max_iter, tol, nt, tx_weights, rx_fields, born_every, m_inout, g_out,
                                     u_out, m_ref, d_obs, o, misfit_hist, iters_done, stats);
  });
}

int fwi_sos_from_contrast(fwi_ctx* c, const fwi_problem* p, const void* m, double* c_out, double* alpha_out) {
  return guarded(c, [&] {
    if (!p || !m || (!c_out && !alpha_out)) throw Error(FWI_E_INVAL, "bad arguments");
    std::string msg;
    int rc = validate_problem(p, msg);
    if (rc) throw Error(rc, msg);
    launch_sos_from_contrast(make_geo(p).n(), kappa0_rho(p->c0, p->alpha0), (const c128*)m, c_out, alpha_out,
                             c->stream);
    FWI_HIP(hipStreamSynchronize(c->stream));
    return FWI_OK;
  });
}

int fwi_apply_operator(fwi_ctx* c, const fwi_problem* p, int precision, const void* m, int B, const int* freq_index,
                       const void* x, void* y) {
  return guarded(c, [&] {
    check_operator_args(p, m, B, freq_index, x, y);
    ensure_cache(c, p);
    apply_operator_in(c, p, precision, m, B, freq_index, x, y, nullptr);
    return FWI_OK;
  });
}

int fwi_apply_operator_noalloc(fwi_ctx* c, const fwi_problem* p, int precision, const void* m, int B,
                               const int* freq_index, const void* x, void* y) {
  return guarded(c, [&] {
    check_operator_args(p, m, B, freq_index, x, y);
    if (problem_key(p) != c->pc.key)
      throw Error(FWI_E_INVAL, "no cached spectra for this problem on this context (building them allocates): "
                               "call an entry point such as fwi_green_spectrum on it first");
    if (!c->scratch_dev) throw Error(FWI_E_DEVICE, "static scratch address unknown");
    Arena s;
    s.base = c->scratch_dev;
    s.cap = kStaticScratchBytes;
    s.dry = false;
    apply_operator_in(c, p, precision, m, B, freq_index, x, y, &s);
    return FWI_OK;
  });
}

int fwi_solve(fwi_ctx* c, const fwi_problem* p, const void* m, int B, const int* freq_index, const void* rhs,
              const fwi_solve_opts* o, void* x_out, fwi_stats* stats) {
  return guarded(c, [&] {
    const double t0 = now_ms();
    if (!m || !rhs || !x_out || !freq_index || B < 1 || !o) throw Error(FWI_E_INVAL, "bad solve arguments");
    for (int b = 0; b < B; ++b)
      if (freq_index[b] < 0 || freq_index[b] >= p->nf) throw Error(FWI_E_INVAL, "frequency index out of range");
    Runner R(c, p, *o);
    auto run = [&](auto tag) {
      using T = decltype(tag);
      SolveBufs<T> sb;
      prepare<T>(c, R, sb, FWI_ENTRY_FORWARD, B);
      hipStream_t st = c->stream;
      check_complex(c, R.n, (const c128*)m, "m");
      launch_copy_c128(R.n, (const c128*)m, R.cb.m64, st);
      launch_cast_64_32(R.n, R.cb.m64, R.cb.m32, st);
      FWI_HIP(hipMemcpyAsync(R.cb.rfreq, freq_index, sizeof(int) * B, hipMemcpyHostToDevice, st));
      const cplx<T>* mT = std::is_same<T, float>::value ? (const cplx<T>*)R.cb.m32 : (const cplx<T>*)R.cb.m64;
      const cplx<T>* gT =
          std::is_same<T, float>::value ? (const cplx<T>*)c->pc.ghat32 : (const cplx<T>*)c->pc.ghat64;
      const int nfreq = (int)std::set<int>(freq_index, freq_index + B).size();
      SolveTotals r = run_solve<T>(c, R.g, R.cb.m64, mT, c->pc.ghat64, gT, B, (const c128*)rhs, R.cb.rfreq,
                                   (c128*)x_out, R.o, sb, nfreq);
      R.tot.merge(r);
    };
    if (o->precision == FWI_FP32_REFINE) run(float{});
    else run(double{});
    collect_iters(c, R.tot);
  fill_stats(stats, R.tot, R.t_setup, now_ms() - t0);
    return finish_rc(R.tot);
  });
}

int fwi_incident(fwi_ctx* c, const fwi_problem* p, int l, void* out) {
  return guarded(c, [&] {
    std::string msg;
    int rc = validate_problem(p, msg);
    if (rc) throw Error(rc, msg);
    if (!out || l < 0 || l >= p->nf) throw Error(FWI_E_INVAL, "bad arguments");
    ensure_cache(c, p);
    const long cnt = c->pc.g.n() * p->ne;
    launch_copy_c128(cnt, c->pc.P0 + (long)l * cnt, (c128*)out, c->stream);
    FWI_HIP(hipStreamSynchronize(c->stream));
    return FWI_OK;
  });
}

int fwi_green_spectrum(fwi_ctx* c, const fwi_problem* p, int l, void* out) {
  return guarded(c, [&] {
    std::string msg;
    int rc = validate_problem(p, msg);
    if (rc) throw Error(rc, msg);
    if (!out || l < 0 || l >= p->nf) throw Error(FWI_E_INVAL, "bad arguments");
    ensure_cache(c, p);
    const long np = c->pc.g.npad();
    launch_copy_c128(np, c->pc.ghat64 + (long)l * np, (c128*)out, c->stream);
    FWI_HIP(hipStreamSynchronize(c->stream));
    return FWI_OK;
  });
}

int fwi_fft_padded(fwi_ctx* c, const fwi_problem* p, int precision, const void* in, void* out) {
  return guarded(c, [&] {
    std::string msg;
    int rc = validate_problem(p, msg);
    if (rc) throw Error(rc, msg);
    if (!in || !out) throw Error(FWI_E_INVAL, "bad arguments");
    const Geo g = make_geo(p);
    const size_t es = precision == FWI_FP32_REFINE ? sizeof(c64) : sizeof(c128);
    Arena dry;
    dry.take<char>(es * g.u1());
    Arena a;
    bind_workspace(c, a, dry.used);
    void* U1 = a.take<char>(es * g.u1());
    if (precision == FWI_FP32_REFINE)
      launch_fft_padded<float>(g, c->tw, (const c64*)in, (c64*)U1, (c64*)out, c->stream);
    else
      launch_fft_padded<double>(g, c->tw, (const c128*)in, (c128*)U1, (c128*)out, c->stream);
    FWI_HIP(hipStreamSynchronize(c->stream));
    return FWI_OK;
  });
}

int fwi_jacobian_apply(fwi_ctx* c, const fwi_problem* p, const void* fields, const void* a, void* out) {
  return guarded(c, [&] {
    std::string msg;
    int rc = validate_problem(p, msg);
    if (rc) throw Error(rc, msg);
    if (!fields || !a || !out) throw Error(FWI_E_INVAL, "bad arguments");
    ensure_cache(c, p);
    const Geo g = make_geo(p);
    const long n = g.n();
    Arena dry;
    dry.take<c128>((size_t)gemm_splits_max(n) * p->nf * p->ne * p->ne);
    Arena ar;
    bind_workspace(c, ar, dry.used);
    CallBufs cb;
    cb.gpart = ar.take<c128>((size_t)gemm_splits_max(n) * p->nf * p->ne * p->ne);
    j_apply(c, p, g, cb, p->ne, (const c128*)fields, (const c128*)fields, (const c128*)a, (c128*)out);
    FWI_HIP(hipStreamSynchronize(c->stream));
    return FWI_OK;
  });
}

int fwi_jacobian_adjoint_apply(fwi_ctx* c, const fwi_problem* p, const void* fields, const void* b, void* out) {
  return guarded(c, [&] {
    std::string msg;
    int rc = validate_problem(p, msg);
    if (rc) throw Error(rc, msg);
    if (!fields || !b || !out) throw Error(FWI_E_INVAL, "bad arguments");
    ensure_cache(c, p);
    const Geo g = make_geo(p);
    const long n = g.n();
    auto plan = [&](Arena& a, CallBufs& cb) {
      cb.lam = a.take<c128>((size_t)p->nf * p->ne * n);
      cb.gpart_len = (long)kGradSeg * n;
      cb.gpart = a.take<c128>(cb.gpart_len);
      cb.gacc = a.take<c128>(n);
    };
    Arena dry;
    CallBufs d;
    plan(dry, d);
    Arena ar;
    bind_workspace(c, ar, dry.used);
    CallBufs cb;
    plan(ar, cb);
    jh_apply(c, p, g, cb, p->nf, p->ne, (const c128*)fields, (const c128*)fields, (const c128*)b, (c128*)out);
    FWI_HIP(hipStreamSynchronize(c->stream));
    return FWI_OK;
  });
}

// Jacobian products with separate transmit fields [nf][nt][n] and receiver
// fields [nf][ne][n] (Sec. IV-B): (J a)_{l,t,j} = k_l^2 dV sum_n p_t p~_j a_n,
// J^H b = dV sum_l conj(k_l^2) sum_t conj(p_t) conj(sum_j conj(b_tj) p~_j).
static void check_tx_fields(const fwi_problem* p, int nt, const void* tx, const void* rx, const void* v,
                            const void* out) {
  if (!tx || !rx || !v || !out) throw Error(FWI_E_INVAL, "bad arguments");
  if (nt < 1 || nt > p->ne) throw Error(FWI_E_INVAL, "need 1 <= nt <= ne transmits");
}

int fwi_jacobian_apply_tx(fwi_ctx* c, const fwi_problem* p, int nt, const void* tx_fields, const void* rx_fields,
                          const void* a, void* out) {
  return guarded(c, [&] {
    std::string msg;
    int rc = validate_problem(p, msg);
    if (rc) throw Error(rc, msg);
    check_tx_fields(p, nt, tx_fields, rx_fields, a, out);
    ensure_cache(c, p);
    const long n = make_geo(p).n();
    const size_t part = (size_t)gemm_splits_max(n) * p->nf * nt * p->ne;
    Arena dry;
    dry.take<c128>(part);
    Arena ar;
    bind_workspace(c, ar, dry.used);
    c128* gpart = ar.take<c128>(part);
    launch_gemm_nt(p->nf, (const c128*)tx_fields, (long)nt * n, nt, (const c128*)a, (const c128*)rx_fields,
                   (long)p->ne * n, p->ne, n, c->pc.coef, gpart, gemm_splits(n, p->nf, nt, p->ne), (c128*)out,
                   c->stream);
    FWI_HIP(hipStreamSynchronize(c->stream));
    return FWI_OK;
  });
}

int fwi_jacobian_adjoint_apply_tx(fwi_ctx* c, const fwi_problem* p, int nt, const void* tx_fields,
                                  const void* rx_fields, const void* b, void* out) {
  return guarded(c, [&] {
    std::string msg;
    int rc = validate_problem(p, msg);
    if (rc) throw Error(rc, msg);
    check_tx_fields(p, nt, tx_fields, rx_fields, b, out);
    ensure_cache(c, p);
    const Geo g = make_geo(p);
    const long n = g.n();
    auto plan = [&](Arena& ar, CallBufs& cb) {
      cb.lam = ar.take<c128>((size_t)p->nf * nt * n);
      cb.gpart_len = (long)kGradSeg * n;
      cb.gpart = ar.take<c128>(cb.gpart_len);
      cb.gacc = ar.take<c128>(n);
    };
    Arena dry;
    CallBufs d;
    plan(dry, d);
    Arena ar;
    bind_workspace(c, ar, dry.used);
    CallBufs cb;
    plan(ar, cb);
    hipStream_t st = c->stream;
    launch_gemm_cn(p->nf, (const c128*)b, nt, p->ne, (const c128*)rx_fields, (long)p->ne * n, n, cb.lam,
                   (long)nt * n, st);
    launch_gradient_accum(n, p->nf, nt, (const c128*)tx_fields, cb.lam, c->pc.k2, cb.gpart, kGradSeg, 1, cb.gacc, st);
    launch_grad_chain(n, cb.gacc, std::pow(g.dx, g.dim), inv_kappa0(g), nullptr, nullptr, (c128*)out, nullptr, nullptr, st);
    FWI_HIP(hipStreamSynchronize(st));
    return FWI_OK;
  });
}

int fwi_autotune(fwi_ctx* c, const fwi_problem* p, int precision, int B, int reps, fwi_tune_report* rep) {
  return guarded(c, [&] {
    std::string msg;
    int rc = validate_problem(p, msg);
    if (rc) throw Error(rc, msg);
    if (B < 1 || reps < 1 || (precision != FWI_FP64 && precision != FWI_FP32_REFINE))
      throw Error(FWI_E_INVAL, "bad autotune arguments");
    ensure_cache(c, p);
    const ProblemCache& pc = c->pc;
    const Geo g = make_geo(p);
    const long n = g.n();
    const bool dbl = precision == FWI_FP64;
    const size_t es = dbl ? sizeof(c128) : sizeof(c64);
    auto plan = [&](Arena& a, int*& rf, char*& x, char*& y, char*& mT, char*& U1, char*& U2) {
      rf = a.take<int>(B);
      x = a.take<char>(es * B * n);
      y = a.take<char>(es * B * n);
      mT = a.take<char>(es * n);
      U1 = a.take<char>(es * B * g.u1());
      U2 = a.take<char>(es * B * std::max(1L, g.u2()));
    };
    int* rf;
    char *x, *y, *mT, *U1, *U2;
    Arena dry;
    plan(dry, rf, x, y, mT, U1, U2);
    Arena ar;
    bind_workspace(c, ar, dry.used);
    plan(ar, rf, x, y, mT, U1, U2);
    hipStream_t st = c->stream;
    const long nsrc = (long)pc.nf * pc.ne;
    std::vector<int> hrf(B);
    for (int b = 0; b < B; ++b) hrf[b] = (int)((b % nsrc) / pc.ne);
    FWI_HIP(hipMemcpyAsync(rf, hrf.data(), sizeof(int) * B, hipMemcpyHostToDevice, st));
    for (int b = 0; b < B; ++b) {
      const c128* src = pc.P0 + (b % nsrc) * n;
      if (dbl) launch_copy_c128(n, src, (c128*)x + (long)b * n, st);
      else launch_cast_64_32(n, src, (c64*)x + (long)b * n, st);
    }
    // a contrast-like operand: a copy of the first incident field
    if (dbl) {
      launch_copy_c128(n, pc.P0, (c128*)mT, st);
    } else {
      launch_cast_64_32(n, pc.P0, (c64*)mT, st);
    }
    tl_nfreq = std::min<long>(pc.nf, (B + pc.ne - 1) / pc.ne);
    tl_active = B;
    EventProfiler local;
    local.mask = (1u << (2 * KC_COUNT)) - 1u;
    LaunchProfiler* saved = tl_prof;
    double t[KC_COUNT][kNumVariants] = {};
    for (int v = 0; v < kNumVariants; ++v) {
      tl_force_variant = v;
      tl_prof = nullptr;
      auto run = [&]() {
        if (dbl)
          launch_vie<double>(g, c->tw, B, (const c128*)x, nullptr, nullptr, (const c128*)mT, pc.ghat64, rf,
                             (c128*)U1, (c128*)U2, (c128*)y, nullptr, EPI_VIE, st);
        else
          launch_vie<float>(g, c->tw, B, (const c64*)x, nullptr, nullptr, (const c64*)mT, pc.ghat32, rf, (c64*)U1,
                            (c64*)U2, (c64*)y, nullptr, EPI_VIE, st);
      };
      run();  // warm
      local.reset();
      tl_prof = &local;
      for (int r = 0; r < reps; ++r) run();
      FWI_HIP(hipStreamSynchronize(st));
      local.flush();
      const int off = dbl ? KC_COUNT : 0;
      for (int k = 0; k < KC_COUNT; ++k)
        t[k][v] = local.cnt[k + off] ? local.tot_ms[k + off] / local.cnt[k + off] : 0.0;
    }
    tl_prof = saved;
    tl_force_variant = -1;
    // class -> pass kind and length
    const int kinds[KC_COUNT] = {PK_ROW_FWD, PK_CONV, PK_ROW_INV, PK_STRIDED, PK_STRIDED, -1, -1, -1};
    const int lens[KC_COUNT] = {g.Lx, g.Lz, g.Lx, g.Ly, g.Ly, 0, 0, 0};
    double strided_sum[kNumVariants] = {};
    for (int v = 0; v < kNumVariants; ++v) strided_sum[v] = t[KC_Y_FWD][v] + t[KC_Y_INV][v];
    for (int k = 0; k < KC_COUNT; ++k) {
      if (kinds[k] < 0 || k == KC_Y_INV) continue;
      const double* tv = k == KC_Y_FWD ? strided_sum : t[k];
      if (tv[0] == 0.0) continue;
      c->tune.v[kinds[k]][dbl ? 1 : 0][length_index(lens[k])] =
          (signed char)pick_variant(tv, default_variant(kinds[k], dbl, lens[k]));
    }
    if (rep) {
      for (int k = 0; k < 5; ++k) {
        for (int v = 0; v < kNumVariants; ++v) rep->variant_ms[k][v] = t[k][v];
        rep->default_variant[k] = kinds[k] >= 0 ? default_variant(kinds[k], dbl, lens[k]) : -1;
        rep->variant[k] = t[k][0] > 0.0 ? pick_variant(t[k], rep->default_variant[k] >= 0 ? rep->default_variant[k] : 0)
                                         : -1;
      }
      // the elevation passes are tuned on their summed time
      if (strided_sum[0] > 0.0) rep->variant[KC_Y_FWD] = rep->variant[KC_Y_INV] =
          pick_variant(strided_sum, default_variant(PK_STRIDED, dbl, g.Ly));
    }
    return FWI_OK;
  });
}

int fwi_autotune_solver(fwi_ctx* c, const fwi_problem* p, const double* cc, const double* alpha, const void* dobs,
                        const fwi_solve_opts* base, const int* max_rhs, int n_mr, const int* restart, int n_rs,
                        const double* inner_rtol, int n_in, int reps, fwi_solver_tune_report* rep) {
  return guarded(c, [&] {
    if (!p || !cc || !dobs || !base || !max_rhs || !restart || !rep || reps < 1)
      throw Error(FWI_E_INVAL, "bad solver autotune arguments");
    if (!inner_rtol) n_in = 1;  // the base options' own inner tolerance
    if (n_mr < 1 || n_mr > 8 || n_rs < 1 || n_rs > 3 || n_in < 1 || n_in > 3)
      throw Error(FWI_E_INVAL, "1..8 batch caps, 1..3 restart lengths and 1..3 inner tolerances");
    std::string msg;
    int rc = validate_opts(base, msg);
    if (rc) throw Error(rc, msg);
    for (int i = 0; i < n_mr; ++i)
      if (max_rhs[i] < 0) throw Error(FWI_E_INVAL, "max_rhs candidates must be >= 0");
    for (int j = 0; j < n_rs; ++j)
      if (restart[j] != 8 && restart[j] != 16 && restart[j] != 32)
        throw Error(FWI_E_INVAL, "restart candidates must be 8, 16 or 32");
    for (int h = 0; inner_rtol && h < n_in; ++h)
      if (!(inner_rtol[h] > 0.0 && inner_rtol[h] < 1.0))
        throw Error(FWI_E_INVAL, "inner_rtol candidates must be in (0, 1)");
    // the library's own workspace grows to the largest candidate's plan;
    // a grown one is released at the end so that the tuning leaves no
    // allocation larger than the caller's own calls make
    const size_t ws_before = c->ws_int_bytes;
    struct Release {
      fwi_ctx* c;
      size_t before;
      ~Release() {
        if (c->ws_int_bytes > before) {
          (void)hipStreamSynchronize(c->stream);
          (void)hipFree(c->ws_int);
          c->ws_int = nullptr;
          c->ws_int_bytes = 0;
        }
      }
    } release{c, ws_before};
    fwi_solver_tune_report r{};
    double best = std::numeric_limits<double>::infinity();
    for (int h = 0; h < n_in; ++h) {
      for (int i = 0; i < n_mr; ++i) {
        for (int j = 0; j < n_rs; ++j) {
          fwi_solve_opts o = *base;
          o.max_rhs = max_rhs[i];
          o.restart = restart[j];
          if (inner_rtol) o.inner_rtol = inner_rtol[h];
          rc = validate_opts(&o, msg);
          if (rc) throw Error(rc, msg);
          double t = std::numeric_limits<double>::infinity();
          bool converged = true;
          for (int k = 0; k <= reps; ++k) {  // the first call is untimed
            const double t0 = now_ms();
            rc = o.precision == FWI_FP32_REFINE
                     ? gradient_impl<float>(c, p, cc, alpha, nullptr, dobs, nullptr, &o, nullptr, nullptr, nullptr,
                                            nullptr, nullptr)
                     : gradient_impl<double>(c, p, cc, alpha, nullptr, dobs, nullptr, &o, nullptr, nullptr, nullptr,
                                             nullptr, nullptr);
            const double dt = now_ms() - t0;  // the call returns after synchronising its stream
            if (rc != FWI_OK && rc != FWI_E_NOCONV) return rc;
            converged = converged && rc == FWI_OK;
            if (k > 0) t = std::min(t, dt);
          }
          r.ms[h][i][j] = t;
          if (converged && t < best) {
            best = t;
            r.max_rhs = o.max_rhs;
            r.restart = o.restart;
            r.inner_rtol = o.inner_rtol;
          }
        }
      }
    }
    if (!(best < std::numeric_limits<double>::infinity()))
      throw Error(FWI_E_NOCONV, "no candidate converged");
    *rep = r;
    return FWI_OK;
  });
}

int fwi_get_tuning(const fwi_ctx* c, signed char* out, int count) {
  if (!c || !out || count != (int)sizeof(FftTuning::v)) return FWI_E_INVAL;
  std::memcpy(out, c->tune.v, sizeof(FftTuning::v));
  return FWI_OK;
}

int fwi_set_tuning(fwi_ctx* c, const signed char* in, int count) {
  if (!c) return FWI_E_INVAL;
  if (!in) {
    c->tune = FftTuning();
    return FWI_OK;
  }
  if (count != (int)sizeof(FftTuning::v)) return FWI_E_INVAL;
  std::memcpy(c->tune.v, in, sizeof(FftTuning::v));
  return FWI_OK;
}

int fwi_adjoint_gradient_batch(fwi_ctx* c, int ninst, const fwi_problem* probs, const double* const* cc,
                               const double* const* alpha, const void* const* d_obs, const fwi_solve_opts* o,
                               double* misfit_out, void* const* grad_m_out, fwi_batch_stats* stats) {
  return guarded(c, [&] {
    if (!o || !d_obs) throw Error(FWI_E_INVAL, "bad batch arguments");
    return o->precision == FWI_FP32_REFINE
               ? batch_impl<float>(c, ninst, probs, cc, alpha, d_obs, o, misfit_out, grad_m_out, nullptr, stats)
               : batch_impl<double>(c, ninst, probs, cc, alpha, d_obs, o, misfit_out, grad_m_out, nullptr, stats);
  });
}

int fwi_forward_batch(fwi_ctx* c, int ninst, const fwi_problem* probs, const double* const* cc,
                      const double* const* alpha, const fwi_solve_opts* o, void* const* data_out,
                      fwi_batch_stats* stats) {
  return guarded(c, [&] {
    if (!o) throw Error(FWI_E_INVAL, "opts is NULL");
    return o->precision == FWI_FP32_REFINE
               ? batch_impl<float>(c, ninst, probs, cc, alpha, nullptr, o, nullptr, nullptr, data_out, stats)
               : batch_impl<double>(c, ninst, probs, cc, alpha, nullptr, o, nullptr, nullptr, data_out, stats);
  });
}

}  // extern "C"
