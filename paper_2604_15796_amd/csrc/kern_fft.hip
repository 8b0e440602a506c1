// FFT passes of the Green's-function convolution (Sec. IV-A): the discrete
// operator y = x - crop(IFFT(Ghat . FFT(pad(m x)))) of Eq. 5, batched over
// right-hand sides.
//
// 2D (grid [nz][nx], padded [Lz][Lx]):
//   pass 1  rows   : U1[b][z][:]  = FFT_Lx(pad(m . s_b x_b[z][:]))
//   pass 2  columns: U1[b][:][kx] = crop(IFFT_Lz(Ghat[f_b][:][kx] . FFT_Lz(pad(U1[b][:][kx]))))   (in place)
//   pass 3  rows   : y_b[z][:]    = s_b x_b[z][:] - crop(IFFT_Lx(U1[b][z][:]))
// 3D adds a forward and an inverse pass along y around the z convolution.
// Every pass reads and writes its data once in HBM; the 1/(Lz Ly Lx) of the
// inverse transform and k^2 are folded into Ghat.
#include "fft.hpp"
#include "internal.hpp"

namespace fwi {

constexpr int NT = 256;

template <typename T>
__host__ __device__ constexpr int pts_per_wg() {
  return sizeof(T) == 4 ? 8192 : 4096;
}
template <typename T, int L>
__host__ __device__ constexpr int row_nl() {
  return pts_per_wg<T>() / L > 1 ? pts_per_wg<T>() / L : 1;
}
template <typename T, int L>
__host__ __device__ constexpr int col_nl() {
  // power of two, 4..16 lines (coalesced 32..128-byte column segments)
  return pts_per_wg<T>() / L >= 16 ? 16 : pts_per_wg<T>() / L >= 8 ? 8 : 4;
}

// ------------------------------------------------------------- row pass 1 ---
template <typename T>
struct RowFwdArgs {
  const cplx<T>* x;      // rows of length nin, row stride in_stride
  const cplx<T>* m;      // [rows_per_rhs][nin] or null
  const cplx<T>* scale;  // [B] or null
  const int* active;     // [B] or null
  cplx<T>* out;          // rows of length L
  const cplx<T>* tw;
  long nrows;
  int rows_per_rhs, nin;
  long in_stride;
};

template <typename T, int L>
__global__ void __launch_bounds__(NT) k_row_fwd(RowFwdArgs<T> a) {
  using C = LineCfg<T, L, row_nl<T, L>(), NT, false>;
  __shared__ cplx<T> sh[C::LDS_ELEMS];
  __shared__ long s_x[C::NL];
  __shared__ int s_m[C::NL];
  __shared__ cplx<T> s_s[C::NL];
  __shared__ int s_ok[C::NL];
  const long g0 = (long)blockIdx.x * C::NL;
  for (int l = threadIdx.x; l < C::NL; l += NT) {
    const long g = g0 + l;
    int ok = g < a.nrows;
    const long b = ok ? g / a.rows_per_rhs : 0;
    if (ok && a.active && !a.active[b]) ok = 0;
    s_ok[l] = ok;
    s_x[l] = g * a.in_stride;
    s_m[l] = (int)(g - b * a.rows_per_rhs) * a.nin;
    s_s[l] = a.scale ? a.scale[b] : mk((T)1, (T)0);
  }
  __syncthreads();
  auto src = [&](int line, int p) -> cplx<T> {
    if (!s_ok[line] || p >= a.nin) return mk((T)0, (T)0);
    cplx<T> v = a.x[s_x[line] + p];
    if (a.m) v = v * a.m[s_m[line] + p];
    if (a.scale) v = v * s_s[line];
    return v;
  };
  auto snk = [&](int line, int p, cplx<T> v) {
    if (s_ok[line]) a.out[(g0 + line) * L + p] = v;
  };
  fft_line_transform<C, 0>(a.tw, sh, src, snk);
}

// ------------------------------------------------------------- row pass 3 ---
template <typename T>
struct RowInvArgs {
  const cplx<T>* in;     // rows of length L
  const cplx<T>* x;      // [rows][nout] operand (scaled by s_b) or null for EPI_COPY
  const cplx<T>* rhs;    // [rows][nout] (EPI_RESID)
  const cplx<T>* scale;
  const int* active;
  cplx<T>* y;            // [rows][nout]
  const cplx<T>* tw;
  long nrows;
  int rows_per_rhs, nout;
};

template <typename T, int L, int EPI>
__global__ void __launch_bounds__(NT) k_row_inv(RowInvArgs<T> a) {
  using C = LineCfg<T, L, row_nl<T, L>(), NT, false>;
  __shared__ cplx<T> sh[C::LDS_ELEMS];
  __shared__ cplx<T> s_s[C::NL];
  __shared__ int s_ok[C::NL];
  const long g0 = (long)blockIdx.x * C::NL;
  for (int l = threadIdx.x; l < C::NL; l += NT) {
    const long g = g0 + l;
    int ok = g < a.nrows;
    const long b = ok ? g / a.rows_per_rhs : 0;
    if (ok && a.active && !a.active[b]) ok = 0;
    s_ok[l] = ok;
    s_s[l] = a.scale ? a.scale[b] : mk((T)1, (T)0);
  }
  __syncthreads();
  auto src = [&](int line, int p) -> cplx<T> {
    if (!s_ok[line]) return mk((T)0, (T)0);
    return a.in[(g0 + line) * L + p];
  };
  auto snk = [&](int line, int p, cplx<T> v) {
    if (!s_ok[line] || p >= a.nout) return;
    const long o = (g0 + line) * a.nout + p;
    if constexpr (EPI == EPI_VIE) {
      cplx<T> xv = a.x[o];
      if (a.scale) xv = xv * s_s[line];
      a.y[o] = xv - v;
    } else if constexpr (EPI == EPI_RESID) {
      a.y[o] = a.rhs[o] - (a.x[o] - v);
    } else {
      a.y[o] = v;
    }
  };
  fft_line_transform<C, 1>(a.tw, sh, src, snk);
}

// --------------------------------------------------------- strided passes ---
template <typename T>
struct StridedArgs {
  const cplx<T>* in;
  cplx<T>* out;
  const cplx<T>* tw;
  const cplx<T>* ghat;    // conv only: [nf][...] same layout as a data plane
  const int* rhs_freq;    // conv only
  const int* active;
  long in_ps, out_ps;     // plane strides
  long pstride;           // elements between consecutive points of a line
  long gstride;           // Ghat stride between frequencies
  int nlines;             // lines per plane
  int planes_per_rhs;
  int lin, lout;          // nonzero input points, output points kept
};

template <typename T, int L, int MODE>  // MODE 0 forward, 1 inverse, 2 convolution
__global__ void __launch_bounds__(NT) k_strided(StridedArgs<T> a) {
  using C = LineCfg<T, L, col_nl<T, L>(), NT, true>;
  __shared__ cplx<T> sh[C::LDS_ELEMS];
  const long plane = blockIdx.y;
  const int b = (int)(plane / a.planes_per_rhs);
  if (a.active && !a.active[b]) return;  // uniform per workgroup
  const int line0 = blockIdx.x * C::NL;
  const cplx<T>* ip = a.in + plane * a.in_ps + line0;
  cplx<T>* op = a.out + plane * a.out_ps + line0;
  const int nl = a.nlines - line0;
  auto src = [&](int line, int p) -> cplx<T> {
    if (p >= a.lin || line >= nl) return mk((T)0, (T)0);
    return ip[p * a.pstride + line];
  };
  auto snk = [&](int line, int p, cplx<T> v) {
    if (p < a.lout && line < nl) op[p * a.pstride + line] = v;
  };
  if constexpr (MODE == 2) {
    const cplx<T>* gp = a.ghat + (long)a.rhs_freq[b] * a.gstride + line0;
    auto gh = [&](int line, int p) -> cplx<T> { return line < nl ? gp[p * a.pstride + line] : mk((T)0, (T)0); };
    fft_line_convolve<C>(a.tw, sh, src, gh, snk);
  } else {
    fft_line_transform<C, MODE>(a.tw, sh, src, snk);
  }
}

// ---------------------------------------------------------------- dispatch ---
template <typename T>
struct Launch {
  template <int L>
  static void row_fwd(const RowFwdArgs<T>& a, hipStream_t st) {
    constexpr int NL = row_nl<T, L>();
    const unsigned grid = (unsigned)((a.nrows + NL - 1) / NL);
    if (grid == 0) return;
    hipLaunchKernelGGL((k_row_fwd<T, L>), dim3(grid), dim3(NT), 0, st, a);
    FWI_LAUNCH_CHECK();
  }
  template <int L>
  static void row_inv(const RowInvArgs<T>& a, int epi, hipStream_t st) {
    constexpr int NL = row_nl<T, L>();
    const unsigned grid = (unsigned)((a.nrows + NL - 1) / NL);
    if (grid == 0) return;
    if (epi == EPI_VIE) hipLaunchKernelGGL((k_row_inv<T, L, EPI_VIE>), dim3(grid), dim3(NT), 0, st, a);
    else if (epi == EPI_RESID) hipLaunchKernelGGL((k_row_inv<T, L, EPI_RESID>), dim3(grid), dim3(NT), 0, st, a);
    else hipLaunchKernelGGL((k_row_inv<T, L, EPI_COPY>), dim3(grid), dim3(NT), 0, st, a);
    FWI_LAUNCH_CHECK();
  }
  template <int L>
  static void strided(const StridedArgs<T>& a, long planes, int mode, hipStream_t st) {
    constexpr int NL = col_nl<T, L>();
    if (planes == 0) return;
    if (planes > 65535) throw Error(-6, "too many planes for one strided pass");
    dim3 grid((a.nlines + NL - 1) / NL, (unsigned)planes);
    if (mode == 0) hipLaunchKernelGGL((k_strided<T, L, 0>), grid, dim3(NT), 0, st, a);
    else if (mode == 1) hipLaunchKernelGGL((k_strided<T, L, 1>), grid, dim3(NT), 0, st, a);
    else hipLaunchKernelGGL((k_strided<T, L, 2>), grid, dim3(NT), 0, st, a);
    FWI_LAUNCH_CHECK();
  }
};

template <typename T>
static void strided_call(int L, const StridedArgs<T>& a, long planes, int mode, hipStream_t st) {
  switch (L) {
    case 32: Launch<T>::template strided<32>(a, planes, mode, st); break;
    case 48: Launch<T>::template strided<48>(a, planes, mode, st); break;
    case 64: Launch<T>::template strided<64>(a, planes, mode, st); break;
    case 96: Launch<T>::template strided<96>(a, planes, mode, st); break;
    case 128: Launch<T>::template strided<128>(a, planes, mode, st); break;
    case 192: Launch<T>::template strided<192>(a, planes, mode, st); break;
    case 256: Launch<T>::template strided<256>(a, planes, mode, st); break;
    case 384: Launch<T>::template strided<384>(a, planes, mode, st); break;
    case 512: Launch<T>::template strided<512>(a, planes, mode, st); break;
    case 768: Launch<T>::template strided<768>(a, planes, mode, st); break;
    case 1024: Launch<T>::template strided<1024>(a, planes, mode, st); break;
    default: throw Error(-6, "unsupported FFT length " + std::to_string(L));
  }
}
template <typename T>
static void row_fwd_call(int L, const RowFwdArgs<T>& a, hipStream_t st) {
  switch (L) {
    case 32: Launch<T>::template row_fwd<32>(a, st); break;
    case 48: Launch<T>::template row_fwd<48>(a, st); break;
    case 64: Launch<T>::template row_fwd<64>(a, st); break;
    case 96: Launch<T>::template row_fwd<96>(a, st); break;
    case 128: Launch<T>::template row_fwd<128>(a, st); break;
    case 192: Launch<T>::template row_fwd<192>(a, st); break;
    case 256: Launch<T>::template row_fwd<256>(a, st); break;
    case 384: Launch<T>::template row_fwd<384>(a, st); break;
    case 512: Launch<T>::template row_fwd<512>(a, st); break;
    case 768: Launch<T>::template row_fwd<768>(a, st); break;
    case 1024: Launch<T>::template row_fwd<1024>(a, st); break;
    default: throw Error(-6, "unsupported FFT length " + std::to_string(L));
  }
}
template <typename T>
static void row_inv_call(int L, const RowInvArgs<T>& a, int epi, hipStream_t st) {
  switch (L) {
    case 32: Launch<T>::template row_inv<32>(a, epi, st); break;
    case 48: Launch<T>::template row_inv<48>(a, epi, st); break;
    case 64: Launch<T>::template row_inv<64>(a, epi, st); break;
    case 96: Launch<T>::template row_inv<96>(a, epi, st); break;
    case 128: Launch<T>::template row_inv<128>(a, epi, st); break;
    case 192: Launch<T>::template row_inv<192>(a, epi, st); break;
    case 256: Launch<T>::template row_inv<256>(a, epi, st); break;
    case 384: Launch<T>::template row_inv<384>(a, epi, st); break;
    case 512: Launch<T>::template row_inv<512>(a, epi, st); break;
    case 768: Launch<T>::template row_inv<768>(a, epi, st); break;
    case 1024: Launch<T>::template row_inv<1024>(a, epi, st); break;
    default: throw Error(-6, "unsupported FFT length " + std::to_string(L));
  }
}

template <typename T>
void launch_vie(const Geo& g, const Twiddles& tw, int B, const cplx<T>* x, const cplx<T>* scale, const int* active,
                const cplx<T>* m, const cplx<T>* ghat, const int* rhs_freq, cplx<T>* U1, cplx<T>* U2, cplx<T>* y,
                const cplx<T>* rhs, int epi, hipStream_t st) {
  const long rows_per_rhs = (long)g.nz * g.ny;
  // pass 1: rows along x
  RowFwdArgs<T> f{};
  f.x = x;
  f.m = m;
  f.scale = epi == EPI_RESID ? nullptr : scale;
  f.active = active;
  f.out = U1;
  f.tw = tw.get<T>(g.Lx);
  f.nrows = rows_per_rhs * B;
  f.rows_per_rhs = (int)rows_per_rhs;
  f.nin = g.nx;
  f.in_stride = g.nx;
  row_fwd_call<T>(g.Lx, f, st);
  if (g.dim == 2) {
    // pass 2: columns along z, convolution, in place
    StridedArgs<T> s{};
    s.in = U1;
    s.out = U1;
    s.tw = tw.get<T>(g.Lz);
    s.ghat = ghat;
    s.rhs_freq = rhs_freq;
    s.active = active;
    s.in_ps = s.out_ps = (long)g.nz * g.Lx;
    s.pstride = g.Lx;
    s.gstride = g.npad();
    s.nlines = g.Lx;
    s.planes_per_rhs = 1;
    s.lin = s.lout = g.nz;
    strided_call<T>(g.Lz, s, B, 2, st);
  } else {
    // forward along y: U1 [b][z][ny][Lx] -> U2 [b][z][Ly][Lx]
    StridedArgs<T> s{};
    s.in = U1;
    s.out = U2;
    s.tw = tw.get<T>(g.Ly);
    s.active = active;
    s.in_ps = (long)g.ny * g.Lx;
    s.out_ps = (long)g.Ly * g.Lx;
    s.pstride = g.Lx;
    s.nlines = g.Lx;
    s.planes_per_rhs = g.nz;
    s.lin = g.ny;
    s.lout = g.Ly;
    strided_call<T>(g.Ly, s, (long)B * g.nz, 0, st);
    // convolution along z, in place on U2
    StridedArgs<T> c{};
    c.in = U2;
    c.out = U2;
    c.tw = tw.get<T>(g.Lz);
    c.ghat = ghat;
    c.rhs_freq = rhs_freq;
    c.active = active;
    c.in_ps = c.out_ps = (long)g.nz * g.Ly * g.Lx;
    c.pstride = (long)g.Ly * g.Lx;
    c.gstride = g.npad();
    c.nlines = g.Ly * g.Lx;
    c.planes_per_rhs = 1;
    c.lin = c.lout = g.nz;
    strided_call<T>(g.Lz, c, B, 2, st);
    // inverse along y with crop: U2 -> U1
    StridedArgs<T> v{};
    v.in = U2;
    v.out = U1;
    v.tw = tw.get<T>(g.Ly);
    v.active = active;
    v.in_ps = (long)g.Ly * g.Lx;
    v.out_ps = (long)g.ny * g.Lx;
    v.pstride = g.Lx;
    v.nlines = g.Lx;
    v.planes_per_rhs = g.nz;
    v.lin = g.Ly;
    v.lout = g.ny;
    strided_call<T>(g.Ly, v, (long)B * g.nz, 1, st);
  }
  // last pass: rows along x, inverse, crop, epilogue
  RowInvArgs<T> r{};
  r.in = U1;
  r.x = x;
  r.rhs = rhs;
  r.scale = scale;
  r.active = active;
  r.y = y;
  r.tw = tw.get<T>(g.Lx);
  r.nrows = rows_per_rhs * B;
  r.rows_per_rhs = (int)rows_per_rhs;
  r.nout = g.nx;
  row_inv_call<T>(g.Lx, r, epi, st);
}

void launch_fft_full(const Geo& g, const Twiddles& tw, const c128* in, c128* work, c128* out, hipStream_t st) {
  // rows: in -> work (full length, no padding)
  RowFwdArgs<double> f{};
  f.x = in;
  f.out = (g.dim == 2) ? out : work;
  f.tw = tw.get<double>(g.Lx);
  f.nrows = (long)g.Lz * g.Ly;
  f.rows_per_rhs = (int)f.nrows;
  f.nin = g.Lx;
  f.in_stride = g.Lx;
  row_fwd_call<double>(g.Lx, f, st);
  if (g.dim == 3) {
    StridedArgs<double> s{};
    s.in = work;
    s.out = out;
    s.tw = tw.get<double>(g.Ly);
    s.in_ps = s.out_ps = (long)g.Ly * g.Lx;
    s.pstride = g.Lx;
    s.nlines = g.Lx;
    s.planes_per_rhs = g.Lz;
    s.lin = s.lout = g.Ly;
    strided_call<double>(g.Ly, s, g.Lz, 0, st);
  }
  StridedArgs<double> z{};
  z.in = out;
  z.out = out;
  z.tw = tw.get<double>(g.Lz);
  z.in_ps = z.out_ps = 0;
  z.pstride = (long)g.Ly * g.Lx;
  z.nlines = g.Ly * g.Lx;
  z.planes_per_rhs = 1;
  z.lin = z.lout = g.Lz;
  strided_call<double>(g.Lz, z, 1, 0, st);
}

template <typename T>
void launch_fft_padded(const Geo& g, const Twiddles& tw, const cplx<T>* in, cplx<T>* U1, cplx<T>* out,
                       hipStream_t st) {
  RowFwdArgs<T> f{};
  f.x = in;
  f.out = U1;
  f.tw = tw.get<T>(g.Lx);
  f.nrows = (long)g.nz * g.ny;
  f.rows_per_rhs = (int)f.nrows;
  f.nin = g.nx;
  f.in_stride = g.nx;
  row_fwd_call<T>(g.Lx, f, st);
  const cplx<T>* cur = U1;
  long cur_ny = g.ny;
  if (g.dim == 3) {
    // y pass: U1 [nz][ny][Lx] -> out [nz][Ly][Lx] (rows z < nz), then z pass in place
    StridedArgs<T> s{};
    s.in = U1;
    s.out = out;
    s.tw = tw.get<T>(g.Ly);
    s.in_ps = (long)g.ny * g.Lx;
    s.out_ps = (long)g.Ly * g.Lx;
    s.pstride = g.Lx;
    s.nlines = g.Lx;
    s.planes_per_rhs = g.nz;
    s.lin = g.ny;
    s.lout = g.Ly;
    strided_call<T>(g.Ly, s, g.nz, 0, st);
    cur = out;
    cur_ny = g.Ly;
  }
  StridedArgs<T> z{};
  z.in = cur;
  z.out = out;
  z.tw = tw.get<T>(g.Lz);
  z.in_ps = z.out_ps = 0;
  z.pstride = (long)cur_ny * g.Lx;
  z.nlines = (int)(cur_ny * g.Lx);
  z.planes_per_rhs = 1;
  z.lin = g.nz;
  z.lout = g.Lz;
  strided_call<T>(g.Lz, z, 1, 0, st);
}

template void launch_vie<double>(const Geo&, const Twiddles&, int, const c128*, const c128*, const int*, const c128*,
                                 const c128*, const int*, c128*, c128*, c128*, const c128*, int, hipStream_t);
template void launch_vie<float>(const Geo&, const Twiddles&, int, const c64*, const c64*, const int*, const c64*,
                                const c64*, const int*, c64*, c64*, c64*, const c64*, int, hipStream_t);
template void launch_fft_padded<double>(const Geo&, const Twiddles&, const c128*, c128*, c128*, hipStream_t);
template void launch_fft_padded<float>(const Geo&, const Twiddles&, const c64*, c64*, c64*, hipStream_t);

}  // namespace fwi
