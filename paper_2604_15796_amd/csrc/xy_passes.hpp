// Fused lateral-elevation passes of the 3D operator (Sec. IV-A): one
// workgroup transforms a whole z-plane of one right-hand side, so the
// intermediate between the lateral (x) and the elevation (y) transforms never
// goes to HBM.
//
// The padded transforms split by the parity classes of the output frequency.
// With Lx = 4 MX and the plane zero beyond x = 2 MX (half padding),
//   X[4k + c] = FFT_MX( w_Lx^{x c} (v[x] + (-i)^c v[x + MX]) )[k],   c = 0..3,
// and with Ly = 2 HY and the plane zero beyond y = HY,
//   Y[2m + d] = FFT_HY( w_Ly^{y d} u[y] )[m],                         d = 0, 1,
// (w_L = exp(-2 pi i / L)); the inverses are the conjugate steps,
//   u[y] = sum_d w_Ly^{-y d} IFFT_HY(Y_d)[y]   (y < HY),
//   v[x + q MX] = sum_c w_Lx^{-x c} (+i)^{c q} IFFT_MX(X_c)[x]   (x < MX, q = 0, 1),
// all unnormalised like the line passes. So a class (c, d) is an MX x HY
// block that fits the LDS: the workgroup keeps the plane in registers, and for
// each class modulates it into LDS, transforms the rows (length MX) and the
// columns (length HY) there and writes the block. The padded spectrum is
// stored class-major, lateral frequency 4k + c at column c MX + k and
// elevation frequency 2m + d at row d HY + m; the convolution pass along z
// treats every (row, column) line alike, and the kernel spectrum of such a
// geometry is stored in the same order.
#pragma once

namespace fwi {

// threads per workgroup: 16 plane points per thread (8 rows, two halves of
// the lateral axis), so the plane fits in registers beside one butterfly
__host__ __device__ constexpr int xy_threads(int MX, int HY) {
  return MX * HY / 8 < 64 ? 64 : MX * HY / 8 > 1024 ? 1024 : MX * HY / 8;
}

template <typename T, int MX, int HY>
struct XyCfg {
  static constexpr int NTX = xy_threads(MX, HY);
  using CX = LineCfg<T, MX, HY, NTX, false>;  // HY rows (y) of MX points (k)
  using CY = LineCfg<T, HY, MX, NTX, true>;   // MX columns (k) of HY points (y, m)
  static constexpr int LDS = CX::LDS_ELEMS > CY::LDS_ELEMS ? CX::LDS_ELEMS : CY::LDS_ELEMS;
  __device__ static __forceinline__ int lx(int y, int k) { return CX::lds(y, k); }
  __device__ static __forceinline__ int ly(int k, int y) { return CY::lds(k, y); }
  // plane ownership: thread t holds the points (y, xl) and (y, xl + MX) for
  // xl = t mod MX and y = t / MX + YS i, i < NI
  static constexpr int YS = NTX / MX;
  static constexpr int NI = HY / YS;
  static_assert(NTX % MX == 0 && HY % YS == 0, "plane ownership");
  static_assert(HY * MX * (int)sizeof(double) <= LDS * (int)sizeof(cplx<T>), "row partials fit the LDS tile");
};

template <typename T>
struct XyArgs {
  int nx, ny, nz, Lx, Ly, B;
  const int* active;  // [B] or null: a converged RHS is skipped
  const cplx<T>* twx;  // exp(-2 pi i m / Lx), m < Lx
  const cplx<T>* twy;  // exp(-2 pi i m / Ly)
  const cplx<T>* twm;  // length-MX table
  const cplx<T>* twh;  // length-HY table
  cplx<T>* U2;         // [B][nz][Ly][Lx], class-major
  // forward operand (as RowFwdArgs): x [B][n], m [n] or null
  const cplx<T>* x;
  const cplx<T>* m;
  const cplx<T>* basis;  // RI_ORTH: V_0, vector i at basis + i vs
  long vs;
  int nvec;
  const c128* coef;  // [B][cstride]
  int cstride;
  cplx<T>* xout;      // RI_ORTH / RI_START: the formed vector is stored here
  double* rowpart;    // RI_ORTH / RI_START: |v|^2 per grid row [B][nz ny]
  const c128* src;    // RI_START: the right-hand sides [B][n]
  // inverse epilogue (as RowInvArgs): y = s (x - conv) or y = conv
  const cplx<T>* scale;
  cplx<T>* y;
  // EPI_VIE_DOT: inner products of y with the basis, one part per plane
  const cplx<T>* dbasis;
  long dvs;
  int dnvec;
  const cplx<T>* vscale;
  c128* dotp;
  int dstride;
};

// All stages of a line transform of C, input in the LDS tile in C's layout;
// the first stage works in place (its loads complete before any store), the
// last stage hands its outputs to snk (which may write the tile too).
template <class C, int dir, class Snk>
__device__ __forceinline__ void xy_lds_transform(const cplx<typename C::T>* __restrict__ tw, cplx<typename C::T>* sh,
                                                 Snk&& snk) {
  using T = typename C::T;
  constexpr int S = plan_stages(C::L, C::BIG);
  constexpr int R0 = stage_radix(C::L, dir, 0, C::BIG);
  const int sgn = dir == 0 ? -1 : +1;
  auto rd = [&](int line, int pb, int ro) { return sh[C::lds(line, pb, ro)]; };
  auto wr = [&](int line, int pb, int ro, cplx<T> v) { sh[C::lds(line, pb, ro)] = v; };
  if constexpr (S == 1) {
    fft_stage<C, R0, 1, true, false, false>(sgn, tw, rd, snk);
  } else {
    fft_stage<C, R0, 1, true, false, false>(sgn, tw, rd, wr);
    __syncthreads();
    fft_mid_stages<C, dir, 1, R0>(sgn, tw, sh);
    constexpr int RL = stage_radix(C::L, dir, S - 1, C::BIG);
    constexpr int NsL = ns_before<C::L, C::BIG, dir, S - 1>();
    fft_stage<C, RL, NsL, true, false, false>(sgn, tw, rd, snk);
  }
}

// As xy_lds_transform, with the first stage reading src (global memory).
template <class C, int dir, class Src, class Snk>
__device__ __forceinline__ void xy_src_transform(const cplx<typename C::T>* __restrict__ tw, cplx<typename C::T>* sh,
                                                 Src&& src, Snk&& snk) {
  using T = typename C::T;
  constexpr int S = plan_stages(C::L, C::BIG);
  constexpr int R0 = stage_radix(C::L, dir, 0, C::BIG);
  static_assert(S >= 2, "two or more stages");
  const int sgn = dir == 0 ? -1 : +1;
  auto rd = [&](int line, int pb, int ro) { return sh[C::lds(line, pb, ro)]; };
  auto wr = [&](int line, int pb, int ro, cplx<T> v) { sh[C::lds(line, pb, ro)] = v; };
  fft_stage<C, R0, 1, false, false, false>(sgn, tw, src, wr);
  __syncthreads();
  fft_mid_stages<C, dir, 1, R0>(sgn, tw, sh);
  constexpr int RL = stage_radix(C::L, dir, S - 1, C::BIG);
  constexpr int NsL = ns_before<C::L, C::BIG, dir, S - 1>();
  fft_stage<C, RL, NsL, true, false, false>(sgn, tw, rd, snk);
}

// The pointer itself, hidden from the optimiser: table loads made through
// it inside the class loop stay there (hoisted, every class's twiddles would
// stay live in registers beside the plane).
template <typename P>
__device__ __forceinline__ P xy_opaque(P p) {
#if defined(__HIP_DEVICE_COMPILE__)
  asm volatile("" : "+s"(p));
#endif
  return p;
}

// (-i)^c z (sgn = -1) or (+i)^c z (sgn = +1)
template <typename T>
__device__ __forceinline__ cplx<T> xy_rot(cplx<T> z, int c, int sgn) {
  return c == 0 ? z : c == 2 ? mk(-z.x, -z.y) : mul_i(z, c == 1 ? sgn : -sgn);
}

// The class tile through all stages of C in place.
template <class C, int dir>
__device__ __forceinline__ void xy_inplace(const cplx<typename C::T>* __restrict__ tw, cplx<typename C::T>* sh) {
  using T = typename C::T;
  xy_lds_transform<C, dir>(xy_opaque(tw), sh, [&](int line, int pb, int ro, cplx<T> v) { sh[C::lds(line, pb, ro)] = v; });
  __syncthreads();
}

// The whole class tile from the row-wise to the column-wise layout
// (ROWS_TO_COLS) or back, each thread moving the same elements both ways.
template <typename T, int MX, int HY, bool ROWS_TO_COLS>
__device__ __forceinline__ void xy_relayout(cplx<T>* sh) {
  using Q = XyCfg<T, MX, HY>;
  constexpr int PER = MX * HY / Q::NTX;
  cplx<T> buf[PER];
#pragma unroll
  for (int q = 0; q < PER; ++q) {
    const int e = (int)threadIdx.x + q * Q::NTX, y = e / MX, k = e % MX;
    buf[q] = sh[ROWS_TO_COLS ? Q::lx(y, k) : Q::ly(k, y)];
  }
  __syncthreads();
#pragma unroll
  for (int q = 0; q < PER; ++q) {
    const int e = (int)threadIdx.x + q * Q::NTX, y = e / MX, k = e % MX;
    sh[ROWS_TO_COLS ? Q::ly(k, y) : Q::lx(y, k)] = buf[q];
  }
  __syncthreads();
}

// Forward: the plane's operand (formed per K as in k_row_fwd: RI_PLAIN x,
// RI_ORTH w + sum_i coef_i V_i, stored, with |v|^2 per grid row, RI_START
// the complex128 source rounded to T, stored, with |src|^2 per row), times m,
// to its eight class blocks of U2.
template <typename T, int MX, int HY, int K>
__device__ __forceinline__ void xy_fwd_body(const XyArgs<T>& a, int z, int b, cplx<T>* sh) {
  using Q = XyCfg<T, MX, HY>;
  constexpr int NI = Q::NI, YS = Q::YS, NP = 2 * NI;
  constexpr bool NORM = K == RI_ORTH || K == RI_START;
  const int t = (int)threadIdx.x, xl = t % MX, y0 = t / MX;
  const long n = (long)a.nx * a.ny * a.nz;
  const long mb = (long)z * a.ny * a.nx;  // plane offset in a grid vector
  const long pb = (long)b * n + mb;       // and in RHS b's vector
  // the thread's points: slot k = 2 i + q is (y0 + YS i, xl + q MX); a point
  // outside the plane loads element 0 of it (in bounds) and counts as zero
  auto yk = [&](int k) { return y0 + YS * (k >> 1); };
  auto xk = [&](int k) { return xl + (k & 1) * MX; };
  auto okk = [&](int k) { return yk(k) < a.ny && xk(k) < a.nx; };
  auto ek = [&](int k) { return okk(k) ? yk(k) * a.nx + xk(k) : 0; };
  cplx<T> pv[NP];
  double nrm[NI];
#pragma unroll
  for (int i = 0; i < NI; ++i) nrm[i] = 0.0;
  if constexpr (K == RI_START) {
    const c128* sp = a.src + pb;
#pragma unroll
    for (int k = 0; k < NP; ++k) {
      const c128 sv = sp[ek(k)];
      pv[k] = mk((T)sv.x, (T)sv.y);
      if (okk(k)) nrm[k >> 1] += norm2(sv);
    }
  } else {
    const cplx<T>* xp = a.x + pb;
#pragma unroll
    for (int k = 0; k < NP; ++k) pv[k] = xp[ek(k)];
    if constexpr (K == RI_ORTH) {
      // classical Gram-Schmidt, accumulated in T in the order of k_row_fwd
      for (int j = 0; j < a.nvec; ++j) {
        const c128 cc = a.coef[(long)b * a.cstride + j];
        const cplx<T> cf = mk((T)cc.x, (T)cc.y);
        const cplx<T>* Vj = a.basis + (long)j * a.vs + pb;
#pragma unroll
        for (int k = 0; k < NP; ++k) pv[k] = cfma(cf, Vj[ek(k)], pv[k]);
      }
#pragma unroll
      for (int k = 0; k < NP; ++k)
        if (okk(k)) nrm[k >> 1] += (double)pv[k].x * (double)pv[k].x + (double)pv[k].y * (double)pv[k].y;
    }
  }
  if constexpr (NORM) {
#pragma unroll
    for (int k = 0; k < NP; ++k)
      if (okk(k)) a.xout[pb + ek(k)] = pv[k];
  }
  // times m, branch-free so that every load is in flight at once: without a
  // contrast the operand stands in for m and the blend makes the factor 1
  {
    const T km = a.m ? (T)1 : (T)0;
    const cplx<T>* mp = a.m ? a.m + mb : a.x + pb;
    cplx<T> mv[NP];
#pragma unroll
    for (int k = 0; k < NP; ++k) mv[k] = mp[ek(k)];
#pragma unroll
    for (int k = 0; k < NP; ++k) {
      const cplx<T> u = pv[k] * mk(km * mv[k].x + ((T)1 - km), km * mv[k].y);
      pv[k] = okk(k) ? u : mk((T)0, (T)0);
    }
  }
  if constexpr (NORM) {
    // per grid row, in a fixed order: the row's MX partials through LDS
    double* part = reinterpret_cast<double*>(sh);
#pragma unroll
    for (int i = 0; i < NI; ++i) part[(y0 + YS * i) * MX + xl] = nrm[i];
    __syncthreads();
    for (int y = t; y < a.ny; y += Q::NTX) {
      double s = 0.0;
      for (int q = 0; q < MX; ++q) s += part[y * MX + q];
      a.rowpart[(long)b * a.nz * a.ny + (long)z * a.ny + y] = s;
    }
  }
  cplx<T>* plane = a.U2 + ((long)b * a.nz + z) * a.Ly * a.Lx;
#pragma unroll 1
  for (int c = 0; c < 4; ++c) {
    const cplx<T> wx = xy_opaque(a.twx)[(xl * c) % a.Lx];
#pragma unroll 1
    for (int d = 0; d < 2; ++d) {
      const cplx<T>* twy = xy_opaque(a.twy);
      const cplx<T>* twm = xy_opaque(a.twm);
      const cplx<T>* twh = xy_opaque(a.twh);
      __syncthreads();  // the tile's previous readers are done
#pragma unroll
      for (int i = 0; i < NI; ++i) {
        const int y = y0 + YS * i;
        cplx<T> u = pv[2 * i] + xy_rot(pv[2 * i + 1], c, -1);
        if (c) u = u * wx;
        if (d) u = u * twy[y];
        sh[Q::lx(y, xl)] = u;
      }
      __syncthreads();
      xy_inplace<typename Q::CX, 0>(twm, sh);  // rows: lateral transform
      xy_relayout<T, MX, HY, true>(sh);
      // columns: elevation transform, the last stage writing the class block
      cplx<T>* blk = plane + (long)(d * HY) * a.Lx + c * MX;
      xy_lds_transform<typename Q::CY, 0>(twh, sh,
                                          [&](int k, int pb_, int ro, cplx<T> v) { blk[(long)(pb_ + ro) * a.Lx + k] = v; });
    }
  }
}

// Inverse: the eight class blocks of U2 back to the plane (cropped), then the
// epilogue of k_row_inv: EPI_COPY y = conv, EPI_VIE y = s (x - conv),
// EPI_VIE_DOT the same with the inner products of y and the basis (one part
// per plane).
template <typename T, int MX, int HY, int EPI>
__device__ __forceinline__ void xy_inv_body(const XyArgs<T>& a, int z, int b, cplx<T>* sh, double* red) {
  using Q = XyCfg<T, MX, HY>;
  using CY = typename Q::CY;
  constexpr int NI = Q::NI, YS = Q::YS, NTX = Q::NTX, NP = 2 * NI;
  const int t = (int)threadIdx.x, xl = t % MX, y0 = t / MX;
  cplx<T> acc[NP];  // slot k = 2 i + q: the point (y0 + YS i, xl + q MX)
#pragma unroll
  for (int k = 0; k < NP; ++k) acc[k] = mk((T)0, (T)0);
  const cplx<T>* plane = a.U2 + ((long)b * a.nz + z) * a.Ly * a.Lx;
#pragma unroll 1
  for (int c = 0; c < 4; ++c) {
    const cplx<T> wxc = xy_opaque(a.twx)[(xl * c) % a.Lx];
    const cplx<T> wx = mk(wxc.x, -wxc.y);
#pragma unroll 1
    for (int d = 0; d < 2; ++d) {
      const cplx<T>* twy = xy_opaque(a.twy);
      const cplx<T>* twm = xy_opaque(a.twm);
      const cplx<T>* twh = xy_opaque(a.twh);
      __syncthreads();  // the tile's previous readers are done
      const cplx<T>* blk = plane + (long)(d * HY) * a.Lx + c * MX;
      // columns: inverse elevation transform, first stage from the class block
      xy_src_transform<CY, 1>(
          twh, sh, [&](int k, int pb_, int ro) { return blk[(long)(pb_ + ro) * a.Lx + k]; },
          [&](int k, int pb_, int ro, cplx<T> v) { sh[CY::lds(k, pb_, ro)] = v; });
      __syncthreads();
      xy_relayout<T, MX, HY, false>(sh);
      xy_inplace<typename Q::CX, 1>(twm, sh);  // rows: inverse lateral transform
#pragma unroll
      for (int i = 0; i < NI; ++i) {
        const int y = y0 + YS * i;
        cplx<T> u = sh[Q::lx(y, xl)];
        if (c) u = u * wx;
        if (d) {
          const cplx<T> w = twy[y];
          u = u * mk(w.x, -w.y);
        }
        acc[2 * i] = acc[2 * i] + u;
        acc[2 * i + 1] = acc[2 * i + 1] + xy_rot(u, c, +1);
      }
    }
  }
  const long n = (long)a.nx * a.ny * a.nz;
  const long pb = (long)b * n + (long)z * a.ny * a.nx;
  const cplx<T> s = a.scale ? a.scale[b] : mk((T)1, (T)0);
  auto yk = [&](int k) { return y0 + YS * (k >> 1); };
  auto xk = [&](int k) { return xl + (k & 1) * MX; };
  auto okk = [&](int k) { return yk(k) < a.ny && xk(k) < a.nx; };
  auto ek = [&](int k) { return okk(k) ? yk(k) * a.nx + xk(k) : 0; };
  if constexpr (EPI == EPI_VIE || EPI == EPI_VIE_DOT) {
    cplx<T> xv[NP];
#pragma unroll
    for (int k = 0; k < NP; ++k) xv[k] = a.x[pb + ek(k)];
#pragma unroll
    for (int k = 0; k < NP; ++k) acc[k] = (xv[k] - acc[k]) * s;  // the operator is linear: s (x - conv(m x))
  }
#pragma unroll
  for (int k = 0; k < NP; ++k)
    if (okk(k)) a.y[pb + ek(k)] = acc[k];
  if constexpr (EPI == EPI_VIE_DOT) {
    // one part per plane: fixed-order sums (thread, wave, then the waves)
    const int lane = t & 63, wv = t >> 6;
    for (int j = 0; j < a.dnvec; ++j) {
      const cplx<T>* Vj = a.dbasis + (long)j * a.dvs + pb;
      double r = 0.0, mm = 0.0;
      cplx<T> vv[NP];
#pragma unroll
      for (int k = 0; k < NP; ++k) vv[k] = Vj[ek(k)];
#pragma unroll
      for (int k = 0; k < NP; ++k) {
        const cplx<T> v = vv[k];
        const double vx = okk(k) ? (double)v.x : 0.0, vy = okk(k) ? (double)v.y : 0.0;
        const double yx = acc[k].x, yy = acc[k].y;
        r = fma(vx, yx, r);
        r = fma(vy, yy, r);
        mm = fma(vx, yy, mm);
        mm = fma(-vy, yx, mm);
      }
      r = wave_sum(r);
      mm = wave_sum(mm);
      if (lane == 0) {
        red[(0 * kMaxDotVec + j) * (NTX / 64) + wv] = r;
        red[(1 * kMaxDotVec + j) * (NTX / 64) + wv] = mm;
      }
    }
    __syncthreads();
    if (t < a.dnvec) {
      double r = 0.0, mm = 0.0;
      for (int w = 0; w < NTX / 64; ++w) {
        r += red[(0 * kMaxDotVec + t) * (NTX / 64) + w];
        mm += red[(1 * kMaxDotVec + t) * (NTX / 64) + w];
      }
      const double sc = (double)a.vscale[(long)t * a.B + b].x;  // stored V_i = basis vector / sc
      a.dotp[((long)b * a.nz + z) * a.dstride + t] = mk(sc * r, sc * mm);
    }
  }
}

#ifndef FWI_XY_BODIES_ONLY  // the CPU emulation of the bodies stops here

// workgroup g: plane z = g / B of RHS b = g mod B (the planes of one z run
// back to back, so the contrast plane is reused from L2 across the RHS)
template <typename T, int MX, int HY, int K>
__global__ void __launch_bounds__(xy_threads(MX, HY)) k_xy_fwd(XyArgs<T> a) {
  __shared__ cplx<T> sh[XyCfg<T, MX, HY>::LDS];
  const int z = (int)(blockIdx.x / (unsigned)a.B), b = (int)(blockIdx.x % (unsigned)a.B);
  if (a.active && !a.active[b]) return;  // uniform per workgroup
  xy_fwd_body<T, MX, HY, K>(a, z, b, sh);
}

template <typename T, int MX, int HY, int EPI>
__global__ void __launch_bounds__(xy_threads(MX, HY)) k_xy_inv(XyArgs<T> a) {
  __shared__ cplx<T> sh[XyCfg<T, MX, HY>::LDS];
  __shared__ double red[EPI == EPI_VIE_DOT ? 2 * kMaxDotVec * (XyCfg<T, MX, HY>::NTX / 64) : 1];
  const int z = (int)(blockIdx.x / (unsigned)a.B), b = (int)(blockIdx.x % (unsigned)a.B);
  if (a.active && !a.active[b]) return;  // uniform per workgroup
  xy_inv_body<T, MX, HY, EPI>(a, z, b, sh, red);
}

// The shapes (Lx / 4, Ly / 2) built with fused passes.
#define FWI_XY_SHAPES(FN, T, MXv, HYv, ...)                                \
  do {                                                                     \
    if (MXv == 64 && HYv == 128) FN<T, 64, 128>(__VA_ARGS__);              \
    else if (MXv == 32 && HYv == 64) FN<T, 32, 64>(__VA_ARGS__);           \
    else throw Error(-6, "no fused lateral-elevation pass for this grid"); \
  } while (0)

template <typename T, int MX, int HY>
void launch_xy_fwd_s(const XyArgs<T>& a, int kind, hipStream_t st) {
  constexpr int NTX = XyCfg<T, MX, HY>::NTX;
  const dim3 grid((unsigned)((long)a.nz * a.B)), block(NTX);
  if (kind == RI_ORTH) FWI_TIMED_LAUNCH((k_xy_fwd<T, MX, HY, RI_ORTH>), grid, block, 0, st, a);
  else if (kind == RI_START) FWI_TIMED_LAUNCH((k_xy_fwd<T, MX, HY, RI_START>), grid, block, 0, st, a);
  else FWI_TIMED_LAUNCH((k_xy_fwd<T, MX, HY, RI_PLAIN>), grid, block, 0, st, a);
  FWI_LAUNCH_CHECK();
}
template <typename T, int MX, int HY>
void launch_xy_inv_s(const XyArgs<T>& a, int epi, hipStream_t st) {
  constexpr int NTX = XyCfg<T, MX, HY>::NTX;
  const dim3 grid((unsigned)((long)a.nz * a.B)), block(NTX);
  if (epi == EPI_VIE_DOT) FWI_TIMED_LAUNCH((k_xy_inv<T, MX, HY, EPI_VIE_DOT>), grid, block, 0, st, a);
  else if (epi == EPI_VIE) FWI_TIMED_LAUNCH((k_xy_inv<T, MX, HY, EPI_VIE>), grid, block, 0, st, a);
  else if (epi == EPI_COPY) FWI_TIMED_LAUNCH((k_xy_inv<T, MX, HY, EPI_COPY>), grid, block, 0, st, a);
  else throw Error(-6, "the fused lateral-elevation pass has no residual epilogue");
  FWI_LAUNCH_CHECK();
}

#endif  // FWI_XY_BODIES_ONLY

}  // namespace fwi
