// Line FFTs for the FFT-accelerated Green's-function convolution (Sec. IV-A).
//
// A workgroup transforms NL independent lines of length L held in LDS. Each
// stage is a radix-R Stockham autosort step (the formulation of Govindaraju et
// al., "High performance discrete Fourier transforms on graphics processors",
// SC'08): butterfly j of a line reads points j + r L/R, applies the twiddles
// w_L^{k r L/(Ns R)} with k = j mod Ns, does a length-R DFT in registers and
// writes points (j/Ns) Ns R + k + r Ns. After the last stage the result is in
// natural order, so no bit reversal is ever done. The first stage reads global
// memory directly (zero padding is a load predicate) and the last stage writes
// global memory directly (cropping is a store predicate), so a pass costs one
// read and one write of its data in HBM and S-1 LDS exchanges in between.
//
// Lengths are 2^a 3^b (32 ... 1024) with radices 8, 6, 4, 3; every plan starts
// with radix 8, which makes the zero half of a padded input a whole set of
// predicated-off loads, and the inverse plan is the reverse of the forward one.
#pragma once

#include "common.hpp"

namespace fwi {

// ---------------------------------------------------------------- plans ---
__host__ __device__ constexpr int plan_stages(int L) {
  return L == 32 || L == 48 || L == 64 ? 2
       : L == 96 || L == 128 || L == 192 || L == 256 || L == 384 || L == 512 ? 3
       : L == 768 || L == 1024 ? 4 : 0;
}
__host__ __device__ constexpr int plan_radix(int L, int s) {
  // forward plan, stage s
  return s == 0 ? 8
       : L == 32 ? 4
       : L == 48 ? 6
       : L == 64 ? 8
       : L == 96 ? (s == 1 ? 4 : 3)
       : L == 128 ? 4
       : L == 192 ? (s == 1 ? 8 : 3)
       : L == 256 ? (s == 1 ? 8 : 4)
       : L == 384 ? (s == 1 ? 8 : 6)
       : L == 512 ? 8
       : L == 768 ? (s == 1 ? 8 : s == 2 ? 4 : 3)
       : L == 1024 ? (s == 1 ? 8 : 4) : 0;
}
// radix of stage s of the plan in direction dir (0: forward order, 1: reversed)
__host__ __device__ constexpr int stage_radix(int L, int dir, int s) {
  return dir == 0 ? plan_radix(L, s) : plan_radix(L, plan_stages(L) - 1 - s);
}

// ------------------------------------------------------------ butterflies ---
// In-place length-R DFT of v with exponent sign `sgn` (-1 forward, +1 inverse):
// X_q = sum_r v_r exp(sgn 2 pi i r q / R).
template <typename T>
__device__ __forceinline__ void dft2(cplx<T>& a, cplx<T>& b) {
  cplx<T> t = a - b;
  a = a + b;
  b = t;
}

template <int R, typename T>
__device__ __forceinline__ void dft(cplx<T>* v, int sgn) {
  if constexpr (R == 2) {
    dft2(v[0], v[1]);
  } else if constexpr (R == 3) {
    const T h = (T)0.86602540378443864676;  // sqrt(3)/2
    cplx<T> s = v[1] + v[2];
    cplx<T> d = v[1] - v[2];
    cplx<T> a = v[0];
    v[0] = a + s;
    cplx<T> m = mk(a.x - (T)0.5 * s.x, a.y - (T)0.5 * s.y);
    cplx<T> rot = mul_i(mk(h * d.x, h * d.y), sgn);  // i sgn (sqrt3/2) d
    v[1] = m + rot;
    v[2] = m - rot;
  } else if constexpr (R == 4) {
    cplx<T> a = v[0] + v[2], b = v[0] - v[2];
    cplx<T> c = v[1] + v[3], d = mul_i(v[1] - v[3], sgn);
    v[0] = a + c;
    v[2] = a - c;
    v[1] = b + d;
    v[3] = b - d;
  } else if constexpr (R == 6) {
    // 6 = 3 x 2: X[k1] = A0[k1] + w6^k1 A1[k1], X[k1+3] = A0[k1] - w6^k1 A1[k1]
    cplx<T> e[3] = {v[0], v[2], v[4]};
    cplx<T> o[3] = {v[1], v[3], v[5]};
    dft<3>(e, sgn);
    dft<3>(o, sgn);
    const T h = (T)0.86602540378443864676;
    cplx<T> w1 = mk((T)0.5, (T)sgn * h);    // exp(sgn i pi/3)
    cplx<T> w2 = mk((T)-0.5, (T)sgn * h);   // exp(sgn 2 i pi/3)
    cplx<T> t0 = o[0], t1 = w1 * o[1], t2 = w2 * o[2];
    v[0] = e[0] + t0;
    v[3] = e[0] - t0;
    v[1] = e[1] + t1;
    v[4] = e[1] - t1;
    v[2] = e[2] + t2;
    v[5] = e[2] - t2;
  } else if constexpr (R == 8) {
    // 8 = 2 x 4: even / odd length-4 DFTs, then X_q = E_q + w8^q O_q
    cplx<T> e[4] = {v[0], v[2], v[4], v[6]};
    cplx<T> o[4] = {v[1], v[3], v[5], v[7]};
    dft<4>(e, sgn);
    dft<4>(o, sgn);
    const T r2 = (T)0.70710678118654752440;
    cplx<T> t0 = o[0];
    cplx<T> t1 = mk(r2 * (o[1].x - (T)sgn * o[1].y), r2 * (o[1].y + (T)sgn * o[1].x));   // (1 + i sgn)/sqrt2
    cplx<T> t2 = mul_i(o[2], sgn);
    cplx<T> t3 = mk(r2 * (-o[3].x - (T)sgn * o[3].y), r2 * (-o[3].y + (T)sgn * o[3].x)); // (-1 + i sgn)/sqrt2
    v[0] = e[0] + t0;
    v[4] = e[0] - t0;
    v[1] = e[1] + t1;
    v[5] = e[1] - t1;
    v[2] = e[2] + t2;
    v[6] = e[2] - t2;
    v[3] = e[3] + t3;
    v[7] = e[3] - t3;
  }
}

// v[r] *= w1^r for r = 1 .. R-1, with the powers built by a product tree of
// depth <= 3 from one table value (one load per butterfly instead of R-1).
template <int R, typename T>
__device__ __forceinline__ void apply_twiddles(cplx<T>* v, cplx<T> w1) {
  if constexpr (R >= 2) v[1] = v[1] * w1;
  if constexpr (R >= 3) {
    const cplx<T> w2 = w1 * w1;
    v[2] = v[2] * w2;
    if constexpr (R >= 4) {
      const cplx<T> w3 = w2 * w1;
      v[3] = v[3] * w3;
      if constexpr (R >= 5) {
        const cplx<T> w4 = w2 * w2;
        v[4] = v[4] * w4;
        if constexpr (R >= 6) v[5] = v[5] * (w4 * w1);
        if constexpr (R >= 7) v[6] = v[6] * (w4 * w2);
        if constexpr (R >= 8) v[7] = v[7] * (w4 * w3);
      }
    }
  }
}

// --------------------------------------------------------- line config ---
// NL lines of length L per workgroup of NT threads. LF (line-fastest): the
// butterfly index b maps to (line = b % NL, j = b / NL) and LDS holds point p of
// a line at p*NL + line (strided passes: neighbouring threads touch
// neighbouring columns in HBM). Otherwise j is fastest and LDS holds a line
// contiguously (row passes).
//
// LDS padding: one extra element (row passes) or one extra row of NL elements
// (strided passes) after every 8 points. The first stage of every plan has
// radix 8 and writes points 8j + r, so without padding the 64 lanes of a wave
// would land on a few banks; with it they spread over all of them.
template <typename T_, int L_, int NL_, int NT_, bool LF_>
struct LineCfg {
  using T = T_;
  static constexpr int L = L_, NL = NL_, NT = NT_;
  static constexpr bool LF = LF_;
  static constexpr int LP = L + L / 8;  // padded line length (points)
  static constexpr int LDS_ELEMS = NL * LP;
  __device__ static __forceinline__ int lds(int line, int p) {
    return LF ? (p + (p >> 3)) * NL + line : line * LP + p + (p >> 3);
  }
  template <int R>
  __device__ static __forceinline__ void split(int b, int& line, int& j) {
    if constexpr (LF) {
      line = b % NL;
      j = b / NL;
    } else {
      j = b % (L / R);
      line = b / (L / R);
    }
  }
};

// One Stockham stage: loads R points per butterfly through src(line, p), then
// (after an optional barrier) twiddles, transforms and stores through
// snk(line, p, value). Twiddle table tw[m] = exp(-2 pi i m / L).
template <class C, int R, int Ns, bool SYNC, class Src, class Snk>
__device__ __forceinline__ void fft_stage(int sgn, const cplx<typename C::T>* __restrict__ tw, Src&& src, Snk&& snk) {
  using T = typename C::T;
  constexpr int L = C::L, NB = C::NL * (L / R), TT = (NB + C::NT - 1) / C::NT;
  cplx<T> v[TT][R];
#pragma unroll
  for (int t = 0; t < TT; ++t) {
    const int b = threadIdx.x + t * C::NT;
    if (NB % C::NT == 0 || b < NB) {
      int line, j;
      C::template split<R>(b, line, j);
#pragma unroll
      for (int r = 0; r < R; ++r) v[t][r] = src(line, j + r * (L / R));
    }
  }
  if constexpr (SYNC) __syncthreads();
#pragma unroll
  for (int t = 0; t < TT; ++t) {
    const int b = threadIdx.x + t * C::NT;
    if (NB % C::NT == 0 || b < NB) {
      int line, j;
      C::template split<R>(b, line, j);
      const int k = j % Ns;
      if constexpr (Ns > 1) {
        cplx<T> w1 = tw[k * (L / (Ns * R))];
        if (sgn > 0) w1.y = -w1.y;
        apply_twiddles<R>(v[t], w1);
      }
      dft<R>(v[t], sgn);
      const int base = (j / Ns) * Ns * R + k;
#pragma unroll
      for (int r = 0; r < R; ++r) snk(line, base + r * Ns, v[t][r]);
    }
  }
}

// Middle of a convolution: last forward stage (radix R, Ns = L/R), pointwise
// multiply by the kernel spectrum gh(line, p), first inverse stage (radix R,
// Ns = 1). The last forward stage leaves butterfly j holding points
// j + r L/R, which are exactly the inputs of inverse butterfly j.
template <class C, int R, class Src, class Gh, class Snk>
__device__ __forceinline__ void fft_conv_mid(const cplx<typename C::T>* __restrict__ tw, Src&& src, Gh&& gh, Snk&& snk) {
  using T = typename C::T;
  constexpr int L = C::L, Ns = L / R, NB = C::NL * (L / R), TT = (NB + C::NT - 1) / C::NT;
  cplx<T> v[TT][R];
#pragma unroll
  for (int t = 0; t < TT; ++t) {
    const int b = threadIdx.x + t * C::NT;
    if (NB % C::NT == 0 || b < NB) {
      int line, j;
      C::template split<R>(b, line, j);
#pragma unroll
      for (int r = 0; r < R; ++r) v[t][r] = src(line, j + r * (L / R));
    }
  }
  __syncthreads();
#pragma unroll
  for (int t = 0; t < TT; ++t) {
    const int b = threadIdx.x + t * C::NT;
    if (NB % C::NT == 0 || b < NB) {
      int line, j;
      C::template split<R>(b, line, j);
      apply_twiddles<R>(v[t], tw[j]);  // k = j < Ns, twiddle step 1
      dft<R>(v[t], -1);
#pragma unroll
      for (int r = 0; r < R; ++r) v[t][r] = v[t][r] * gh(t, r, line, j + r * Ns);
      dft<R>(v[t], +1);
#pragma unroll
      for (int r = 0; r < R; ++r) snk(line, j * R + r, v[t][r]);
    }
  }
}

// LDS -> LDS stages s .. S-2 of direction dir (the last stage is done by the caller).
template <class C, int dir, int s, int Ns>
__device__ __forceinline__ void fft_mid_stages(int sgn, const cplx<typename C::T>* __restrict__ tw,
                                               cplx<typename C::T>* sh) {
  constexpr int S = plan_stages(C::L);
  if constexpr (s < S - 1) {
    constexpr int R = stage_radix(C::L, dir, s);
    fft_stage<C, R, Ns, true>(
        sgn, tw, [&](int line, int p) { return sh[C::lds(line, p)]; },
        [&](int line, int p, cplx<typename C::T> v) { sh[C::lds(line, p)] = v; });
    __syncthreads();
    fft_mid_stages<C, dir, s + 1, Ns * R>(sgn, tw, sh);
  }
}

// Ns before stage s of direction dir
template <int L, int dir, int s>
__host__ __device__ constexpr int ns_before() {
  if constexpr (s == 0) return 1;
  else return ns_before<L, dir, s - 1>() * stage_radix(L, dir, s - 1);
}

// Full forward/inverse transform: first stage from src (global), middle stages
// in LDS, last stage to snk (global). dir 0 = forward plan (sgn -1), 1 = inverse.
template <class C, int dir, class Src, class Snk>
__device__ __forceinline__ void fft_line_transform(const cplx<typename C::T>* __restrict__ tw, cplx<typename C::T>* sh,
                                                   Src&& src, Snk&& snk) {
  using T = typename C::T;
  constexpr int S = plan_stages(C::L);
  const int sgn = dir == 0 ? -1 : +1;
  constexpr int R0 = stage_radix(C::L, dir, 0);
  fft_stage<C, R0, 1, false>(sgn, tw, src, [&](int line, int p, cplx<T> v) { sh[C::lds(line, p)] = v; });
  __syncthreads();
  fft_mid_stages<C, dir, 1, R0>(sgn, tw, sh);
  constexpr int RL = stage_radix(C::L, dir, S - 1);
  constexpr int NsL = ns_before<C::L, dir, S - 1>();
  fft_stage<C, RL, NsL, false>(sgn, tw, [&](int line, int p) { return sh[C::lds(line, p)]; }, snk);
}

// Points of the convolution middle stage held by this thread: butterfly t,
// leg r -> (line, p). Used to prefetch the kernel spectrum into registers.
template <class C>
struct ConvMidMap {
  static constexpr int S = plan_stages(C::L);
  static constexpr int R = stage_radix(C::L, 0, S - 1);
  static constexpr int NB = C::NL * (C::L / R);
  static constexpr int TT = (NB + C::NT - 1) / C::NT;
  __device__ static __forceinline__ bool at(int t, int r, int& line, int& p) {
    const int b = threadIdx.x + t * C::NT;
    if (!(NB % C::NT == 0 || b < NB)) return false;
    int j;
    C::template split<R>(b, line, j);
    p = j + r * (C::L / R);
    return true;
  }
};

// Convolution along a line: forward (from src), multiply by gh, inverse (to snk).
template <class C, class Src, class Gh, class Snk>
__device__ __forceinline__ void fft_line_convolve(const cplx<typename C::T>* __restrict__ tw, cplx<typename C::T>* sh,
                                                  Src&& src, Gh&& gh, Snk&& snk) {
  using T = typename C::T;
  constexpr int S = plan_stages(C::L);
  constexpr int R0 = stage_radix(C::L, 0, 0);
  fft_stage<C, R0, 1, false>(-1, tw, src, [&](int line, int p, cplx<T> v) { sh[C::lds(line, p)] = v; });
  __syncthreads();
  fft_mid_stages<C, 0, 1, R0>(-1, tw, sh);
  constexpr int RL = stage_radix(C::L, 0, S - 1);
  fft_conv_mid<C, RL>(tw, [&](int line, int p) { return sh[C::lds(line, p)]; }, gh,
                      [&](int line, int p, cplx<T> v) { sh[C::lds(line, p)] = v; });
  __syncthreads();
  // inverse plan is the reverse of the forward plan; its first stage (radix RL) is done
  fft_mid_stages<C, 1, 1, RL>(+1, tw, sh);
  constexpr int RI = stage_radix(C::L, 1, S - 1);
  constexpr int NsI = ns_before<C::L, 1, S - 1>();
  fft_stage<C, RI, NsI, false>(+1, tw, [&](int line, int p) { return sh[C::lds(line, p)]; }, snk);
}

}  // namespace fwi
