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
// Lengths are 2^a 3^b (32 ... 1024) with radices 8, 6, 4, 3, or 32, 16 and 12
// for tiles with many points per thread; every plan starts with a radix of at
// least 8, which makes the zero half of a padded input a whole set of
// predicated-off loads, and the inverse plan is the reverse of the forward one.
#pragma once

#include <type_traits>

#include "common.hpp"

namespace fwi {

// A stage source is called as src(line, pb, ro), or, if it takes them, with
// the butterfly slot t and leg r of the calling thread as well (sources that
// hold values prepared per slot in registers).
template <class Src>
__device__ __forceinline__ auto stage_load(Src& src, int line, int pb, int ro, int t, int r) {
  if constexpr (std::is_invocable_v<Src&, int, int, int, int, int>) return src(line, pb, ro, t, r);
  else return src(line, pb, ro);
}

// ---------------------------------------------------------------- plans ---
// Two plan families: radices 8/6/4/3 (any tile), and for tiles holding at
// least big_ppt(L) points per thread, radices 32/16/12 with fewer stages
// (fewer LDS exchanges and barriers, fewer twiddled points). Length 192 has
// a 16 x 12 plan for the strided (line-fastest) tiles only; length 768 an
// 8 x 8 x 12 plan (three stages instead of 8 x 8 x 4 x 3).
__host__ __device__ constexpr int big_ppt(int L, bool lf = true) {
  return L == 512 || L == 1024 ? 32
       : (L == 128 || L == 256) ? 16
       : L == 768 ? 12
       : (L == 192 && lf) ? 12 : 1 << 30;
}
__host__ __device__ constexpr int plan_stages(int L, bool big = false) {
  return big ? (L == 768 ? 3 : 2)
       : L == 32 || L == 48 || L == 64 ? 2
       : L == 96 || L == 128 || L == 192 || L == 256 || L == 384 || L == 512 ? 3
       : L == 768 || L == 1024 ? 4 : 0;
}
__host__ __device__ constexpr int plan_radix(int L, int s, bool big = false) {
  // forward plan, stage s
  return big ? (L == 128 ? (s == 0 ? 16 : 8)
              : L == 192 ? (s == 0 ? 16 : 12)
              : L == 256 ? 16
              : L == 512 ? (s == 0 ? 16 : 32)
              : L == 768 ? (s == 2 ? 12 : 8)
              : L == 1024 ? 32 : 0)
       : s == 0 ? 8
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
// Twiddle power tables (convolution passes): a twiddled stage with radix R
// stores the powers w^1 .. w^(R-1) of each butterfly class k < Ns in a row of
// pow_stride(R) slots (R - 1 rounded up to a power of two, so rows stay
// aligned for 16-byte LDS loads).
__host__ __device__ constexpr int pow_stride(int R) {
  return R <= 2 ? 1 : R <= 3 ? 2 : R <= 5 ? 4 : R <= 9 ? 8 : R <= 17 ? 16 : 32;
}
// radix of stage s of the plan in direction dir (0: forward order, 1: reversed)
__host__ __device__ constexpr int stage_radix(int L, int dir, int s, bool big = false) {
  return dir == 0 ? plan_radix(L, s, big) : plan_radix(L, plan_stages(L, big) - 1 - s, big);
}

// exp(sgn 2 pi i m / 32) for compile-time m (after unrolling)
__host__ __device__ constexpr double cos32(int m) {
  constexpr double t[32] = {1.0, 0.9807852804032304, 0.9238795325112867, 0.8314696123025452, 0.7071067811865476, 0.5555702330196023, 0.38268343236508984, 0.19509032201612833, 6.123233995736766e-17, -0.1950903220161282, -0.3826834323650897, -0.555570233019602, -0.7071067811865475, -0.8314696123025453, -0.9238795325112867, -0.9807852804032304, -1.0, -0.9807852804032304, -0.9238795325112868, -0.8314696123025455, -0.7071067811865477, -0.5555702330196022, -0.38268343236509034, -0.19509032201612866, -1.8369701987210297e-16, 0.1950903220161283, 0.38268343236509, 0.5555702330196018, 0.7071067811865474, 0.8314696123025452, 0.9238795325112865, 0.9807852804032303};
  return t[m & 31];
}
__host__ __device__ constexpr double sin32(int m) {
  constexpr double t[32] = {0.0, 0.19509032201612825, 0.3826834323650898, 0.5555702330196022, 0.7071067811865475, 0.8314696123025452, 0.9238795325112867, 0.9807852804032304, 1.0, 0.9807852804032304, 0.9238795325112867, 0.8314696123025455, 0.7071067811865476, 0.5555702330196022, 0.3826834323650899, 0.1950903220161286, 1.2246467991473532e-16, -0.19509032201612836, -0.38268343236508967, -0.555570233019602, -0.7071067811865475, -0.8314696123025452, -0.9238795325112865, -0.9807852804032303, -1.0, -0.9807852804032304, -0.9238795325112866, -0.8314696123025455, -0.7071067811865477, -0.5555702330196022, -0.3826834323650904, -0.19509032201612872};
  return t[m & 31];
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

template <int R1, int R2, typename T>
__device__ __forceinline__ void dft_ct(cplx<T>* v, int sgn);
template <typename T>
__device__ __forceinline__ cplx<T> rot32(cplx<T> a, int m, int sgn);

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
  } else if constexpr (R == 12) {
    // prime-factor split 12 = 3 x 4 (Good-Thomas): input n = 4 n1 + 3 n2,
    // output k = 4 k1 + 9 k2 (mod 12), i.e. k = k1 mod 3 and k = k2 mod 4, so
    // the kernel exp(sgn 2 pi i n k / 12) factors into a 3-point and a
    // 4-point one with no twiddles in between
    cplx<T> a[4][3];
#pragma unroll
    for (int n2 = 0; n2 < 4; ++n2) {
#pragma unroll
      for (int n1 = 0; n1 < 3; ++n1) a[n2][n1] = v[(4 * n1 + 3 * n2) % 12];
      dft<3>(a[n2], sgn);
    }
#pragma unroll
    for (int k1 = 0; k1 < 3; ++k1) {
      cplx<T> b[4] = {a[0][k1], a[1][k1], a[2][k1], a[3][k1]};
      dft<4>(b, sgn);
#pragma unroll
      for (int k2 = 0; k2 < 4; ++k2) v[(4 * k1 + 9 * k2) % 12] = b[k2];
    }
  } else if constexpr (R == 16) {
    dft_ct<4, 4>(v, sgn);
  } else if constexpr (R == 32) {
    dft_ct<8, 4>(v, sgn);
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

// Length R1*R2 DFT by one Cooley-Tukey split: n = R2 n1 + n2, k = k1 + R1 k2;
// R1-point DFTs over n1, internal twiddles w_R^{n2 k1} (compile-time
// constants), R2-point DFTs over n2.
template <int R1, int R2, typename T>
__device__ __forceinline__ void dft_ct(cplx<T>* v, int sgn) {
  constexpr int R = R1 * R2;
  cplx<T> a[R2][R1];
#pragma unroll
  for (int n2 = 0; n2 < R2; ++n2) {
#pragma unroll
    for (int n1 = 0; n1 < R1; ++n1) a[n2][n1] = v[R2 * n1 + n2];
    dft<R1>(a[n2], sgn);
#pragma unroll
    for (int k1 = 1; k1 < R1; ++k1) {
      a[n2][k1] = rot32(a[n2][k1], n2 * k1 * (32 / R), sgn);
    }
  }
#pragma unroll
  for (int k1 = 0; k1 < R1; ++k1) {
    cplx<T> b[R2];
#pragma unroll
    for (int n2 = 0; n2 < R2; ++n2) b[n2] = a[n2][k1];
    dft<R2>(b, sgn);
#pragma unroll
    for (int k2 = 0; k2 < R2; ++k2) v[k1 + R1 * k2] = b[k2];
  }
}

// a * exp(sgn 2 pi i m / 32) for a compile-time m (after unrolling)
template <typename T>
__device__ __forceinline__ cplx<T> rot32(cplx<T> a, int m, int sgn) {
  m &= 31;
  if (m == 0) return a;
  if (m == 8) return mul_i(a, sgn);
  if (m == 16) return mk(-a.x, -a.y);
  if (m == 24) return mul_i(a, -sgn);
  return a * mk((T)cos32(m), (T)(sgn * sin32(m)));
}

// Length-R DFT of a vector whose legs R/2 .. R-1 are zero (a first stage over
// zero-padded data): even outputs are the R/2-point DFT of the nonzero half,
// odd outputs the R/2-point DFT of it times w_R^r.
template <int R, typename T>
__device__ __forceinline__ void dft_half_in(cplx<T>* v, int sgn) {
  static_assert(R == 8 || R == 16 || R == 32, "half-input DFT radix");
  constexpr int H = R / 2;
  cplx<T> e[H], o[H];
#pragma unroll
  for (int r = 0; r < H; ++r) {
    e[r] = v[r];
    o[r] = rot32(v[r], r * (32 / R), sgn);
  }
  dft<H>(e, sgn);
  dft<H>(o, sgn);
#pragma unroll
  for (int m = 0; m < H; ++m) {
    v[2 * m] = e[m];
    v[2 * m + 1] = o[m];
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

// Radix 12 / 16 / 32: w^r = (w^8)^(r div 8) w^(r mod 8) from two table values.
template <int R, typename T>
__device__ __forceinline__ void apply_twiddles_big(cplx<T>* v, cplx<T> w1, cplx<T> w8) {
  cplx<T> p[8];
  p[1] = w1;
  p[2] = w1 * w1;
  p[3] = p[2] * w1;
  p[4] = p[2] * p[2];
  p[5] = p[4] * w1;
  p[6] = p[4] * p[2];
  p[7] = p[4] * p[3];
  cplx<T> q[(R + 7) / 8];
  if constexpr (R > 8) q[1] = w8;
  if constexpr (R / 8 > 2) {
    q[2] = w8 * w8;
    q[3] = q[2] * w8;
  }
#pragma unroll
  for (int r = 1; r < R; ++r) {
    const int lo = r & 7, hi = r >> 3;
    if (hi == 0) v[r] = v[r] * p[lo];
    else if (lo == 0) v[r] = v[r] * q[hi];
    else v[r] = v[r] * (q[hi] * p[lo]);
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
// radix 8 or more and writes points R j + r, so without padding the 64 lanes
// of a wave would land on a few banks; with it they spread over all of them.
// Strided tiles whose row of NL points spans 128 bytes or more need no
// padding: the 16 lanes served together are the NL lines of one point (or
// part of them), contiguous in LDS, and every index is then a per-thread base
// plus a compile-time offset (no per-point padding arithmetic).
template <typename T_, int L_, int NL_, int NT_, bool LF_>
struct LineCfg {
  using T = T_;
  static constexpr int L = L_, NL = NL_, NT = NT_;
  static constexpr bool LF = LF_;
  static constexpr bool PAD = !LF || NL * (int)sizeof(cplx<T>) < 128;
  static constexpr int LP = PAD ? L + L / 8 : L;  // padded line length (points)
  static constexpr bool BIG = NL * L / NT >= big_ppt(L, LF);  // radix-32/16/12 plan
  static constexpr int LDS_ELEMS = NL * LP;
  __device__ static __forceinline__ int pad(int p) { return PAD ? p + (p >> 3) : p; }
  __device__ static __forceinline__ int lds(int line, int p) { return LF ? pad(p) * NL + line : line * LP + pad(p); }
  // LDS index of point pb + ro, where ro is a compile-time offset and (for a
  // padded layout) ro or pb is a multiple of 8: the padding term splits and ro
  // becomes an immediate offset of the LDS instruction.
  __device__ static __forceinline__ int lds(int line, int pb, int ro) {
    return lds(line, pb) + pad(ro) * (LF ? NL : 1);
  }
  // (line, j) of butterfly t of this thread in a radix-R stage; the butterfly
  // index is threadIdx.x + t NT.
  template <int R>
  __device__ static __forceinline__ void split(int t, int& line, int& j) {
    if constexpr (LF) {
      static_assert(NT % NL == 0, "lines must divide the workgroup");
      line = (int)threadIdx.x % NL;  // fixed for the thread
      j = (int)threadIdx.x / NL + t * (NT / NL);
    } else if constexpr (NT % (L / R) == 0) {
      j = (int)threadIdx.x % (L / R);
      line = (int)threadIdx.x / (L / R) + t * (NT / (L / R));
    } else {
      const int b = (int)threadIdx.x + t * NT;
      j = b % (L / R);
      line = b / (L / R);
    }
  }
};

// One Stockham stage: loads R points per butterfly through src(line, pb, ro)
// (see stage_load), then (after an optional barrier) twiddles, transforms and
// stores through
// snk(line, pb, ro, value); the point index is pb + ro with ro a compile-time
// offset (see LineCfg::lds). Twiddle table tw[m] = exp(-2 pi i m / L).
// HIN: legs R/2 .. R-1 are zero and not loaded (first stage over zero-padded
// data). HOUT: only legs 0 .. R/2-1 are stored (last stage of a cropped
// transform), so the rest of the butterfly is never computed.
// PT: the stage's twiddle powers come from a power table in LDS (pt, see
// pow_stride), not from one table value and a product tree. hook() runs after
// the stage has issued its loads and before it waits for them: further loads
// issued there (a prefetch) are in flight with the stage's own and are not
// waited for by its butterflies.
struct NoHook {
  __device__ void operator()() const {}
};
template <class C, int R, int Ns, bool SYNC, bool HIN, bool HOUT, bool PT = false, class Src, class Snk,
          class Hook = NoHook>
__device__ __forceinline__ void fft_stage(int sgn, const cplx<typename C::T>* __restrict__ tw, Src&& src, Snk&& snk,
                                          const cplx<typename C::T>* pt = nullptr, Hook&& hook = Hook()) {
  using T = typename C::T;
  constexpr int L = C::L, NB = C::NL * (L / R), TT = (NB + C::NT - 1) / C::NT;
  static_assert(!HIN || Ns == 1, "zero legs only in a first stage");
  static_assert(!HOUT || Ns * R == L, "cropping only in a last stage");
  static_assert(!PT || R <= 16, "power tables for radices up to 16");
  constexpr int RIN = HIN ? R / 2 : R, ROUT = HOUT ? R / 2 : R;
  constexpr bool RD_SPLIT = (L / R) % 8 == 0;
  constexpr bool WR_SPLIT = Ns % 8 == 0 || (Ns == 1 && R % 8 == 0);
  cplx<T> v[TT][R];
  cplx<T> tw1[TT], tw8[TT];  // twiddle table values, loaded with the data
#pragma unroll
  for (int t = 0; t < TT; ++t) {
    if (NB % C::NT == 0 || (int)threadIdx.x + t * C::NT < NB) {
      int line, j;
      C::template split<R>(t, line, j);
#pragma unroll
      for (int r = 0; r < RIN; ++r)
        v[t][r] = RD_SPLIT ? stage_load(src, line, j, r * (L / R), t, r) : stage_load(src, line, j + r * (L / R), 0, t, r);
      if constexpr (Ns > 1 && !PT) {
        const int k = j % Ns;
        tw1[t] = tw[k * (L / (Ns * R))];
        if constexpr (R > 8) tw8[t] = tw[8 * k * (L / (Ns * R))];
      }
    }
  }
  hook();
  if constexpr (SYNC) __syncthreads();
#pragma unroll
  for (int t = 0; t < TT; ++t) {
    if (NB % C::NT == 0 || (int)threadIdx.x + t * C::NT < NB) {
      int line, j;
      C::template split<R>(t, line, j);
      const int k = j % Ns;
      if constexpr (Ns > 1 && PT) {
        const cplx<T>* pw = pt + k * pow_stride(R);
#pragma unroll
        for (int r = 1; r < R; ++r) v[t][r] = v[t][r] * pw[r - 1];
      } else if constexpr (Ns > 1) {
        cplx<T> w1 = tw1[t];
        if (sgn > 0) w1.y = -w1.y;
        if constexpr (R > 8) {
          cplx<T> w8 = tw8[t];
          if (sgn > 0) w8.y = -w8.y;
          apply_twiddles_big<R>(v[t], w1, w8);
        } else {
          apply_twiddles<R>(v[t], w1);
        }
      }
      if constexpr (HIN) dft_half_in<R>(v[t], sgn);
      else dft<R>(v[t], sgn);
      const int base = (j / Ns) * Ns * R + k;
#pragma unroll
      for (int r = 0; r < ROUT; ++r) {
        if constexpr (WR_SPLIT) snk(line, base, r * Ns, v[t][r]);
        else snk(line, base + r * Ns, 0, v[t][r]);
      }
    }
  }
}

// Middle of a convolution: last forward stage (radix R, Ns = L/R), pointwise
// multiply by the kernel spectrum gh(t, r, line, p), first inverse stage
// (radix R, Ns = 1). The last forward stage leaves butterfly j holding points
// j + r L/R, which are exactly the inputs of inverse butterfly j.
template <class C, int R, bool PT = false, class Src, class Gh, class Snk>
__device__ __forceinline__ void fft_conv_mid(const cplx<typename C::T>* __restrict__ tw, Src&& src, Gh&& gh, Snk&& snk,
                                             const cplx<typename C::T>* pt = nullptr) {
  using T = typename C::T;
  constexpr int L = C::L, Ns = L / R, NB = C::NL * (L / R), TT = (NB + C::NT - 1) / C::NT;
  constexpr bool RD_SPLIT = (L / R) % 8 == 0;
  cplx<T> v[TT][R];
  cplx<T> tw1[TT], tw8[TT];  // twiddle table values, loaded with the data
#pragma unroll
  for (int t = 0; t < TT; ++t) {
    if (NB % C::NT == 0 || (int)threadIdx.x + t * C::NT < NB) {
      int line, j;
      C::template split<R>(t, line, j);
#pragma unroll
      for (int r = 0; r < R; ++r)
        v[t][r] = RD_SPLIT ? stage_load(src, line, j, r * (L / R), t, r) : stage_load(src, line, j + r * (L / R), 0, t, r);
      if constexpr (!PT) {
        tw1[t] = tw[j];  // k = j < Ns, step 1
        if constexpr (R > 8) tw8[t] = tw[8 * j];
      }
    }
  }
  __syncthreads();
#pragma unroll
  for (int t = 0; t < TT; ++t) {
    if (NB % C::NT == 0 || (int)threadIdx.x + t * C::NT < NB) {
      int line, j;
      C::template split<R>(t, line, j);
      if constexpr (PT) {
        static_assert(R <= 16, "power tables for radices up to 16");
        const cplx<T>* pw = pt + j * pow_stride(R);
#pragma unroll
        for (int r = 1; r < R; ++r) v[t][r] = v[t][r] * pw[r - 1];
      } else if constexpr (R > 8) {
        apply_twiddles_big<R>(v[t], tw1[t], tw8[t]);
      } else {
        apply_twiddles<R>(v[t], tw1[t]);
      }
      dft<R>(v[t], -1);
#pragma unroll
      for (int r = 0; r < R; ++r) v[t][r] = v[t][r] * gh(t, r, line, j + r * Ns);
      dft<R>(v[t], +1);
#pragma unroll
      for (int r = 0; r < R; ++r) {
        if constexpr (R % 8 == 0) snk(line, j * R, r, v[t][r]);
        else snk(line, j * R + r, 0, v[t][r]);
      }
    }
  }
}

// LDS -> LDS stages s .. S-2 of direction dir (the last stage is done by the caller).
// Ns before stage s of direction dir
template <int L, bool BIG, int dir, int s>
__host__ __device__ constexpr int ns_before() {
  if constexpr (s == 0) return 1;
  else return ns_before<L, BIG, dir, s - 1>() * stage_radix(L, dir, s - 1, BIG);
}

// Power table of a convolution (forward plan, then the reversed inverse
// plan): the rows of stage (dir, s), s >= 1, start at pow_off<L, BIG, dir,
// s>() (multiples of 8 slots), one row per butterfly class k < Ns; row k holds
// w^(k r L / (Ns R)) for r = 1 .. R-1 with the stage's sign (conjugated in
// the inverse plan). pow_off<L, BIG, 1, S>() is the table size.
template <int L, bool BIG, int dir, int s>
__host__ __device__ constexpr int pow_off() {
  if constexpr (dir == 0 && s <= 1) {
    return 0;
  } else if constexpr (dir == 1 && s <= 1) {
    return pow_off<L, BIG, 0, plan_stages(L, BIG)>();
  } else {
    constexpr int size = ns_before<L, BIG, dir, s - 1>() * pow_stride(stage_radix(L, dir, s - 1, BIG));
    return (pow_off<L, BIG, dir, s - 1>() + size + 7) / 8 * 8;
  }
}
template <int L, bool BIG, int s = 0>
__host__ __device__ constexpr int plan_max_radix() {
  if constexpr (s >= plan_stages(L, BIG)) {
    return 0;
  } else {
    constexpr int r = plan_radix(L, s, BIG), rest = plan_max_radix<L, BIG, s + 1>();
    return r > rest ? r : rest;
  }
}
template <class C>
__host__ __device__ constexpr int pow_table_size() {
  return pow_off<C::L, C::BIG, 1, plan_stages(C::L, C::BIG)>();
}
// The table is built in two halves: pow_load issues the table loads into
// registers (one slot per thread and iteration, so that no wave carries the
// whole table; a thread per row, filling R - 1 slots, measured slower), and
// pow_store writes them to LDS later, so that their latency overlaps other
// work. pow_regs<C>() registers per thread hold the values in between.
template <class C, int dir = 0, int s = 1>
__host__ __device__ constexpr int pow_regs() {
  constexpr int S = plan_stages(C::L, C::BIG);
  if constexpr (s < S) {
    constexpr int slots = ns_before<C::L, C::BIG, dir, s>() * pow_stride(stage_radix(C::L, dir, s, C::BIG));
    return (slots + C::NT - 1) / C::NT + pow_regs<C, dir, s + 1>();
  } else if constexpr (dir == 0) {
    return pow_regs<C, 1, 1>();
  } else {
    return 0;
  }
}
template <class C, bool STORE, int dir = 0, int s = 1, int K = 0>
__device__ __forceinline__ void pow_fill(const cplx<typename C::T>* __restrict__ tw, cplx<typename C::T>* tab,
                                         cplx<typename C::T>* rv) {
  constexpr int S = plan_stages(C::L, C::BIG);
  if constexpr (s < S) {
    constexpr int R = stage_radix(C::L, dir, s, C::BIG), Ns = ns_before<C::L, C::BIG, dir, s>();
    constexpr int SR = pow_stride(R), OFF = pow_off<C::L, C::BIG, dir, s>(), STEP = C::L / (Ns * R);
    constexpr int IT = (Ns * SR + C::NT - 1) / C::NT;
#pragma unroll
    for (int q = 0; q < IT; ++q) {
      const int i = (int)threadIdx.x + q * C::NT;
      const int k = i / SR, r = i % SR + 1;
      const bool used = i < Ns * SR && r < R;
      if constexpr (STORE) {
        cplx<typename C::T> w = rv[K + q];
        if (dir == 1) w.y = -w.y;  // here, not at the load: nothing waits for the load before the store
        if (used) tab[OFF + i] = w;
      } else {
        // unconditional (a spare slot loads entry 0), so that no branch
        // around a load makes the compiler wait for it early
        rv[K + q] = tw[used ? k * r * STEP : 0];  // k r STEP < L
      }
    }
    pow_fill<C, STORE, dir, s + 1, K + IT>(tw, tab, rv);
  } else if constexpr (dir == 0) {
    pow_fill<C, STORE, 1, 1, K>(tw, tab, rv);
  }
}

// LDS -> LDS stages s .. S-2 of direction dir (the last stage is done by the
// caller); PT: twiddle powers from the power table tab.
template <class C, int dir, int s, int Ns, bool PT = false>
__device__ __forceinline__ void fft_mid_stages(int sgn, const cplx<typename C::T>* __restrict__ tw,
                                               cplx<typename C::T>* sh, const cplx<typename C::T>* tab = nullptr) {
  constexpr int S = plan_stages(C::L, C::BIG);
  if constexpr (s < S - 1) {
    constexpr int R = stage_radix(C::L, dir, s, C::BIG);
    fft_stage<C, R, Ns, true, false, false, PT>(
        sgn, tw, [&](int line, int pb, int ro) { return sh[C::lds(line, pb, ro)]; },
        [&](int line, int pb, int ro, cplx<typename C::T> v) { sh[C::lds(line, pb, ro)] = v; },
        PT ? tab + pow_off<C::L, C::BIG, dir, s>() : nullptr);
    __syncthreads();
    fft_mid_stages<C, dir, s + 1, Ns * R, PT>(sgn, tw, sh, tab);
  }
}

// Full forward/inverse transform: first stage from src (global), middle stages
// in LDS, last stage to snk (global). dir 0 = forward plan (sgn -1), 1 = inverse.
// HIN / HOUT as in fft_stage, for the first / last stage.
template <class C, int dir, bool HIN, bool HOUT, class Src, class Snk>
__device__ __forceinline__ void fft_line_transform(const cplx<typename C::T>* __restrict__ tw, cplx<typename C::T>* sh,
                                                   Src&& src, Snk&& snk) {
  using T = typename C::T;
  constexpr int S = plan_stages(C::L, C::BIG);
  const int sgn = dir == 0 ? -1 : +1;
  constexpr int R0 = stage_radix(C::L, dir, 0, C::BIG);
  fft_stage<C, R0, 1, false, HIN, false>(
      sgn, tw, src, [&](int line, int pb, int ro, cplx<T> v) { sh[C::lds(line, pb, ro)] = v; });
  __syncthreads();
  fft_mid_stages<C, dir, 1, R0>(sgn, tw, sh);
  constexpr int RL = stage_radix(C::L, dir, S - 1, C::BIG);
  constexpr int NsL = ns_before<C::L, C::BIG, dir, S - 1>();
  fft_stage<C, RL, NsL, false, false, HOUT>(
      sgn, tw, [&](int line, int pb, int ro) { return sh[C::lds(line, pb, ro)]; }, snk);
}

// Points of the convolution middle stage held by this thread: butterfly t,
// leg r -> (line, p). Used to prefetch the kernel spectrum into registers.
template <class C>
struct ConvMidMap {
  static constexpr int S = plan_stages(C::L, C::BIG);
  static constexpr int R = stage_radix(C::L, 0, S - 1, C::BIG);
  static constexpr int NB = C::NL * (C::L / R);
  static constexpr int TT = (NB + C::NT - 1) / C::NT;
  __device__ static __forceinline__ bool at(int t, int r, int& line, int& p) {
    if (!(NB % C::NT == 0 || (int)threadIdx.x + t * C::NT < NB)) return false;
    int j;
    C::template split<R>(t, line, j);
    p = j + r * (C::L / R);
    return true;
  }
};

// Convolution along a line: forward (from src), multiply by gh, inverse (to
// snk). The input occupies at most the first half of the line and only the
// first half of the output is kept (linear convolution by zero padding).
// PT: the twiddle powers of every twiddled stage come from a power table that
// the workgroup builds in LDS at tab (pow_table_size<C>() values): its loads
// are issued after the first stage's data loads and stored after that stage's
// butterflies; the first barrier publishes it. pre() runs at the same point
// (the caller's prefetch of the kernel spectrum), so neither delays the first
// stage.
template <class C, bool PT = false, class Src, class Gh, class Snk, class Pre = NoHook>
__device__ __forceinline__ void fft_line_convolve(const cplx<typename C::T>* __restrict__ tw, cplx<typename C::T>* sh,
                                                  Src&& src, Gh&& gh, Snk&& snk, cplx<typename C::T>* tab = nullptr,
                                                  Pre&& pre = Pre()) {
  using T = typename C::T;
  constexpr int S = plan_stages(C::L, C::BIG);
  constexpr int R0 = stage_radix(C::L, 0, 0, C::BIG);
  static_assert(!PT || plan_max_radix<C::L, C::BIG>() <= 16, "power tables for radices up to 16");
  auto to_lds = [&](int line, int pb, int ro, cplx<T> v) { sh[C::lds(line, pb, ro)] = v; };
  auto from_lds = [&](int line, int pb, int ro) { return sh[C::lds(line, pb, ro)]; };
  constexpr int NREG = PT ? pow_regs<C>() : 1;
  cplx<T> rv[NREG];
  // (the table loads go first: loads complete in issue order, and the table is
  // stored before the first barrier, the spectrum only used after it)
  fft_stage<C, R0, 1, false, true, false>(-1, tw, src, to_lds, nullptr, [&] {
    if constexpr (PT) pow_fill<C, false>(tw, tab, rv);
    pre();
  });
  if constexpr (PT) pow_fill<C, true>(tw, tab, rv);
  __syncthreads();
  fft_mid_stages<C, 0, 1, R0, PT>(-1, tw, sh, tab);
  constexpr int RL = stage_radix(C::L, 0, S - 1, C::BIG);
  fft_conv_mid<C, RL, PT>(tw, from_lds, gh, to_lds, PT ? tab + pow_off<C::L, C::BIG, 0, S - 1>() : nullptr);
  __syncthreads();
  // inverse plan is the reverse of the forward plan; its first stage (radix RL) is done
  fft_mid_stages<C, 1, 1, RL, PT>(+1, tw, sh, tab);
  constexpr int RI = stage_radix(C::L, 1, S - 1, C::BIG);
  constexpr int NsI = ns_before<C::L, C::BIG, 1, S - 1>();
  fft_stage<C, RI, NsI, false, false, true, PT>(+1, tw, from_lds, snk,
                                                PT ? tab + pow_off<C::L, C::BIG, 1, S - 1>() : nullptr);
}

}  // namespace fwi
