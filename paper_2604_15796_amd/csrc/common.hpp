// Shared device/host helpers for the FWI HIP library: complex arithmetic,
// launch checks and small reductions. gfx950 only (wave64).
#pragma once

#include <hip/hip_runtime.h>
#include <cstddef>
#include <cstdint>

namespace fwi {

constexpr int WAVE = 64;

template <typename T>
struct alignas(2 * sizeof(T)) cplx {
  T x, y;
};
using c64 = cplx<float>;
using c128 = cplx<double>;

template <typename T>
__host__ __device__ __forceinline__ cplx<T> mk(T a, T b) {
  cplx<T> r;
  r.x = a;
  r.y = b;
  return r;
}
template <typename T>
__host__ __device__ __forceinline__ cplx<T> operator+(cplx<T> a, cplx<T> b) {
  return mk(a.x + b.x, a.y + b.y);
}
template <typename T>
__host__ __device__ __forceinline__ cplx<T> operator-(cplx<T> a, cplx<T> b) {
  return mk(a.x - b.x, a.y - b.y);
}
template <typename T>
__host__ __device__ __forceinline__ cplx<T> operator*(cplx<T> a, cplx<T> b) {
  return mk(a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x);
}
template <typename T>
__host__ __device__ __forceinline__ cplx<T> operator*(T s, cplx<T> a) {
  return mk(s * a.x, s * a.y);
}
template <typename T>
__host__ __device__ __forceinline__ cplx<T> conj(cplx<T> a) {
  return mk(a.x, -a.y);
}
// conj(a) * b
template <typename T>
__host__ __device__ __forceinline__ cplx<T> cmulc(cplx<T> a, cplx<T> b) {
  return mk(a.x * b.x + a.y * b.y, a.x * b.y - a.y * b.x);
}
// acc + a * b as four fused multiply-adds
template <typename T>
__host__ __device__ __forceinline__ cplx<T> cfma(cplx<T> a, cplx<T> b, cplx<T> acc) {
  acc.x = fma(a.x, b.x, acc.x);
  acc.x = fma(-a.y, b.y, acc.x);
  acc.y = fma(a.x, b.y, acc.y);
  acc.y = fma(a.y, b.x, acc.y);
  return acc;
}
template <typename T>
__host__ __device__ __forceinline__ T norm2(cplx<T> a) {
  return a.x * a.x + a.y * a.y;
}
template <typename To, typename Ti>
__host__ __device__ __forceinline__ cplx<To> cvt(cplx<Ti> a) {
  return mk((To)a.x, (To)a.y);
}
// multiply by +i (sign>0) or -i
template <typename T>
__host__ __device__ __forceinline__ cplx<T> mul_i(cplx<T> a, int sign) {
  return sign > 0 ? mk(-a.y, a.x) : mk(a.y, -a.x);
}

// Wave-level sum of a double (wave64, butterfly shuffles).
__device__ __forceinline__ double wave_sum(double v) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
  return v;
}

// Block sum of a double across NT threads (NT multiple of 64); result valid in
// all threads. `red` must hold NT/64 doubles of LDS.
template <int NT>
__device__ __forceinline__ double block_sum(double v, double* red) {
  v = wave_sum(v);
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  __syncthreads();
  if (lane == 0) red[w] = v;
  __syncthreads();
  double s = 0.0;
#pragma unroll
  for (int i = 0; i < NT / 64; ++i) s += red[i];
  return s;
}

}  // namespace fwi
