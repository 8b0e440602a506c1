// Raw buffer views for the device-side FFT passes (device translation units
// only).
#pragma once

#include "common.hpp"

namespace fwi {

// Raw buffer view of device memory (gfx9 buffer resource, stride 0): byte
// offsets are 32-bit, loads at or past `bytes` return zero and stores there
// are dropped, so zero padding and cropping need no per-access predicates.
// Views must cover less than 2 GiB.
constexpr int kBufferWord3 = 0x00020000;  // gfx9 raw-buffer format bits
constexpr unsigned kBufferOut = 0x80000000u;  // an offset past every view

struct BufView {
  __amdgpu_buffer_rsrc_t r;
  __device__ __forceinline__ BufView(const void* p, unsigned bytes)
      : r(__builtin_amdgcn_make_buffer_rsrc(const_cast<void*>(p), (short)0, (int)bytes, kBufferWord3)) {}
  template <typename T>
  __device__ __forceinline__ cplx<T> ld(unsigned off) const {
    if constexpr (sizeof(T) == 4) {
      return __builtin_bit_cast(cplx<T>, __builtin_amdgcn_raw_buffer_load_b64(r, off, 0, 0));
    } else {
      return __builtin_bit_cast(cplx<T>, __builtin_amdgcn_raw_buffer_load_b128(r, off, 0, 0));
    }
  }
  template <typename T>
  __device__ __forceinline__ void st(unsigned off, cplx<T> v) const {
    if constexpr (sizeof(T) == 4) {
      using V = decltype(__builtin_amdgcn_raw_buffer_load_b64(r, 0, 0, 0));
      __builtin_amdgcn_raw_buffer_store_b64(__builtin_bit_cast(V, v), r, off, 0, 0);
    } else {
      using V = decltype(__builtin_amdgcn_raw_buffer_load_b128(r, 0, 0, 0));
      __builtin_amdgcn_raw_buffer_store_b128(__builtin_bit_cast(V, v), r, off, 0, 0);
    }
  }
};

}  // namespace fwi
