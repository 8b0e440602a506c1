// Host stand-in for the HIP runtime header, used only to compile the line-FFT
// device code on the CPU: a workgroup is NT std::threads, __syncthreads() is
// a barrier shared by them, threadIdx is thread-local.
#pragma once
#include <barrier>
#include <cmath>
#define __device__
#define __host__
#define __global__
#define __forceinline__ inline
#define __restrict__
#define __launch_bounds__(x)
struct EmuIdx {
  unsigned x, y, z;
};
extern thread_local EmuIdx threadIdx;
extern thread_local EmuIdx blockIdx;
extern std::barrier<>* emu_bar;
inline void __syncthreads() { emu_bar->arrive_and_wait(); }
inline double __shfl_xor(double v, int, int) { return v; }
typedef int hipStream_t;
