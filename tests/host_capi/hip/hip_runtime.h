// Host stand-in for the HIP runtime, used to build the library's C ABI
// (capi.cpp) with g++ and the address / undefined-behaviour sanitizers and
// run it without a GPU. "Device" memory is host heap memory, streams run
// their work at once, and stream capture records that work into graphs that
// hipGraphLaunch replays, with the fork / join rules of stream capture checked
// (a forked stream must be joined back before the capture ends; no waits on
// events recorded outside the capture; no synchronising or allocating call
// from the capturing thread). The kernels are replaced by stand-ins
// (stub_kernels.cpp) that read and write the ranges each kernel's contract
// names, so the sanitizers see every buffer extent the host code plans.
#pragma once
#include <cmath>
#include <cstddef>
#include <cstdint>

#define __device__
#define __host__
#define __global__
#define __forceinline__ inline
#define __restrict__
#define __launch_bounds__(x)
#define __align__(x) alignas(x)

struct EmuDim {
  unsigned x = 0, y = 0, z = 0;
};
extern thread_local EmuDim threadIdx;
inline void __syncthreads() {}
inline double __shfl_xor(double v, int, int) { return v; }

enum hipError_t {
  hipSuccess = 0,
  hipErrorInvalidValue = 1,
  hipErrorOutOfMemory = 2,
  hipErrorInvalidHandle = 400,
  hipErrorStreamCaptureUnsupported = 900,
  hipErrorStreamCaptureInvalidated = 901,
  hipErrorStreamCaptureUnjoined = 904,
  hipErrorStreamCaptureIsolation = 905,
  hipErrorStreamCaptureWrongThread = 908,
  hipErrorIllegalState = 401,
};

enum hipMemcpyKind {
  hipMemcpyHostToHost = 0,
  hipMemcpyHostToDevice = 1,
  hipMemcpyDeviceToHost = 2,
  hipMemcpyDeviceToDevice = 3,
  hipMemcpyDefault = 4
};

enum hipStreamCaptureMode {
  hipStreamCaptureModeGlobal = 0,
  hipStreamCaptureModeThreadLocal = 1,
  hipStreamCaptureModeRelaxed = 2
};

#define hipStreamDefault 0x0
#define hipStreamNonBlocking 0x1
#define hipEventDefault 0x0
#define hipEventDisableTiming 0x2
#define hipEventDisableSystemFence 0x20000000
#define hipHostMallocDefault 0x0

struct EmuStream;
struct EmuEvent;
struct EmuGraph;
struct EmuExec;
typedef EmuStream* hipStream_t;
typedef EmuEvent* hipEvent_t;
typedef EmuGraph* hipGraph_t;
typedef EmuExec* hipGraphExec_t;
typedef struct EmuNode* hipGraphNode_t;

const char* hipGetErrorString(hipError_t e);
hipError_t hipGetLastError();
hipError_t hipGetDeviceCount(int* count);
hipError_t hipSetDevice(int dev);
hipError_t hipGetDevice(int* dev);
hipError_t hipMemGetInfo(size_t* free_b, size_t* total_b);
hipError_t hipMalloc(void** p, size_t bytes);
hipError_t hipFree(void* p);
hipError_t hipHostMalloc(void** p, size_t bytes, unsigned flags);
hipError_t hipHostFree(void* p);
hipError_t hipMemcpy(void* dst, const void* src, size_t bytes, hipMemcpyKind kind);
hipError_t hipMemcpyAsync(void* dst, const void* src, size_t bytes, hipMemcpyKind kind, hipStream_t st);
hipError_t hipMemsetAsync(void* dst, int value, size_t bytes, hipStream_t st);
hipError_t hipStreamCreateWithFlags(hipStream_t* st, unsigned flags);
hipError_t hipStreamDestroy(hipStream_t st);
hipError_t hipStreamSynchronize(hipStream_t st);
hipError_t hipDeviceSynchronize();
hipError_t hipStreamWaitEvent(hipStream_t st, hipEvent_t ev, unsigned flags);
hipError_t hipEventCreateWithFlags(hipEvent_t* ev, unsigned flags);
hipError_t hipEventDestroy(hipEvent_t ev);
hipError_t hipEventRecord(hipEvent_t ev, hipStream_t st);
hipError_t hipEventSynchronize(hipEvent_t ev);
hipError_t hipEventElapsedTime(float* ms, hipEvent_t a, hipEvent_t b);
hipError_t hipStreamBeginCapture(hipStream_t st, hipStreamCaptureMode mode);
hipError_t hipStreamEndCapture(hipStream_t st, hipGraph_t* g);
hipError_t hipGraphInstantiate(hipGraphExec_t* exec, hipGraph_t g, hipGraphNode_t* err_node, char* log,
                               size_t log_size);
hipError_t hipGraphDestroy(hipGraph_t g);
hipError_t hipGraphExecDestroy(hipGraphExec_t e);
hipError_t hipGraphLaunch(hipGraphExec_t e, hipStream_t st);
hipError_t hipGetSymbolAddress(void** p, const void* symbol);
#define HIP_SYMBOL(s) (&(s))
