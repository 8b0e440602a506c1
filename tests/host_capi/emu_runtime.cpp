// Host stand-in for the HIP runtime calls that the library's host code makes
// (see hip/hip_runtime.h). Stream capture follows the rules of the real
// runtime that matter here:
//  - work enqueued on a capturing stream is recorded, not run;
//  - a stream joins a capture by waiting on an event recorded inside it;
//  - every stream that joined must be waited on again (joined back) by the
//    capture before it ends, else the end fails with ...CaptureUnjoined;
//  - a capturing stream may not wait on an event recorded outside the
//    capture (...CaptureIsolation);
//  - in thread-local and global capture modes the capturing thread may not
//    allocate, free, copy synchronously or synchronise a capturing stream
//    (...CaptureUnsupported, and the capture is invalidated).
// Any such error, and any copy or fill node captured into a graph, counts as
// a violation that the driver reports.
#include <hip/hip_runtime.h>

#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <map>
#include <set>
#include <vector>

#include "emu.hpp"

thread_local EmuDim threadIdx;

struct EmuOp {
  const char* name;
  bool kernel;
  std::function<void()> body;
};

struct EmuGraph {
  std::vector<EmuOp> ops;
  EmuStream* origin = nullptr;
  std::set<EmuStream*> members;
  bool invalid = false;
  bool ended = false;
};

struct EmuExec {
  std::vector<EmuOp> ops;
};

struct EmuStream {
  EmuGraph* cap = nullptr;
  long seq = 0;         // operations enqueued while capturing
  long joined_seq = 0;  // ops of this stream that another captured stream waits on
  bool capture_owner_thread_local = false;
};

struct EmuEvent {
  EmuGraph* cap = nullptr;  // capture it was recorded in (null: recorded live)
  EmuStream* st = nullptr;
  long seq = 0;
  bool recorded = false;
};

namespace emu {
int iters_base = 12, iters_spread = 5;
size_t mem_free = size_t(8) << 30;
static Counts g_counts;
Counts& counts() { return g_counts; }
void violation(const char* what) {
  g_counts.violations += 1;
  std::fprintf(stderr, "[emu] VIOLATION: %s\n", what);
}
}  // namespace emu

namespace {
EmuStream g_null_stream;
thread_local int tl_capturing = 0;  // captures begun (thread-local / global mode) on this thread
std::set<EmuGraph*> g_active;       // captures in progress

EmuStream* S(hipStream_t st) { return st ? st : &g_null_stream; }

hipError_t prohibited(const char* what) {
  if (tl_capturing > 0) {
    for (EmuGraph* g : g_active) g->invalid = true;
    emu::violation(what);
    return hipErrorStreamCaptureUnsupported;
  }
  return hipSuccess;
}

void enqueue(EmuStream* s, const char* name, bool kernel, std::function<void()> body) {
  if (s->cap) {
    s->cap->ops.push_back({name, kernel, std::move(body)});
    s->seq += 1;
    if (kernel) {
      emu::g_counts.kernels_captured += 1;
    } else {
      emu::g_counts.copies_captured += 1;
      emu::violation("copy or fill node captured into a graph");
    }
  } else {
    body();
    if (kernel) emu::g_counts.kernels_live += 1;
  }
}
}  // namespace

namespace emu {
void submit(hipStream_t st, const char* name, std::function<void()> body) { enqueue(S(st), name, true, std::move(body)); }
void rd(const void* p, size_t bytes) {
  if (!bytes) return;
  if (!p) {
    violation("kernel reads through a null pointer");
    return;
  }
  const volatile unsigned char* c = static_cast<const volatile unsigned char*>(p);
  unsigned acc = 0;
  for (size_t i = 0; i < bytes; i += 64) acc += c[i];
  acc += c[bytes - 1];
  (void)acc;
}
void wr(void* p, size_t bytes) {
  if (!bytes) return;
  if (!p) {
    violation("kernel writes through a null pointer");
    return;
  }
  std::memset(p, 0, bytes);
}
}  // namespace emu

const char* hipGetErrorString(hipError_t e) {
  switch (e) {
    case hipSuccess: return "hipSuccess";
    case hipErrorStreamCaptureUnsupported: return "operation not permitted when stream is capturing";
    case hipErrorStreamCaptureInvalidated: return "capture invalidated";
    case hipErrorStreamCaptureUnjoined: return "capture unjoined";
    case hipErrorStreamCaptureIsolation: return "capture isolation";
    case hipErrorStreamCaptureWrongThread: return "capture wrong thread";
    default: return "emulated HIP error";
  }
}
hipError_t hipGetLastError() { return hipSuccess; }
hipError_t hipGetDeviceCount(int* count) {
  *count = 1;
  return hipSuccess;
}
hipError_t hipSetDevice(int dev) { return dev == 0 ? hipSuccess : hipErrorInvalidValue; }
hipError_t hipGetDevice(int* dev) {
  *dev = 0;
  return hipSuccess;
}
hipError_t hipMemGetInfo(size_t* free_b, size_t* total_b) {
  *free_b = emu::mem_free;
  *total_b = size_t(16) << 30;
  return hipSuccess;
}
hipError_t hipMalloc(void** p, size_t bytes) {
  if (hipError_t e = prohibited("hipMalloc while capturing")) return e;
  *p = std::malloc(bytes ? bytes : 1);
  return *p ? hipSuccess : hipErrorOutOfMemory;
}
hipError_t hipFree(void* p) {
  if (hipError_t e = prohibited("hipFree while capturing")) return e;
  std::free(p);
  return hipSuccess;
}
hipError_t hipHostMalloc(void** p, size_t bytes, unsigned) {
  if (hipError_t e = prohibited("hipHostMalloc while capturing")) return e;
  *p = std::calloc(1, bytes ? bytes : 1);
  return *p ? hipSuccess : hipErrorOutOfMemory;
}
hipError_t hipHostFree(void* p) {
  if (hipError_t e = prohibited("hipHostFree while capturing")) return e;
  std::free(p);
  return hipSuccess;
}
hipError_t hipMemcpy(void* dst, const void* src, size_t bytes, hipMemcpyKind) {
  if (hipError_t e = prohibited("synchronous hipMemcpy while capturing")) return e;
  std::memcpy(dst, src, bytes);
  return hipSuccess;
}
hipError_t hipMemcpyAsync(void* dst, const void* src, size_t bytes, hipMemcpyKind, hipStream_t st) {
  enqueue(S(st), "memcpy", false, [=] { std::memcpy(dst, src, bytes); });
  return hipSuccess;
}
hipError_t hipMemsetAsync(void* dst, int value, size_t bytes, hipStream_t st) {
  enqueue(S(st), "memset", false, [=] { std::memset(dst, value, bytes); });
  return hipSuccess;
}
hipError_t hipStreamCreateWithFlags(hipStream_t* st, unsigned) {
  *st = new EmuStream();
  return hipSuccess;
}
hipError_t hipStreamDestroy(hipStream_t st) {
  if (!st) return hipErrorInvalidHandle;
  if (st->cap) {
    emu::violation("stream destroyed while capturing");
    return hipErrorIllegalState;
  }
  delete st;
  return hipSuccess;
}
hipError_t hipStreamSynchronize(hipStream_t st) {
  if (S(st)->cap) {
    emu::violation("hipStreamSynchronize on a capturing stream");
    S(st)->cap->invalid = true;
    return hipErrorStreamCaptureUnsupported;
  }
  return hipSuccess;
}
hipError_t hipDeviceSynchronize() { return prohibited("hipDeviceSynchronize while capturing"); }
hipError_t hipEventCreateWithFlags(hipEvent_t* ev, unsigned) {
  *ev = new EmuEvent();
  return hipSuccess;
}
hipError_t hipEventDestroy(hipEvent_t ev) {
  delete ev;
  return hipSuccess;
}
hipError_t hipEventRecord(hipEvent_t ev, hipStream_t st) {
  if (!ev) return hipErrorInvalidHandle;
  EmuStream* s = S(st);
  ev->cap = s->cap;
  ev->st = s;
  ev->seq = s->seq;
  ev->recorded = true;
  return hipSuccess;
}
hipError_t hipEventSynchronize(hipEvent_t ev) {
  if (!ev) return hipErrorInvalidHandle;
  if (ev->cap) {
    emu::violation("hipEventSynchronize on an event recorded in a capture");
    return hipErrorStreamCaptureUnsupported;
  }
  return hipSuccess;
}
hipError_t hipEventElapsedTime(float* ms, hipEvent_t a, hipEvent_t b) {
  if (!a || !b || !a->recorded || !b->recorded) return hipErrorInvalidHandle;
  *ms = 0.01f;
  return hipSuccess;
}
hipError_t hipStreamWaitEvent(hipStream_t st, hipEvent_t ev, unsigned) {
  if (!ev) return hipErrorInvalidHandle;
  EmuStream* s = S(st);
  if (ev->cap && (ev->cap->ended || !g_active.count(ev->cap))) {
    emu::violation("wait on an event recorded in a capture that has ended");
    return hipErrorStreamCaptureIsolation;
  }
  if (s->cap) {
    if (!ev->cap) {
      emu::violation("capturing stream waits on an event recorded outside the capture");
      s->cap->invalid = true;
      return hipErrorStreamCaptureIsolation;
    }
    if (ev->cap != s->cap) {
      emu::violation("wait across two captures");
      return hipErrorStreamCaptureIsolation;
    }
    if (ev->seq > ev->st->joined_seq) ev->st->joined_seq = ev->seq;
    return hipSuccess;
  }
  if (ev->cap) {  // s joins the capture
    s->cap = ev->cap;
    s->seq = 0;
    s->joined_seq = 0;
    ev->cap->members.insert(s);
  }
  return hipSuccess;
}
hipError_t hipStreamBeginCapture(hipStream_t st, hipStreamCaptureMode mode) {
  EmuStream* s = S(st);
  if (!st) {
    emu::violation("capture on the null stream");
    return hipErrorIllegalState;
  }
  if (s->cap) {
    emu::violation("capture begun on a stream that is already capturing");
    return hipErrorIllegalState;
  }
  EmuGraph* g = new EmuGraph();
  g->origin = s;
  g->members.insert(s);
  s->cap = g;
  s->seq = 0;
  s->joined_seq = 0;
  s->capture_owner_thread_local = mode != hipStreamCaptureModeRelaxed;
  if (s->capture_owner_thread_local) tl_capturing += 1;
  g_active.insert(g);
  emu::g_counts.captures += 1;
  return hipSuccess;
}
hipError_t hipStreamEndCapture(hipStream_t st, hipGraph_t* out) {
  EmuStream* s = S(st);
  *out = nullptr;
  EmuGraph* g = s->cap;
  if (!g) {
    emu::violation("end of a capture that was not begun");
    return hipErrorIllegalState;
  }
  if (g->origin != s) {
    emu::violation("capture ended on a stream other than its origin");
    return hipErrorStreamCaptureWrongThread;
  }
  hipError_t rc = hipSuccess;
  for (EmuStream* m : g->members) {
    if (m != s && m->seq > m->joined_seq) {
      emu::violation("forked stream not joined back before the end of the capture");
      rc = hipErrorStreamCaptureUnjoined;
    }
  }
  for (EmuStream* m : g->members) {
    m->cap = nullptr;
    m->seq = m->joined_seq = 0;
  }
  if (s->capture_owner_thread_local) tl_capturing -= 1;
  g->ended = true;
  g_active.erase(g);
  if (g->invalid && rc == hipSuccess) rc = hipErrorStreamCaptureInvalidated;
  if (rc != hipSuccess) {
    delete g;
    return rc;
  }
  *out = g;
  return hipSuccess;
}
hipError_t hipGraphInstantiate(hipGraphExec_t* exec, hipGraph_t g, hipGraphNode_t*, char*, size_t) {
  if (!g) return hipErrorInvalidHandle;
  if (hipError_t e = prohibited("hipGraphInstantiate while capturing")) return e;
  EmuExec* x = new EmuExec();
  x->ops = g->ops;
  *exec = x;
  return hipSuccess;
}
hipError_t hipGraphDestroy(hipGraph_t g) {
  delete g;
  return hipSuccess;
}
hipError_t hipGraphExecDestroy(hipGraphExec_t e) {
  delete e;
  return hipSuccess;
}
hipError_t hipGraphLaunch(hipGraphExec_t e, hipStream_t st) {
  if (!e) return hipErrorInvalidHandle;
  if (S(st)->cap) {
    emu::violation("graph launched into a capture");
    return hipErrorStreamCaptureUnsupported;
  }
  for (EmuOp& op : e->ops) op.body();
  emu::g_counts.graph_launches += 1;
  return hipSuccess;
}
hipError_t hipGetSymbolAddress(void** p, const void* symbol) {
  *p = const_cast<void*>(symbol);
  return hipSuccess;
}
