// Work submission of the host stand-in for the HIP runtime: stand-in kernels
// run their body at once on a live stream and are recorded into the graph of
// a capturing stream (replayed by hipGraphLaunch).
#pragma once
#include <hip/hip_runtime.h>

#include <cstddef>
#include <functional>

namespace emu {
void submit(hipStream_t st, const char* name, std::function<void()> body);
// Touch a range as a kernel would: every 64th byte and the last one read, or
// the whole range written (zero bytes), so the sanitizers check the extent.
void rd(const void* p, size_t bytes);
void wr(void* p, size_t bytes);
// Counters of the run, printed by the driver.
struct Counts {
  long kernels_live = 0, kernels_captured = 0, graph_launches = 0, captures = 0, copies_captured = 0;
  long violations = 0;
};
Counts& counts();
void violation(const char* what);
// Iterations after which a stand-in Krylov state reports a RHS as converged
// (RHS b needs base + b % spread iterations).
extern int iters_base, iters_spread;
// Free device memory reported by hipMemGetInfo.
extern size_t mem_free;
}  // namespace emu
