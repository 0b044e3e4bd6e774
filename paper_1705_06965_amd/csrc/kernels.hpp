// Internal helpers shared by the workload entry points (not part of the C ABI).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include <initializer_list>

#include "gsys.h"

namespace gsys_internal {

// 0 if [dev, dev + bytes) lies inside one registered host buffer, else -EFAULT.
int check_host_range(gsys_ctx* ctx, uint64_t dev, uint64_t bytes);
// Device scratch for per-launch kernel-call state (256 bytes, zeroed by the
// entry points before a launch that uses it).
void* kstate(gsys_ctx* ctx);
// Work-groups of `kernel` that fit on the device at once.
uint32_t resident_grid(gsys_ctx* ctx, const void* kernel, uint32_t block, uint32_t lds);
// A persistent grid size requested through GSYS_PERSISTENT_GRID (0 = none).
uint32_t persistent_grid_override(gsys_ctx* ctx);
uint64_t hash_words(std::initializer_list<uint64_t> w);
// Two host-coherent control words owned by the context (a 256-byte line of
// the page set up by gsys_init; nothing is allocated here).
int control_page(gsys_ctx* ctx, void** host, uint64_t* dev);
// true for a CPU-only context (GSYS_CFG_NO_DEVICE): nothing may be launched
// (declared with the other test accessors in testing_access.hpp too).
bool no_device(gsys_ctx* ctx);
// The HIP device ordinal of the context.
int device_of(gsys_ctx* ctx);
// Set-up of the allocation-free serving entry point's scratch array on
// `device`, which must be current (called by gsys_init).  Weak: a host-only
// build of the context and pool (the sanitizer test driver) has no kernels,
// and there the symbol is null.
int serve_scratch_setup(int device) __attribute__((weak));
// Device wall-clock ticks per millisecond.
uint64_t ticks_per_ms(gsys_ctx* ctx);
int launch(gsys_ctx* ctx, const void* kernel, uint32_t grid, uint32_t block, uint32_t lds,
           void** args, hipStream_t s);
// One kernel launch of a graph form.
struct KLaunch {
  const void* kernel;
  dim3 grid, block;
  uint32_t lds;
  void** args;
};
// Launch the chain k[0], ..., k[n - 1] (each after the one before) as a
// hipGraph: built and instantiated the first time `key` is seen (the key
// must name the kernels and their shapes), then replayed with this call's
// arguments set into its nodes.
int launch_graph(gsys_ctx* ctx, uint64_t key, const KLaunch* k, uint32_t n, hipStream_t s);
// Kernel-granularity call sites per context for user kernels (16 bytes each).
constexpr uint32_t kSites = 64;

}  // namespace gsys_internal
