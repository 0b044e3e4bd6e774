// gsys_launch: running a user kernel that issues calls through the device
// API (gsys_device.hpp).  Every launch starts from cleared kernel-call sites,
// so kernel-granularity calls elect their caller afresh (section 5: the
// designated caller of a kernel call is chosen per launch).  The persistent
// forms clamp the grid to what is resident at once: a kernel-granularity
// call waits on every work-group of the launch, and a work-group that is not
// running can never arrive (section 4.1).  The graph form builds the clear and
// the user kernel into one hipGraph per (kernel, shape) and sets each
// launch's arguments into it before it is replayed.
#include "gsys_device.hpp"
#include "gsys.h"
#include "kernels.hpp"

#include <errno.h>
#include <stdio.h>

namespace gsys_ln {

__global__ void clear_sites(unsigned long long* p, uint32_t n) {
  const uint32_t i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) p[i] = 0;
}

}  // namespace gsys_ln

int gsys_launch(gsys_ctx* c, const gsys_launch_desc* d, void* stream) {
  if (!c || !d || !d->kernel) return -EINVAL;
  const dim3 b(d->block[0] ? d->block[0] : 1, d->block[1] ? d->block[1] : 1,
               d->block[2] ? d->block[2] : 1);
  dim3 g(d->grid[0], d->grid[1] ? d->grid[1] : 1, d->grid[2] ? d->grid[2] : 1);
  const uint64_t threads = (uint64_t)b.x * b.y * b.z;
  if (!g.x || threads > 1024) return -EINVAL;
  const bool persistent = d->mode == GSYS_PERSISTENT || d->mode == GSYS_GRAPH;
  if (!persistent && d->mode != GSYS_PLAIN) return -EINVAL;
  if (persistent && (g.y != 1 || g.z != 1)) return -EINVAL;  // a one-dimensional grid
  if (gsys_internal::no_device(c)) return -ENODEV;  // a CPU-only context launches nothing
  if (persistent) {
    const uint32_t r = gsys_internal::resident_grid(c, d->kernel, (uint32_t)threads, d->lds_bytes);
    if (!r) return -ENODEV;
    if (g.x > r) g.x = r;
  }
  gsys_dev_ctx dc;
  if (int e = gsys_device_ctx(c, &dc)) return e;
  unsigned long long* sites = reinterpret_cast<unsigned long long*>(dc.ksites);
  uint32_t words = dc.n_ksites * (uint32_t)(sizeof(gsys::KState) / 8);
  void* clear_args[] = {&sites, &words};
  const gsys_internal::KLaunch k[2] = {
      {(const void*)gsys_ln::clear_sites, dim3((words + 255) / 256), dim3(256), 0, clear_args},
      {d->kernel, g, b, d->lds_bytes, d->args}};
  hipStream_t s = (hipStream_t)stream;
  if (d->mode == GSYS_GRAPH) {
    const uint64_t key = gsys_internal::hash_words(
        {0x1A0ull, (uint64_t)d->kernel, g.x, b.x, b.y, b.z, d->lds_bytes});
    return gsys_internal::launch_graph(c, key, k, 2, s);
  }
  hipSetDevice(gsys_internal::device_of(c));
  for (const auto& l : k) {
    const hipError_t e = hipLaunchKernel(l.kernel, l.grid, l.block, l.args, l.lds, s);
    if (e != hipSuccess) {
      fprintf(stderr, "gsys: gsys_launch: %s\n", hipGetErrorString(e));
      return -ENODEV;
    }
  }
  return 0;
}
