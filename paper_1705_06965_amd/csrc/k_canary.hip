// Visibility canary for producer calls: every work-item stamps its 64 bytes
// of a host buffer and the stamped buffer is written to a file with pwrite,
// issued at work-item, work-group or kernel granularity.  A producer call
// needs every work-item of its group to have finished its stores before the
// call (section 4.1: producers keep the barrier before the call under relaxed
// ordering; strong ordering adds the barrier after).  If any stamp were not
// yet visible to the host when the call ran, the file would hold the
// buffer's earlier contents instead of the stamp.
#include "gsys_device.hpp"
#include "gsys.h"
#include "kernels.hpp"

#include <algorithm>

namespace gsys_cn {

using namespace gsys;

__device__ __forceinline__ uint64_t stamp_word(uint64_t seed, uint64_t item, uint32_t k) {
  return (seed * 0x9E3779B97F4A7C15ull) ^ ((item * 8 + k + 1) * 0xD1B54A32D192ED03ull);
}

struct CnArgs {
  gsys_dev_ctx c;
  uint64_t buf;        // host buffer, 64 bytes per item
  int64_t* out_ret;    // device: per item (work-item), per group or [0] (kernel)
  KState* ks;
  uint64_t n;
  uint64_t seed;
  int32_t fd;
};

template <G g, O o, B b>
__global__ __launch_bounds__(1024) void canary(CnArgs A) {
  const uint64_t first = (uint64_t)blockIdx.x * blockDim.x;
  const uint64_t item = first + threadIdx.x;
  const bool valid = item < A.n;
  if (valid) {
    gptr_t<uint64_t> p = gp<uint64_t>(A.buf + item * 64);
#pragma unroll
    for (uint32_t k = 0; k < 8; ++k) p[k] = stamp_word(A.seed, item, k);
  }
  if constexpr (g == G::WorkItem) {
    if (valid) {
      Ticket tk;
      int64_t r = call_wi<b>(A.c, GSYS_NR_PWRITE64,
                             Args6{{(uint64_t)(int64_t)A.fd, A.buf + item * 64, 64, item * 64, 0, 0}},
                             &tk);
      if constexpr (b == B::NonBlocking) r = r ? r : wait_wi(A.c, tk);
      A.out_ret[item] = r;
    }
  } else if constexpr (g == G::WorkGroup) {
    const uint64_t cnt = std::min<uint64_t>(blockDim.x, A.n - first);
    Ticket tk{0, 0, 0};
    int64_t r = call_wg<o, b>(A.c, GSYS_NR_PWRITE64, 0,
                              Args6{{(uint64_t)(int64_t)A.fd, A.buf + first * 64, cnt * 64,
                                     first * 64, 0, 0}},
                              &tk);
    if constexpr (b == B::NonBlocking) r = wait_wg(A.c, tk);
    if (threadIdx.x == 0) A.out_ret[blockIdx.x] = r;
  } else {
    Ticket tk{0, 0, 0};
    int64_t r = call_kernel<b>(
        A.c, A.ks, GSYS_NR_PWRITE64, 0, [] {},
        [&] { return Args6{{(uint64_t)(int64_t)A.fd, A.buf, A.n * 64, 0, 0, 0}}; }, &tk);
    // the last work-group to arrive made the call; it records the result
    if constexpr (b == B::NonBlocking) {
      if (tk.n) {
        const int64_t w = wait_wg(A.c, tk);
        if (threadIdx.x == 0) A.out_ret[0] = w;
      }
    } else {
      if (threadIdx.x == 0 && r != GSYS_NOT_WAITED) A.out_ret[0] = r;
    }
  }
}

__global__ void zero_words(unsigned long long* p, uint32_t n) {
  const uint32_t i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) p[i] = 0;
}

}  // namespace gsys_cn

using namespace gsys_cn;

int gsys_canary(gsys_ctx* ctx, int fd, uint64_t buf, uint64_t n_items, uint64_t seed,
                uint64_t out_ret, uint32_t cell, uint32_t wg_size, void* stream) {
  if (!ctx || !out_ret || !n_items) return -EINVAL;
  if (wg_size == 0 || wg_size > 1024 || wg_size % 64) return -EINVAL;
  if (gsys_internal::check_host_range(ctx, buf, n_items * 64)) return -EFAULT;
  CnArgs A;
  if (int e = gsys_device_ctx(ctx, &A.c)) return e;
  A.buf = buf;
  A.out_ret = (int64_t*)out_ret;
  A.ks = (KState*)gsys_internal::kstate(ctx);
  A.n = n_items;
  A.seed = seed;
  A.fd = fd;
  const uint32_t gran = GSYS_CELL_GRAN(cell);
  const bool strong = (cell & GSYS_CELL_STRONG) != 0;
  const bool blocking = (cell & GSYS_CELL_BLOCKING) != 0;
  const void* k = nullptr;
  if (gran == GSYS_GRAN_WI) {
    if (!strong) return -EINVAL;
    k = blocking ? (const void*)canary<G::WorkItem, O::Strong, B::Blocking>
                 : (const void*)canary<G::WorkItem, O::Strong, B::NonBlocking>;
  } else if (gran == GSYS_GRAN_WG) {
    if (strong)
      k = blocking ? (const void*)canary<G::WorkGroup, O::Strong, B::Blocking>
                   : (const void*)canary<G::WorkGroup, O::Strong, B::NonBlocking>;
    else
      k = blocking ? (const void*)canary<G::WorkGroup, O::Relaxed, B::Blocking>
                   : (const void*)canary<G::WorkGroup, O::Relaxed, B::NonBlocking>;
  } else if (gran == GSYS_GRAN_KERNEL) {
    if (strong) return -EINVAL;
    k = blocking ? (const void*)canary<G::Kernel, O::Relaxed, B::Blocking>
                 : (const void*)canary<G::Kernel, O::Relaxed, B::NonBlocking>;
    if (gsys_internal::no_device(ctx)) return -ENODEV;
    hipLaunchKernelGGL(zero_words, dim3(1), dim3(64), 0, (hipStream_t)stream,
                       (unsigned long long*)A.ks, (uint32_t)(sizeof(KState) / 8));
  } else {
    return -EINVAL;
  }
  const uint64_t grid = (n_items + wg_size - 1) / wg_size;
  if (grid > 0x7fffffffull) return -EINVAL;
  void* args[] = {&A};
  return gsys_internal::launch(ctx, k, (uint32_t)grid, wg_size, 0, args, (hipStream_t)stream);
}
