// Per-item pread + FNV-1a-64 on gfx950: the pread microbenchmark of section 6
// (Fig. 5) issued at work-item, work-group or kernel granularity, strong or
// relaxed, blocking or non-blocking, and a persistent form that drains the
// items in one launch with double-buffered non-blocking group calls.
//
// Data path: the host pool preads each item into pinned host staging; the GPU
// reads the staging bytes once over the host link with coalesced 16-byte
// loads (each group of 16 lanes fetches one item's next 256 bytes), transposes
// them through LDS, and every lane runs the FNV-1a chain of its own item.
// FNV-1a is a serial byte chain, so one lane per item is the parallel grain.
#include "gsys_device.hpp"
#include "fnv_wave.hpp"
#include "gsys.h"
#include "kernels.hpp"

#include <algorithm>

namespace gsys_k {

using namespace gsys;

// Default persistent grid (work-groups); see gsys_fnv4k.  With 256-wide
// groups, 64 keep 32,768 reads in flight, which is enough for the host pool,
// and fewer waiters poll host memory: on the 262,144-item sweep 64 ran at
// 13.4 M calls/s against 12.8 M with 128 and 12.5 M with 256.
constexpr uint32_t kPersistentGrid = 64;

struct FnvArgs {
  gsys_dev_ctx c;
  const uint64_t* offsets;
  uint64_t n_items;
  uint64_t staging;
  gsys_iodesc* lists;
  uint64_t* out_fnv;
  int64_t* out_ret;
  KState* ks;
  int32_t fd;
  uint32_t item_bytes;
  uint32_t ring;  // persistent forms: 1 = each work-group owns two batch buffers
  uint32_t lds_list;  // strong work-group cells: aggregate the list in LDS first
};

// Staging address of item `item` of batch `bt` (slot = item - bt * batch).
__device__ __forceinline__ uint64_t stage_addr(const FnvArgs& A, uint64_t bt, uint32_t batch,
                                               uint64_t item) {
  if (!A.ring) return A.staging + item * A.item_bytes;
  const uint64_t buf = (uint64_t)blockIdx.x * 2 + (bt / gridDim.x) % 2;
  return A.staging + (buf * batch + (item - bt * batch)) * A.item_bytes;
}

// `row0` is the staging address of the item of lane 0 of this wavefront; the
// wavefront's items follow it at item_bytes apart.
template <uint32_t CH>
__device__ __forceinline__ void consume_item(const FnvArgs& A, uint64_t item, bool valid,
                                             int64_t ret, uint8_t* lds, uint64_t row0) {
  const uint32_t wave = threadIdx.x >> 6;
  const uint32_t nbytes =
      (valid && ret > 0) ? (uint32_t)min<int64_t>(ret, (int64_t)A.item_bytes) : 0u;
  const uint64_t h = wave_fnv_t<CH>(row0, nbytes, A.item_bytes, lds + wave * Tile<CH>::kBytes);
  if (valid) {
    A.out_fnv[item] = h;
    A.out_ret[item] = ret;
  }
}

// Plain form: one launch, one item per work-item, the call made at the
// granularity / ordering / blocking of the template.
template <G g, O o, B b, uint32_t WGMAX>
__global__ __launch_bounds__(WGMAX, WGMAX <= 256 ? 2 : 4) void fnv4k_plain(FnvArgs A) {
  constexpr uint32_t CH = chunk_for<WGMAX>();
  extern __shared__ __align__(16) uint8_t lds[];
  const uint64_t first = (uint64_t)blockIdx.x * blockDim.x;
  const uint64_t item = first + threadIdx.x;
  const bool valid = item < A.n_items;
  int64_t ret = 0;
  if constexpr (g == G::WorkItem) {
    if (valid) {
      Args6 a{{(uint64_t)(int64_t)A.fd, A.staging + item * A.item_bytes, A.item_bytes,
               A.offsets[item], 0, 0}};
      Ticket tk;
      ret = call_wi<b>(A.c, GSYS_NR_PREAD64, a, &tk);
      if constexpr (b == B::NonBlocking) ret = ret ? ret : wait_wi(A.c, tk);
    }
  } else if constexpr (g == G::WorkGroup) {
    gsys_iodesc* L = A.lists + first;
    const uint32_t cnt = (uint32_t)min<uint64_t>(blockDim.x, A.n_items - first);
    if constexpr (o == O::Strong) {
      const gsys_iodesc d{valid ? A.offsets[item] : 0, threadIdx.x * A.item_bytes,
                          (int32_t)A.item_bytes};
      if (A.lds_list) {
        // aggregated in LDS (the transposer's tile space, unused until the
        // hash): every work-item stores its descriptor there, and after a
        // barrier the caller's wavefront copies the list to the host-visible
        // buffer with 16-byte stores; the call's barrier before releases them
        gsys_iodesc* S = reinterpret_cast<gsys_iodesc*>(lds);
        *lp(reinterpret_cast<u32x4*>(S + threadIdx.x)) = *reinterpret_cast<const u32x4*>(&d);
        __syncthreads();
        if (threadIdx.x < 64)
          for (uint32_t i = threadIdx.x; i < cnt; i += 64)
            stg16((uint64_t)(L + i), *lp(reinterpret_cast<u32x4*>(S + i)));
      } else if (valid) {
        // every work-item writes its own descriptor straight into the host-
        // visible list (a wavefront's 64 are 1 KiB of consecutive bytes);
        // the barrier before the call makes all of them visible to the host
        L[threadIdx.x] = d;
      }
    } else {
      // relaxed consumer call: no barrier before it, so the designated
      // caller's wavefront builds the list from the offset table itself
      if (threadIdx.x < 64)
        for (uint32_t i = threadIdx.x; i < cnt; i += 64)
          L[i] = gsys_iodesc{A.offsets[first + i], i * A.item_bytes, (int32_t)A.item_bytes};
    }
    Args6 a{{(uint64_t)(int64_t)A.fd, (uint64_t)L, cnt, A.staging + first * A.item_bytes, 0, 0}};
    Ticket tk{0, 0, 0};
    int64_t r = call_wg<o, b>(A.c, GSYS_NR_PREAD64, GSYS_F_LIST, a, &tk);
    if constexpr (b == B::NonBlocking) r = wait_wg(A.c, tk);
    ret = valid ? (r < 0 ? r : (int64_t)__hip_atomic_load(&L[threadIdx.x].len_ret, __ATOMIC_RELAXED,
                                                          __HIP_MEMORY_SCOPE_SYSTEM))
                : 0;
  } else {
    Ticket tk{0, 0, 0};
    int64_t r = call_kernel<b>(
        A.c, A.ks, GSYS_NR_PREAD64, GSYS_F_LIST,
        [&]() {
          for (uint64_t i = threadIdx.x; i < A.n_items; i += blockDim.x)
            A.lists[i] = gsys_iodesc{A.offsets[i], (uint32_t)(i * A.item_bytes), (int32_t)A.item_bytes};
        },
        [&]() {
          return Args6{{(uint64_t)(int64_t)A.fd, (uint64_t)A.lists, A.n_items, A.staging, 0, 0}};
        },
        &tk);
    if constexpr (b == B::NonBlocking) r = r ? r : wait_kernel(A.c, tk);
    ret = valid ? (r < 0 ? r : (int64_t)__hip_atomic_load(&A.lists[item].len_ret, __ATOMIC_RELAXED,
                                                          __HIP_MEMORY_SCOPE_SYSTEM))
                : 0;
  }
  const uint64_t row0 = A.staging + (first + (threadIdx.x & ~63u)) * A.item_bytes;
  consume_item<CH>(A, item, valid, ret, lds, row0);
}

// Persistent form: a co-resident grid; work-group w handles batches w,
// w + grid, ...; each batch is one work-group call (relaxed consumer,
// non-blocking) whose descriptor list the caller's wavefront builds.  The
// call for the next batch is issued before waiting on the current one, so
// host servicing overlaps the GPU's consumption.
__device__ __forceinline__ Ticket issue_batch(const FnvArgs& A, uint64_t bt, uint32_t batch) {
  const uint64_t first = bt * batch;
  const uint32_t cnt = (uint32_t)min<uint64_t>(batch, A.n_items - first);
  gsys_iodesc* L = A.lists + first;
  if (threadIdx.x < 64)
    for (uint32_t i = threadIdx.x; i < cnt; i += 64)
      L[i] = gsys_iodesc{A.offsets[first + i], i * A.item_bytes, (int32_t)A.item_bytes};
  Args6 a{{(uint64_t)(int64_t)A.fd, (uint64_t)L, cnt, stage_addr(A, bt, batch, first), 0, 0}};
  Ticket tk{0, 0, 0};
  call_wg<O::Relaxed, B::NonBlocking>(A.c, GSYS_NR_PREAD64, GSYS_F_LIST, a, &tk);
  return tk;
}

template <uint32_t WGMAX>
__global__ __launch_bounds__(WGMAX, WGMAX <= 256 ? 2 : 4) void fnv4k_persistent(FnvArgs A) {
  constexpr uint32_t CH = chunk_for<WGMAX>();
  extern __shared__ __align__(16) uint8_t lds[];
  const uint32_t batch = blockDim.x;
  const uint64_t nb = (A.n_items + batch - 1) / batch;
  uint64_t bt = blockIdx.x;
  if (bt >= nb) return;
  Ticket tk = issue_batch(A, bt, batch);
  while (bt < nb) {
    const uint64_t bn = bt + gridDim.x;
    Ticket tkn{0, 0, 0};
    if (bn < nb) tkn = issue_batch(A, bn, batch);
    const int64_t r = wait_wg(A.c, tk);
    const uint64_t item = bt * batch + threadIdx.x;
    const bool valid = item < A.n_items;
    const int64_t ret =
        valid ? (r < 0 ? r : (int64_t)__hip_atomic_load(&A.lists[item].len_ret, __ATOMIC_RELAXED,
                                                        __HIP_MEMORY_SCOPE_SYSTEM))
              : 0;
    const uint64_t row0 = stage_addr(A, bt, batch, bt * batch + (threadIdx.x & ~63u));
    consume_item<CH>(A, item, valid, ret, lds, row0);
    // the buffer of batch bt is reused by batch bt + 2 * grid, issued in the
    // next iteration: every lane must be done reading it first
    __syncthreads();
    bt = bn;
    tk = tkn;
  }
}

// Kernel-split form: the host has already read every item (section 2,
// Fig. 1 left); a plain kernel checksums staging.  rets[i] is the byte count
// of item i (<= 0: no bytes).
template <uint32_t WGMAX, uint32_t CH>
__global__ __launch_bounds__(WGMAX, WGMAX <= 256 ? 2 : 4) void fnv4k_consume(
    uint64_t staging, const int64_t* rets, uint64_t n_items, uint32_t item_bytes,
    uint64_t* out_fnv) {
  extern __shared__ __align__(16) uint8_t lds[];
  const uint32_t wave = threadIdx.x >> 6;
  for (uint64_t first = (uint64_t)blockIdx.x * blockDim.x; first < n_items;
       first += (uint64_t)gridDim.x * blockDim.x) {
    const uint64_t item = first + threadIdx.x;
    const bool valid = item < n_items;
    const int64_t ret = valid ? rets[item] : 0;
    const uint32_t nbytes = ret > 0 ? (uint32_t)min<int64_t>(ret, (int64_t)item_bytes) : 0u;
    const uint64_t row0 = staging + (first + (threadIdx.x & ~63u)) * (uint64_t)item_bytes;
    const uint64_t h = wave_fnv_t<CH>(row0, nbytes, item_bytes, lds + wave * Tile<CH>::kBytes);
    if (valid) out_fnv[item] = h;
  }
}

__global__ void zero_words(unsigned long long* p, uint32_t n) {
  const uint32_t i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) p[i] = 0;
}

}  // namespace gsys_k

// ---------------------------------------------------------------- host side
using namespace gsys_k;

int gsys_fnv4k(gsys_ctx* ctx, int fd, uint64_t offsets, uint64_t n_items, uint32_t item_bytes,
               uint64_t staging, uint64_t staging_bytes, uint64_t lists, uint64_t out_fnv,
               uint64_t out_ret, uint32_t cell, uint32_t form, uint32_t wg_size, void* stream) {
  if (!ctx) return -EINVAL;
  if (!n_items) return 0;
  if (item_bytes == 0 || item_bytes % 64 || item_bytes > (1u << 20)) return -EINVAL;
  if (!(wg_size == 64 || wg_size == 128 || wg_size == 256 || wg_size == 512 || wg_size == 1024))
    return -EINVAL;
  if (!offsets || !out_fnv || !out_ret) return -EINVAL;
  if (n_items > (1ull << 32)) return -EINVAL;
  const uint64_t stage_bytes = n_items * (uint64_t)item_bytes;
  if (!staging_bytes) staging_bytes = stage_bytes;
  if (gsys_internal::check_host_range(ctx, staging, staging_bytes)) return -EFAULT;
  const bool persistent = form == GSYS_PERSISTENT || form == GSYS_GRAPH;
  const uint64_t batch_bytes = (uint64_t)wg_size * item_bytes;
  if (staging_bytes < stage_bytes && (!persistent || staging_bytes < 2 * batch_bytes))
    return -EINVAL;
  if (gsys_internal::check_host_range(ctx, lists, n_items * sizeof(gsys_iodesc))) return -EFAULT;

  FnvArgs A;
  if (int e = gsys_device_ctx(ctx, &A.c)) return e;
  A.offsets = (const uint64_t*)offsets;
  A.n_items = n_items;
  A.staging = staging;
  A.lists = (gsys_iodesc*)lists;
  A.out_fnv = (uint64_t*)out_fnv;
  A.out_ret = (int64_t*)out_ret;
  A.ks = (KState*)gsys_internal::kstate(ctx);
  A.fd = fd;
  A.item_bytes = item_bytes;
  A.ring = 0;
  {
    // Strong work-group cells aggregate their descriptor list in LDS before
    // one wavefront copies it out; GSYS_LDS_LISTS=0 has every work-item write
    // its own descriptor to host memory instead (measured equal, within 1%,
    // on the full sweep: the host pool, not the list, bounds these cells)
    const char* e = getenv("GSYS_LDS_LISTS");
    A.lds_list = (e && *e == '0') ? 0u : 1u;
  }
  hipStream_t s = (hipStream_t)stream;
  const bool small = wg_size <= 256;
  const uint32_t lds = (wg_size / 64) * (small ? Tile<256>::kBytes : Tile<128>::kBytes);

  if (form == GSYS_PERSISTENT || form == GSYS_GRAPH) {
    const uint64_t nb = (n_items + wg_size - 1) / wg_size;
    const void* kp = small ? (const void*)fnv4k_persistent<256> : (const void*)fnv4k_persistent<1024>;
    uint32_t grid = gsys_internal::resident_grid(ctx, kp, wg_size, lds);
    if (grid == 0) return -ENODEV;
    if ((uint64_t)grid > nb) grid = (uint32_t)nb;
    const uint32_t req = gsys_internal::persistent_grid_override(ctx);
    if (req && req < grid) grid = req;
    // waiting work-groups poll host memory: no more of them than keep the
    // host pool and the link busy
    if (!req && grid > kPersistentGrid) grid = kPersistentGrid;
    if (staging_bytes < stage_bytes) {
      // staging ring: two batch buffers per resident work-group
      A.ring = 1;
      const uint64_t fit = staging_bytes / (2 * batch_bytes);
      if ((uint64_t)grid > fit) grid = (uint32_t)fit;
    }
    void* args[] = {&A};
    if (form == GSYS_GRAPH) {
      const uint64_t key = gsys_internal::hash_words({0xF4Bull, (uint64_t)kp, grid, wg_size, lds});
      const gsys_internal::KLaunch k{kp, dim3(grid), dim3(wg_size), lds, args};
      return gsys_internal::launch_graph(ctx, key, &k, 1, s);
    }
    return gsys_internal::launch(ctx, kp, grid, wg_size, lds, args, s);
  }

  const uint32_t gran = GSYS_CELL_GRAN(cell);
  const bool strong = (cell & GSYS_CELL_STRONG) != 0;
  const bool blocking = (cell & GSYS_CELL_BLOCKING) != 0;
  const uint64_t grid64 = (n_items + wg_size - 1) / wg_size;
  if (grid64 > 0x7fffffffull) return -EINVAL;
  const uint32_t grid = (uint32_t)grid64;
  const void* k = nullptr;
  if (gran == GSYS_GRAN_WI) {
    if (!strong) return -EINVAL;  // work-item calls are implicitly strong
    k = blocking ? (small ? (const void*)fnv4k_plain<G::WorkItem, O::Strong, B::Blocking, 256> : (const void*)fnv4k_plain<G::WorkItem, O::Strong, B::Blocking, 1024>)
                 : (small ? (const void*)fnv4k_plain<G::WorkItem, O::Strong, B::NonBlocking, 256> : (const void*)fnv4k_plain<G::WorkItem, O::Strong, B::NonBlocking, 1024>);
  } else if (gran == GSYS_GRAN_WG) {
    if (strong)
      k = blocking ? (small ? (const void*)fnv4k_plain<G::WorkGroup, O::Strong, B::Blocking, 256> : (const void*)fnv4k_plain<G::WorkGroup, O::Strong, B::Blocking, 1024>)
                   : (small ? (const void*)fnv4k_plain<G::WorkGroup, O::Strong, B::NonBlocking, 256> : (const void*)fnv4k_plain<G::WorkGroup, O::Strong, B::NonBlocking, 1024>);
    else
      k = blocking ? (small ? (const void*)fnv4k_plain<G::WorkGroup, O::Relaxed, B::Blocking, 256> : (const void*)fnv4k_plain<G::WorkGroup, O::Relaxed, B::Blocking, 1024>)
                   : (small ? (const void*)fnv4k_plain<G::WorkGroup, O::Relaxed, B::NonBlocking, 256> : (const void*)fnv4k_plain<G::WorkGroup, O::Relaxed, B::NonBlocking, 1024>);
  } else if (gran == GSYS_GRAN_KERNEL) {
    if (strong) return -EINVAL;  // kernel calls are relaxed only
    if (stage_bytes > 0xffffffffull) return -EINVAL;  // descriptor offsets are 32-bit
    k = blocking ? (small ? (const void*)fnv4k_plain<G::Kernel, O::Relaxed, B::Blocking, 256> : (const void*)fnv4k_plain<G::Kernel, O::Relaxed, B::Blocking, 1024>)
                 : (small ? (const void*)fnv4k_plain<G::Kernel, O::Relaxed, B::NonBlocking, 256> : (const void*)fnv4k_plain<G::Kernel, O::Relaxed, B::NonBlocking, 1024>);
    // fresh per-launch state for the kernel-granularity call site
    if (gsys_internal::no_device(ctx)) return -ENODEV;
    hipLaunchKernelGGL(zero_words, dim3(1), dim3(64), 0, s, (unsigned long long*)A.ks,
                       (uint32_t)(sizeof(KState) / 8));
    if (hipGetLastError() != hipSuccess) return -ENODEV;
  } else {
    return -EINVAL;
  }
  void* args[] = {&A};
  return gsys_internal::launch(ctx, k, grid, wg_size, lds, args, s);
}

int gsys_fnv4k_consume(gsys_ctx* ctx, uint64_t staging, uint64_t rets, uint64_t n_items,
                       uint32_t item_bytes, uint64_t out_fnv, uint32_t wg_size, uint32_t grid,
                       void* stream) {
  if (!ctx) return -EINVAL;
  if (!n_items) return 0;  // the outputs are empty and may be null
  if (!staging || !rets || !out_fnv) return -EINVAL;
  if (item_bytes == 0 || item_bytes % 64 || item_bytes > (1u << 20)) return -EINVAL;
  if (!(wg_size == 64 || wg_size == 128 || wg_size == 256 || wg_size == 512 || wg_size == 1024))
    return -EINVAL;
  const uint64_t nb = (n_items + wg_size - 1) / wg_size;
  if (!grid || grid > nb) grid = (uint32_t)std::min<uint64_t>(nb, 0x7fffffffull);
  const bool small = wg_size <= 256;
  const uint32_t lds = (wg_size / 64) * (small ? Tile<256>::kBytes : Tile<128>::kBytes);
  void* args[] = {&staging, &rets, &n_items, &item_bytes, &out_fnv};
  const void* k = small ? (const void*)fnv4k_consume<256, 256> : (const void*)fnv4k_consume<1024, 128>;
  return gsys_internal::launch(ctx, k, grid, wg_size, lds, args, (hipStream_t)stream);
}
