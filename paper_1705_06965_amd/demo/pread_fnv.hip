// A user program of the library, written against its public headers only
// (gsys.h for the host side, gsys_device.hpp for the calls): items of a file
// are read with GPU-issued pread at one of the three granularities of
// section 4.1 and hashed with FNV-1a-64, and the kernel is started with
// gsys_launch in any of its modes.
//   work-item:  every work-item preads its own item at offsets[i]
//               (implicitly strong, blocking);
//   work-group: work-item 0 preads the group's items, which lie next to each
//               other at off0 + i * item_bytes, in one call (relaxed,
//               non-blocking, then gsys_wait);
//   kernel:     one pread of all n items for the whole launch (relaxed,
//               blocking);
//   two sites:  two kernel-granularity preads, the first half of the items
//               at call site 1 and the rest at call site 2 (each call of a
//               launch needs its own site); a call at a site past the
//               context's last one is refused with -EINVAL and makes none.
// Every kernel loops over its items with the grid's stride, so a clamped
// persistent grid covers them all.
//   late wait:  a non-blocking work-group pread whose ticket is kept in
//               device memory, `flood` more work-item calls in a second
//               launch, and the wait for the first ticket in a third.
#include <gsys.h>
#include <gsys_device.hpp>

#include <errno.h>

namespace demo {

using gsys::B;
using gsys::G;
using gsys::O;

struct Args {
  gsys_dev_ctx c;
  uint64_t staging;          // registered host buffer, n * item_bytes
  const uint64_t* offsets;   // device: item offsets (work-item form)
  uint64_t off0;             // group and kernel forms: item i at off0 + i * item_bytes
  uint64_t n;
  uint64_t* out_fnv;         // device uint64[n]
  int64_t* out_ret;          // device int64[n]: bytes of the item read, or -errno
  int32_t fd;
  uint32_t item_bytes;       // a multiple of 16
};

// FNV-1a-64 of `len` bytes of host staging at p (16-byte loads).
__device__ uint64_t fnv(uint64_t p, int64_t len) {
  uint64_t h = 0xcbf29ce484222325ull;
  for (int64_t i = 0; i < len; i += 16) {
    const gsys::u32x4 v = gsys::ldg16(p + (uint64_t)i);
    const uint32_t w[4] = {v.x, v.y, v.z, v.w};
    for (int k = 0; k < 16 && i + k < len; ++k) {
      h ^= (w[k >> 2] >> (8 * (k & 3))) & 0xffu;
      h *= 0x100000001b3ull;
    }
  }
  return h;
}

// Item i's share of a call that read `r` bytes of consecutive items from item i0 on.
__device__ __forceinline__ int64_t share(int64_t r, uint64_t i, uint64_t i0, uint32_t ib) {
  if (r < 0) return r;
  const int64_t left = r - (int64_t)((i - i0) * ib);
  return left <= 0 ? 0 : (left < (int64_t)ib ? left : (int64_t)ib);
}

__global__ void by_work_item(Args A) {
  const uint64_t stride = (uint64_t)gridDim.x * blockDim.x;
  for (uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; i < A.n; i += stride) {
    const uint64_t dst = A.staging + i * A.item_bytes;
    const int64_t r = gsys::pread<G::WorkItem>(A.c, A.fd, dst, A.item_bytes, A.offsets[i]);
    A.out_ret[i] = r;
    A.out_fnv[i] = fnv(dst, r > 0 ? r : 0);
  }
}

__global__ void by_work_group(Args A) {
  const uint64_t per = blockDim.x;
  for (uint64_t i0 = (uint64_t)blockIdx.x * per; i0 < A.n; i0 += (uint64_t)gridDim.x * per) {
    const uint64_t cnt = A.n - i0 < per ? A.n - i0 : per;
    gsys::Ticket tk{0, 0, 0};
    gsys::pread<G::WorkGroup, O::Relaxed, B::NonBlocking>(
        A.c, A.fd, A.staging + i0 * A.item_bytes, cnt * A.item_bytes, A.off0 + i0 * A.item_bytes,
        &tk);
    const int64_t r = gsys::gsys_wait<G::WorkGroup>(A.c, tk);
    const uint64_t i = i0 + threadIdx.x;
    if (threadIdx.x < cnt) {
      const int64_t got = share(r, i, i0, A.item_bytes);
      A.out_ret[i] = got;
      A.out_fnv[i] = fnv(A.staging + i * A.item_bytes, got > 0 ? got : 0);
    }
    __syncthreads();  // the group's next call starts after every item is hashed
  }
}

__global__ void by_kernel(Args A) {
  const int64_t r = gsys::pread<G::Kernel, O::Relaxed, B::Blocking>(
      A.c, A.fd, A.staging, A.n * A.item_bytes, A.off0);
  const uint64_t stride = (uint64_t)gridDim.x * blockDim.x;
  for (uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; i < A.n; i += stride) {
    const int64_t got = share(r, i, 0, A.item_bytes);
    A.out_ret[i] = got;
    A.out_fnv[i] = fnv(A.staging + i * A.item_bytes, got > 0 ? got : 0);
  }
}

__global__ void by_kernel_sites(Args A) {
  const uint64_t h = A.n / 2;
  const gsys::Args6 none{{0, 0, 0, 0, 0, 0}};
  const int64_t bad = gsys::gsys_call_site<O::Relaxed, B::Blocking>(A.c, A.c.n_ksites,
                                                                     GSYS_NR_PREAD64, none);
  const gsys::Args6 a1{{(uint64_t)(int64_t)A.fd, A.staging, h * A.item_bytes, A.off0, 0, 0}};
  const int64_t r1 = gsys::gsys_call_site<O::Relaxed, B::Blocking>(A.c, 1, GSYS_NR_PREAD64, a1);
  const gsys::Args6 a2{{(uint64_t)(int64_t)A.fd, A.staging + h * A.item_bytes,
                        (A.n - h) * A.item_bytes, A.off0 + h * A.item_bytes, 0, 0}};
  const int64_t r2 = gsys::gsys_call_site<O::Relaxed, B::Blocking>(A.c, 2, GSYS_NR_PREAD64, a2);
  const uint64_t stride = (uint64_t)gridDim.x * blockDim.x;
  for (uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; i < A.n; i += stride) {
    const int64_t got = i < h ? share(r1, i, 0, A.item_bytes) : share(r2, i, h, A.item_bytes);
    // a refusal that did not come back is reported as a wrong byte count
    A.out_ret[i] = bad == GSYS_EINVAL_RET ? got : -1000;
    A.out_fnv[i] = fnv(A.staging + i * A.item_bytes, got > 0 ? got : 0);
  }
}

// Late wait (three launches on one stream).  issue_late: work-group 0
// preads item_bytes at off0 without waiting and keeps its ticket.
__global__ void issue_late(Args A, gsys::Ticket* keep) {
  gsys::Ticket tk{0, 0, 0};
  gsys::pread<G::WorkGroup, O::Relaxed, B::NonBlocking>(A.c, A.fd, A.staging, A.item_bytes,
                                                         A.off0, &tk);
  if (threadIdx.x == 0) *keep = tk;
}

// flood: A.n work-item preads of 0 bytes, each result in out_ret[i].
__global__ void flood(Args A) {
  const uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < A.n) A.out_ret[i] = gsys::pread<G::WorkItem>(A.c, A.fd, A.staging, 0, 0);
}

// wait_late: work-group 0 waits for the kept ticket; the result goes to
// out_fnv[0] (as int64).
__global__ void wait_late(Args A, const gsys::Ticket* keep) {
  const gsys::Ticket tk = *keep;
  const int64_t r = gsys::gsys_wait<G::WorkGroup>(A.c, tk);
  if (threadIdx.x == 0) A.out_fnv[0] = (uint64_t)r;
}

}  // namespace demo

// gran: GSYS_GRAN_WI, GSYS_GRAN_WG, GSYS_GRAN_KERNEL, or 3 for two
// kernel-granularity calls at two call sites; mode: a gsys_launch mode.  The argument array lives on this function's stack, so every call
// passes gsys_launch the same address with new values.
extern "C" int gsys_demo_pread_fnv(gsys_ctx* ctx, uint32_t gran, uint32_t mode, uint32_t grid,
                                   uint32_t block, int fd, uint64_t staging, uint64_t offsets,
                                   uint64_t off0, uint64_t n, uint32_t item_bytes,
                                   uint64_t out_fnv, uint64_t out_ret, void* stream) {
  if (!ctx || !n || !item_bytes || item_bytes % 16 || !out_fnv || !out_ret) return -EINVAL;
  if (n * item_bytes > (1ull << 31)) return -EINVAL;
  demo::Args A;
  if (int e = gsys_device_ctx(ctx, &A.c)) return e;
  A.staging = staging;
  A.offsets = (const uint64_t*)offsets;
  A.off0 = off0;
  A.n = n;
  A.out_fnv = (uint64_t*)out_fnv;
  A.out_ret = (int64_t*)out_ret;
  A.fd = fd;
  A.item_bytes = item_bytes;
  const void* k = gran == GSYS_GRAN_WI ? (const void*)demo::by_work_item
                  : gran == GSYS_GRAN_WG ? (const void*)demo::by_work_group
                  : gran == GSYS_GRAN_KERNEL ? (const void*)demo::by_kernel
                  : gran == 3 ? (const void*)demo::by_kernel_sites : nullptr;
  if (!k || (gran == GSYS_GRAN_WI && !offsets)) return -EINVAL;
  void* args[] = {&A};
  gsys_launch_desc d;
  d.kernel = k;
  d.grid[0] = grid; d.grid[1] = 1; d.grid[2] = 1;
  d.block[0] = block; d.block[1] = 1; d.block[2] = 1;
  d.lds_bytes = 0;
  d.mode = mode;
  d.args = args;
  return gsys_launch(ctx, &d, stream);
}

// A non-blocking call's result collected late: launch 1 issues it and keeps
// the ticket in `keep` (device, 16 bytes), launch 2 makes `flood` work-item
// calls (0-byte preads; results in out_ret[flood]), launch 3 waits for the
// kept ticket (result in out_wait[0]).  All plain launches of 256
// work-items on `stream`.
extern "C" int gsys_demo_late_wait(gsys_ctx* ctx, int fd, uint64_t staging, uint32_t item_bytes,
                                   uint64_t flood, uint64_t keep, uint64_t out_ret,
                                   uint64_t out_wait, void* stream) {
  if (!ctx || !staging || !item_bytes || !keep || !out_wait || (flood && !out_ret))
    return -EINVAL;
  if (flood > (1ull << 24)) return -EINVAL;
  demo::Args A{};
  if (int e = gsys_device_ctx(ctx, &A.c)) return e;
  A.staging = staging;
  A.n = flood;
  A.out_fnv = (uint64_t*)out_wait;
  A.out_ret = (int64_t*)out_ret;
  A.fd = fd;
  A.item_bytes = item_bytes;
  gsys::Ticket* kp = (gsys::Ticket*)keep;
  void* with_keep[] = {&A, &kp};
  void* only_args[] = {&A};
  struct Step {
    const void* k;
    uint32_t grid;
    void** args;
  };
  const Step steps[3] = {{(const void*)demo::issue_late, 1, with_keep},
                         {(const void*)demo::flood, (uint32_t)((flood + 255) / 256), only_args},
                         {(const void*)demo::wait_late, 1, with_keep}};
  for (const Step& st : steps) {
    if (!st.grid) continue;
    gsys_launch_desc d;
    d.kernel = st.k;
    d.grid[0] = st.grid; d.grid[1] = 1; d.grid[2] = 1;
    d.block[0] = 256; d.block[1] = 1; d.block[2] = 1;
    d.lds_bytes = 0;
    d.mode = GSYS_PLAIN;
    d.args = st.args;
    if (int e = gsys_launch(ctx, &d, stream)) return e;
  }
  return 0;
}
