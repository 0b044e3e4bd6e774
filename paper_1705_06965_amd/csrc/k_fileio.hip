// Stateful file calls from the GPU: read() and write() advance the file
// offset of the description they go through, so their results depend on the
// order the host executes them in (section 4.1 and section 8.1 discuss calls
// whose effect is order-dependent).  Both workloads here issue every
// stateful call blocking, one at a time per description, which makes that
// order the program order of the caller.
//
//  * Work-group round trip: every work-group opens its own file by name
//    beneath an allowed directory (openat, created and truncated), writes
//    its bytes in pieces with write(), closes it, opens it again read-only,
//    reads it back in the same pieces with read() plus one read at the end
//    of the file (which must return 0), closes it, and compares what it
//    read against the bytes it wrote.  The writes are producers (section
//    4.1): the group's stores into the piece's staging are released and
//    the group synchronised before each write, under strong or relaxed
//    ordering.
//  * Kernel granularity: one write() or read() for the whole kernel through
//    a descriptor the caller opened.  For a write every work-group stores its
//    slice of the data into staging and the last work-group to arrive makes
//    the call; for a read the first work-group to arrive makes the call and
//    every work-group then checks its slice.  Consecutive launches therefore
//    append to (or consume) the file in launch order.
#include "gsys_device.hpp"
#include "gsys.h"
#include "kernels.hpp"

#include <fcntl.h>

#include <algorithm>

namespace gsys_fio {

using namespace gsys;

constexpr uint32_t kWG = 256;
constexpr uint32_t kEofRead = 16;  // bytes asked for by the read at the end of the file

struct RtArgs {
  gsys_dev_ctx c;
  uint64_t paths;        // registered host buffer: nfiles x GSYS_PATH_MAX bytes
  const uint8_t* data;   // device: nfiles x file_bytes
  uint64_t staging;      // registered host buffer: per file, write area then read area
  uint64_t area;         // bytes of each area (>= max(file_bytes, kEofRead), 16-aligned)
  int64_t* rets;         // device: nfiles x (2 * pieces + 5)
  unsigned long long* mismatch;  // device: nfiles
  uint64_t file_bytes;
  uint32_t piece;
  uint32_t pieces;
  int32_t dirfd;
};

// The work-group copies n bytes from HBM to host staging: 16-byte vectors
// when both ends are 16-byte aligned, then the remaining bytes one by one.
__device__ __forceinline__ void copy_to_host(uint64_t dst, const uint8_t* src, uint64_t n) {
  uint64_t head = 0;
  if (((dst | (uint64_t)src) & 15) == 0) {
    const uint64_t nv = n / 16;
    for (uint64_t i = threadIdx.x; i < nv; i += blockDim.x)
      stg16(dst + 16 * i, ldg16((uint64_t)src + 16 * i));
    head = nv * 16;
  }
  for (uint64_t i = head + threadIdx.x; i < n; i += blockDim.x) gp<uint8_t>(dst)[i] = src[i];
}

template <O o>
__global__ __launch_bounds__(kWG) void roundtrip(RtArgs A) {
  const uint32_t f = blockIdx.x;
  const uint64_t R = 2ull * A.pieces + 5;
  int64_t* rets = A.rets + (uint64_t)f * R;
  const uint64_t wst = A.staging + (uint64_t)f * 2 * A.area;
  const uint64_t rst = wst + A.area;
  const uint8_t* src = A.data + (uint64_t)f * A.file_bytes;
  const uint64_t path = A.paths + (uint64_t)f * GSYS_PATH_MAX;
  uint32_t k = 0;  // next entry of rets

  auto put = [&](int64_t r) {
    if (threadIdx.x == 0) rets[k] = r;
    ++k;
  };
  auto piece_len = [&](uint32_t p) {
    return (uint32_t)min<uint64_t>(A.piece, A.file_bytes - (uint64_t)p * A.piece);
  };

  // write phase: openat is a consumer (every work-item needs the descriptor)
  const int64_t wfd = call_wg<O::Relaxed, B::Blocking>(
      A.c, GSYS_NR_OPENAT, 0,
      Args6{{(uint64_t)(int64_t)A.dirfd, path, (uint64_t)(O_WRONLY | O_CREAT | O_TRUNC), 0600, 0,
             0}});
  put(wfd);
  if (wfd < 0) return;
  for (uint32_t p = 0; p < A.pieces; ++p) {
    const uint32_t n = piece_len(p);
    copy_to_host(wst + (uint64_t)p * A.piece, src + (uint64_t)p * A.piece, n);
    // a producer: the call's barrier before makes every work-item's stores
    // visible to the host first
    const int64_t r = call_wg<o, B::Blocking>(
        A.c, GSYS_NR_WRITE, 0,
        Args6{{(uint64_t)wfd, wst + (uint64_t)p * A.piece, n, 0, 0, 0}});
    // relaxed producers return the result to the caller's wavefront only
    put(r);
  }
  put(call_wg<O::Relaxed, B::Blocking>(A.c, GSYS_NR_CLOSE, 0, Args6{{(uint64_t)wfd, 0, 0, 0, 0, 0}}));

  // read phase
  const int64_t rfd = call_wg<O::Relaxed, B::Blocking>(
      A.c, GSYS_NR_OPENAT, 0,
      Args6{{(uint64_t)(int64_t)A.dirfd, path, (uint64_t)O_RDONLY, 0, 0, 0}});
  put(rfd);
  if (rfd < 0) return;
  for (uint32_t p = 0; p < A.pieces; ++p)
    put(call_wg<O::Relaxed, B::Blocking>(
        A.c, GSYS_NR_READ, 0,
        Args6{{(uint64_t)rfd, rst + (uint64_t)p * A.piece, piece_len(p), 0, 0, 0}}));
  put(call_wg<O::Relaxed, B::Blocking>(A.c, GSYS_NR_READ, 0,
                                       Args6{{(uint64_t)rfd, rst, kEofRead, 0, 0, 0}}));
  put(call_wg<O::Relaxed, B::Blocking>(A.c, GSYS_NR_CLOSE, 0, Args6{{(uint64_t)rfd, 0, 0, 0, 0, 0}}));

  // the reads were consumers: their barrier after orders the loads below
  // after the host's data; the end-of-file read stored nothing
  uint32_t bad = 0;
  const gptr_t<const uint8_t> back = gp<const uint8_t>(rst);
  for (uint64_t i = threadIdx.x; i < A.file_bytes; i += blockDim.x) bad += back[i] != src[i];
  if (bad) atomicAdd(&A.mismatch[f], (unsigned long long)bad);
}

struct KioArgs {
  gsys_dev_ctx c;
  KState* ks;
  const uint8_t* data;   // device: the bytes to write / expected bytes
  uint64_t staging;      // registered host buffer of `bytes`
  uint64_t bytes;
  int64_t* ret;          // device: [0] the call's result
  unsigned long long* mismatch;  // device: [0]
  int32_t fd;
};

__device__ __forceinline__ void slice(uint64_t bytes, uint64_t* lo, uint64_t* hi) {
  const uint64_t per = (bytes + gridDim.x - 1) / gridDim.x;
  *lo = min<uint64_t>(bytes, (uint64_t)blockIdx.x * per);
  *hi = min<uint64_t>(bytes, *lo + per);
}

// Kernel-granularity write: a producer, so the last work-group to arrive
// makes the call after every work-group has stored its slice.
__global__ __launch_bounds__(kWG) void kernel_write(KioArgs A) {
  uint64_t lo, hi;
  slice(A.bytes, &lo, &hi);
  copy_to_host(A.staging + lo, A.data + lo, hi - lo);
  const int64_t r = call_kernel<B::Blocking>(
      A.c, A.ks, GSYS_NR_WRITE, 0, [] {},
      [&] { return Args6{{(uint64_t)(int64_t)A.fd, A.staging, A.bytes, 0, 0, 0}}; });
  if (threadIdx.x == 0 && r != GSYS_NOT_WAITED) A.ret[0] = r;
}

// Kernel-granularity read: a consumer, so the first work-group to arrive
// makes the call and every work-group waits for it before checking its
// slice of what was read.
__global__ __launch_bounds__(kWG) void kernel_read(KioArgs A) {
  const int64_t r = call_kernel<B::Blocking>(
      A.c, A.ks, GSYS_NR_READ, 0, [] {},
      [&] { return Args6{{(uint64_t)(int64_t)A.fd, A.staging, A.bytes, 0, 0, 0}}; });
  if (blockIdx.x == 0 && threadIdx.x == 0) A.ret[0] = r;
  if (r < 0) return;
  uint64_t lo, hi;
  slice(min<uint64_t>(A.bytes, (uint64_t)r), &lo, &hi);
  const gptr_t<const uint8_t> back = gp<const uint8_t>(A.staging);
  uint32_t bad = 0;
  for (uint64_t i = lo + threadIdx.x; i < hi; i += blockDim.x) bad += back[i] != A.data[i];
  if (bad) atomicAdd(&A.mismatch[0], (unsigned long long)bad);
}

__global__ void zero_words(unsigned long long* p, uint64_t n) {
  for (uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n;
       i += (uint64_t)gridDim.x * blockDim.x)
    p[i] = 0;
}

}  // namespace gsys_fio

using namespace gsys_fio;

int gsys_file_roundtrip(gsys_ctx* ctx, int dirfd, uint64_t paths, uint32_t nfiles, uint64_t data,
                        uint64_t file_bytes, uint32_t piece, uint64_t staging,
                        uint64_t staging_bytes, uint64_t rets, uint64_t mismatch, uint32_t cell,
                        void* stream) {
  if (!ctx || !piece || file_bytes > (1ull << 31)) return -EINVAL;
  // stateful calls are issued blocking, at work-group granularity
  if (GSYS_CELL_GRAN(cell) != GSYS_GRAN_WG || !(cell & GSYS_CELL_BLOCKING)) return -EINVAL;
  const uint64_t pieces = (file_bytes + piece - 1) / piece;
  if (pieces > (1u << 20)) return -EINVAL;
  if (!nfiles) return 0;  // the outputs are empty and may be null
  if (!rets || !mismatch || (file_bytes && !data)) return -EINVAL;
  const uint64_t area = (std::max<uint64_t>(file_bytes, kEofRead) + 15) & ~15ull;
  if (staging_bytes < 2 * area * nfiles) return -EINVAL;
  if (gsys_internal::check_host_range(ctx, staging, 2 * area * nfiles)) return -EFAULT;
  if (gsys_internal::check_host_range(ctx, paths, (uint64_t)nfiles * GSYS_PATH_MAX)) return -EFAULT;
  hipStream_t s = (hipStream_t)stream;
  RtArgs A;
  if (int e = gsys_device_ctx(ctx, &A.c)) return e;
  A.paths = paths;
  A.data = (const uint8_t*)data;
  A.staging = staging;
  A.area = area;
  A.rets = (int64_t*)rets;
  A.mismatch = (unsigned long long*)mismatch;
  A.file_bytes = file_bytes;
  A.piece = piece;
  A.pieces = (uint32_t)pieces;
  A.dirfd = dirfd;
  if (gsys_internal::no_device(ctx)) return -ENODEV;
  hipLaunchKernelGGL(zero_words, dim3((nfiles + 255) / 256), dim3(256), 0, s,
                     (unsigned long long*)mismatch, (uint64_t)nfiles);
  if (hipGetLastError() != hipSuccess) return -ENODEV;
  const void* k = (cell & GSYS_CELL_STRONG) ? (const void*)roundtrip<O::Strong>
                                             : (const void*)roundtrip<O::Relaxed>;
  void* args[] = {&A};
  return gsys_internal::launch(ctx, k, nfiles, kWG, 0, args, s);
}

int gsys_file_kernel_io(gsys_ctx* ctx, int fd, uint32_t nr, uint64_t data, uint64_t bytes,
                        uint64_t staging, uint64_t ret, uint64_t mismatch, uint32_t grid,
                        void* stream) {
  if (!ctx || !data || !ret || !mismatch || !bytes || !grid) return -EINVAL;
  if (nr != GSYS_NR_WRITE && nr != GSYS_NR_READ) return -EINVAL;
  if (bytes > (1ull << 31) || grid > 65535) return -EINVAL;
  if (gsys_internal::check_host_range(ctx, staging, bytes)) return -EFAULT;
  hipStream_t s = (hipStream_t)stream;
  KioArgs A;
  if (int e = gsys_device_ctx(ctx, &A.c)) return e;
  A.ks = (KState*)gsys_internal::kstate(ctx);
  A.data = (const uint8_t*)data;
  A.staging = staging;
  A.bytes = bytes;
  A.ret = (int64_t*)ret;
  A.mismatch = (unsigned long long*)mismatch;
  A.fd = fd;
  if (gsys_internal::no_device(ctx)) return -ENODEV;
  hipLaunchKernelGGL(zero_words, dim3(1), dim3(64), 0, s, (unsigned long long*)A.ks,
                     (uint64_t)(sizeof(KState) / 8));
  hipLaunchKernelGGL(zero_words, dim3(1), dim3(64), 0, s, (unsigned long long*)mismatch,
                     (uint64_t)1);
  if (hipGetLastError() != hipSuccess) return -ENODEV;
  void* args[] = {&A};
  const void* k = nr == GSYS_NR_WRITE ? (const void*)kernel_write : (const void*)kernel_read;
  return gsys_internal::launch(ctx, k, grid, kWG, 0, args, s);
}
