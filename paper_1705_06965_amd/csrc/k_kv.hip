// Key-value GET server on the GPU over loopback UDP: the network case study
// of section 7.3 (a server whose GPU part receives and answers datagrams with
// recvfrom / sendto at work-group granularity, blocking, relaxed), serving GET
// requests from a GPU-resident hash table instead of echoing.
//
// Request datagram (32 B): u64 id; u8 op (1 = GET); u8 pad[7]; u8 key[16].
// Reply datagram (16 + len B): u64 id; u8 status (0 hit, 1 miss, 2 bad
// request); u8 pad; u16 len; u32 pad; value[len].  A request of any other
// length or op gets status 2 with the id taken from its first 8 bytes (0 if
// shorter).
//
// Table: open addressing in HBM, bucket = floor(hash * cap / 2^64) with
// hash = FNV-1a-64 of the key, linear probing; 32-byte buckets.  Values live
// in an HBM heap, each 16-byte aligned.
//
// Server loop of one work-group: a recvfrom list call of up to 256
// datagrams (relaxed consumer), lookups by every lane that got a datagram,
// replies copied by whole wavefronts into pinned host staging (one reply per
// step, 64 lanes x 16 B, coalesced), then a sendto list call (relaxed
// producer: the barrier comes before it).  Two forms of the loop:
//   pipelined (default): two sets of lists and buffers; the receive of the
//     next batch is in flight while this one is answered, and sends are
//     non-blocking, waited for only before their set is reused, so the host
//     pool always holds a call of every work-group;
//   blocking (GSYS_KV_BLOCKING): one set; each receive and send is a
//     blocking call (only the caller's wavefront waits for a send).
#include "gsys_device.hpp"
#include "gsys.h"
#include "kernels.hpp"

#include <algorithm>

namespace gsys_kv {

using namespace gsys;

constexpr uint32_t kWG = 256;
constexpr uint32_t kReqBuf = 64;              // bytes per received datagram slot
constexpr uint32_t kRepBuf = 1040;            // bytes per reply slot (16 + 1024)

struct Bucket {
  uint64_t k0, k1;   // key bytes 0..7, 8..15 (little-endian words)
  uint64_t voff;     // heap offset (16-byte aligned)
  uint32_t vlen;
  uint32_t used;
};
static_assert(sizeof(Bucket) == 32, "bucket is 32 bytes");

// Per-work-group I/O region in pinned host memory: two sets of lists and
// buffers (the blocking loop uses the first).
constexpr uint32_t kOffRecvList = 0;
static_assert(sizeof(gsys_netdesc) == 32, "descriptors are written as two 16-byte vectors");
constexpr uint32_t kOffSendList = kOffRecvList + kWG * sizeof(gsys_netdesc);
constexpr uint32_t kOffRecv = kOffSendList + kWG * sizeof(gsys_netdesc);
constexpr uint32_t kOffSend = kOffRecv + kWG * kReqBuf;
constexpr uint32_t kSetBytes = kOffSend + kWG * kRepBuf;
constexpr uint32_t kIoBytes = 2 * kSetBytes;

__device__ __forceinline__ uint64_t fnv16(uint64_t k0, uint64_t k1) {
  uint64_t h = 0xcbf29ce484222325ull;
#pragma unroll
  for (int i = 0; i < 8; ++i) {
    h ^= (k0 >> (8 * i)) & 0xffu;
    h *= 0x100000001b3ull;
  }
#pragma unroll
  for (int i = 0; i < 8; ++i) {
    h ^= (k1 >> (8 * i)) & 0xffu;
    h *= 0x100000001b3ull;
  }
  return h;
}

__global__ void zero_u64(uint64_t* p, uint64_t n) {
  for (uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n;
       i += (uint64_t)gridDim.x * blockDim.x)
    p[i] = 0;
}

__global__ void kv_build(Bucket* tab, uint64_t cap, const uint8_t* keys, const uint64_t* voff,
                         const uint32_t* vlen, uint64_t n) {
  const uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  const uint64_t k0 = reinterpret_cast<const uint64_t*>(keys)[2 * i];
  const uint64_t k1 = reinterpret_cast<const uint64_t*>(keys)[2 * i + 1];
  uint64_t b = __umul64hi(fnv16(k0, k1), cap);
  for (uint64_t n_probe = 0; n_probe < cap; ++n_probe) {
    if (atomicCAS(&tab[b].used, 0u, 1u) == 0u) {
      tab[b].k0 = k0;
      tab[b].k1 = k1;
      tab[b].voff = voff[i];
      tab[b].vlen = vlen[i];
      return;
    }
    b = b + 1 == cap ? 0 : b + 1;
  }
}

struct KvArgs {
  gsys_dev_ctx c;
  const Bucket* tab;
  uint64_t cap;
  const uint8_t* heap;
  uint64_t io;                     // base of the work-groups' I/O regions
  const uint64_t* stop;            // host-coherent: nonzero = exit
  unsigned long long* served;      // device: datagrams answered
  uint64_t lifetime_ticks;         // the server exits after this long regardless
  int32_t fd;
  uint32_t batch;                  // datagrams per recvfrom list (<= 256)
};

// One set of a work-group's lists and buffers.
struct IoSet {
  gsys_netdesc* rl;   // receive list
  gsys_netdesc* sl;   // send list
  uint8_t* rbuf;      // received datagrams, kReqBuf each
  uint8_t* sbuf;      // replies, kRepBuf each
  uint64_t rbase, sbase;
};

__device__ __forceinline__ IoSet io_set(const KvArgs& A, uint32_t k) {
  const uint64_t base = A.io + (uint64_t)blockIdx.x * kIoBytes + (uint64_t)k * kSetBytes;
  uint8_t* io = reinterpret_cast<uint8_t*>(base);
  return IoSet{reinterpret_cast<gsys_netdesc*>(io + kOffRecvList),
               reinterpret_cast<gsys_netdesc*>(io + kOffSendList), io + kOffRecv, io + kOffSend,
               base + kOffRecv, base + kOffSend};
}

// The receive list of a set: batch empty datagram slots.  Written by the
// caller's wavefront only (a relaxed consumer call has no barrier before it);
// every work-item calls this.  Returns the call's result to every work-item
// (blocking) or GSYS_NOT_WAITED with the ticket in *tk on thread 0.
template <B b>
__device__ __forceinline__ int64_t post_recv(const KvArgs& A, const IoSet& S, Ticket* tk) {
  const uint32_t tid = threadIdx.x;
  if (tid < 64)
    for (uint32_t i = tid; i < A.batch; i += 64) {
      // {buf_off, len_ret, addr_len, pad}, then an empty address
      stg16((uint64_t)(S.rl + i), u32x4{i * kReqBuf, kReqBuf, 0u, 0u});
      stg16((uint64_t)(S.rl + i) + 16, u32x4{0u, 0u, 0u, 0u});
    }
  Args6 ra{{(uint64_t)(int64_t)A.fd, (uint64_t)S.rl, A.batch, S.rbase, 0, 0}};
  return call_wg<O::Relaxed, b>(A.c, GSYS_NR_RECVFROM, GSYS_F_LIST, ra, tk);
}

// This work-item's datagram of a completed receive list, if it got one
// (datagrams arrive as a prefix of the list: the host stops at -EAGAIN).
// `ret` is the list call's result: when it failed, the list is not read at
// all (a call the host never ran leaves every descriptor as the GPU wrote
// it), and the batch is dropped: clients send again, and a GET is
// idempotent.
__device__ __forceinline__ int32_t received(const KvArgs& A, const IoSet& S, int64_t ret) {
  const uint32_t tid = threadIdx.x;
  if (ret < 0) return -1;
  return tid < A.batch ? __hip_atomic_load(gp(&S.rl[tid].len_ret), __ATOMIC_RELAXED,
                                           __HIP_MEMORY_SCOPE_SYSTEM)
                       : -1;
}

// A call failure that ends the server: the host stopped serving the
// context, or a wait outlived the watchdog.
__device__ __forceinline__ bool fatal(int64_t ret) {
  return ret == GSYS_ETIMEDOUT_RET || ret == GSYS_ESHUTDOWN_RET;
}

// Look up every received request and write its reply and send descriptor
// into the set.  Every work-item calls this.
__device__ void answer(const KvArgs& A, const IoSet& S, int32_t got) {
  const uint32_t tid = threadIdx.x;
  const uint32_t lane = lane_id();
  const bool have = got >= 0;
  uint64_t id = 0, voff = 0;
  uint32_t status = 2, vlen = 0;
  if (have) {
    const uint8_t* q = S.rbuf + tid * kReqBuf;
    const u32x4 w0 = ldg16((uint64_t)q);
    const u32x4 w1 = ldg16((uint64_t)(q + 16));
    if (got >= 8) id = ((uint64_t)w0.y << 32) | w0.x;
    if (got == 32 && (w0.z & 0xffu) == 1u) {
      const uint64_t k0 = ((uint64_t)w1.y << 32) | w1.x;
      const uint64_t k1 = ((uint64_t)w1.w << 32) | w1.z;
      uint64_t b = __umul64hi(fnv16(k0, k1), A.cap);
      status = 1;
      for (uint64_t p = 0; p < A.cap; ++p) {
        const gptr_t<const Bucket> bk = gp<const Bucket>((uint64_t)(A.tab + b));
        if (!bk->used) break;
        if (bk->k0 == k0 && bk->k1 == k1) {
          status = 0;
          voff = bk->voff;
          vlen = bk->vlen;
          break;
        }
        b = b + 1 == A.cap ? 0 : b + 1;
      }
    }
    // reply descriptor {buf_off, len_ret, addr_len, pad, addr}: back to
    // the sender recvfrom reported
    const u32x4 rh = ldg16((uint64_t)(S.rl + tid));
    const u32x4 ra = ldg16((uint64_t)(S.rl + tid) + 16);
    stg16((uint64_t)(S.sl + tid), u32x4{tid * kRepBuf, 16u + vlen, rh.z, 0u});
    stg16((uint64_t)(S.sl + tid) + 16, ra);
  }
  // replies: one wavefront copies one reply per step, 16 B per lane
  uint64_t m = __ballot(have);
  while (m) {
    const uint32_t j = first_lane(m);
    m &= m - 1;
    const uint64_t jid = bcast64(id, j);
    const uint64_t jvoff = bcast64(voff, j);
    const uint32_t jst = __builtin_amdgcn_readlane(status, j);
    const uint32_t jlen = __builtin_amdgcn_readlane(vlen, j);
    uint8_t* dst = S.sbuf + (uint64_t)((tid & ~63u) + j) * kRepBuf;
    const uint32_t chunks = 1 + (jlen + 15) / 16;
    for (uint32_t c = lane; c < chunks; c += 64) {
      u32x4 v;
      if (c == 0) {
        v = u32x4{(uint32_t)jid, (uint32_t)(jid >> 32), jst | (jlen << 16), 0u};
      } else {
        v = ldg16((uint64_t)(A.heap + jvoff + 16 * (c - 1)));
      }
      stg16((uint64_t)(dst + 16 * c), v);
    }
  }
}

// Back off before asking an empty socket again (thread 0 sleeps; the
// barrier ends its region before the loop's back edge, where the next
// iteration opens with another thread-0 region: two such regions joined
// across a back edge can leave thread 0 out of the following barrier).
__device__ __forceinline__ void idle_backoff(uint32_t idle) {
  if (threadIdx.x == 0) {
    const uint32_t reps = 1u << min(idle, 8u);
    for (uint32_t r = 0; r < reps; ++r) __builtin_amdgcn_s_sleep(8);
  }
  __syncthreads();
}

__device__ __forceinline__ bool stop_now(const KvArgs& A, uint64_t t_end) {
  __shared__ int s_stop;
  if (threadIdx.x == 0) s_stop = ld_sys(A.stop) != 0 || wall_clock64() > t_end;
  __syncthreads();
  const bool r = s_stop != 0;
  __syncthreads();  // s_stop is written again by the next check
  return r;
}

__global__ __launch_bounds__(kWG) void kv_serve(KvArgs A) {
  const uint32_t tid = threadIdx.x;
  const IoSet S = io_set(A, 0);
  uint32_t idle = 0;
  const uint64_t t_end = wall_clock64() + A.lifetime_ticks;
  for (;;) {
    if (stop_now(A, t_end)) break;
    const int64_t rr = post_recv<B::Blocking>(A, S, nullptr);
    if (fatal(rr)) break;
    const int32_t got = received(A, S, rr);
    const uint32_t n = (uint32_t)__syncthreads_count(got >= 0);
    if (n == 0) {
      idle_backoff(idle++);
      continue;
    }
    idle = 0;
    answer(A, S, got);
    // send the replies (producer call: every lane's reply is released before)
    Args6 sa{{(uint64_t)(int64_t)A.fd, (uint64_t)S.sl, n, S.sbase, 0, 0}};
    call_wg<O::Relaxed, B::Blocking>(A.c, GSYS_NR_SENDTO, GSYS_F_LIST, sa);
    if (tid == 0) atomicAdd(A.served, (unsigned long long)n);
    // the caller's wavefront waited for the sends; the rest wait here before
    // the buffers are reused
    __syncthreads();
  }
}

__global__ __launch_bounds__(kWG) void kv_serve_pipelined(KvArgs A) {
  const uint32_t tid = threadIdx.x;
  // tickets are meaningful on thread 0; send_busy is uniform
  Ticket r0{0, 0, 0}, r1{0, 0, 0}, s0{0, 0, 0}, s1{0, 0, 0};
  bool send_busy0 = false, send_busy1 = false;
  uint32_t idle = 0, k = 0;
  const uint64_t t_end = wall_clock64() + A.lifetime_ticks;
  post_recv<B::NonBlocking>(A, io_set(A, 0), &r0);
  for (;;) {
    if (stop_now(A, t_end)) break;
    const IoSet S = io_set(A, k);
    // the next batch's receive goes out before this one is answered (its
    // set was answered in the previous step)
    Ticket nr{0, 0, 0};
    post_recv<B::NonBlocking>(A, io_set(A, k ^ 1u), &nr);
    if (k) r0 = nr;
    else r1 = nr;
    const Ticket rt = k ? r1 : r0;  // by value: a selected reference would live in memory
    const int64_t rr = wait_wg(A.c, rt);
    if (fatal(rr)) {
      k ^= 1u;  // the receive just posted is the one in flight
      break;
    }
    const int32_t got = received(A, S, rr);
    const uint32_t n = (uint32_t)__syncthreads_count(got >= 0);
    if (n == 0) {
      idle_backoff(idle++);
      k ^= 1u;
      continue;
    }
    idle = 0;
    // the set's previous send must be done before its list and replies are
    // rewritten
    if (k ? send_busy1 : send_busy0) {
      const Ticket wt = k ? s1 : s0;
      wait_wg(A.c, wt);
    }
    answer(A, S, got);
    Args6 sa{{(uint64_t)(int64_t)A.fd, (uint64_t)S.sl, n, S.sbase, 0, 0}};
    Ticket st{0, 0, 0};
    call_wg<O::Relaxed, B::NonBlocking>(A.c, GSYS_NR_SENDTO, GSYS_F_LIST, sa, &st);
    if (k) {
      s1 = st;
      send_busy1 = true;
    } else {
      s0 = st;
      send_busy0 = true;
    }
    if (tid == 0) atomicAdd(A.served, (unsigned long long)n);
    __syncthreads();  // closes the thread-0 region before the back edge
    k ^= 1u;
  }
  // the receive in flight and the sends not yet waited for finish before
  // the work-group leaves (stop is raised once every request is answered,
  // so the receive finds an empty socket)
  const Ticket last = k ? r1 : r0;
  wait_wg(A.c, last);
  if (send_busy0) wait_wg(A.c, s0);
  if (send_busy1) wait_wg(A.c, s1);
}

}  // namespace gsys_kv

using namespace gsys_kv;

int gsys_kv_build(gsys_ctx* ctx, uint64_t table, uint64_t cap, uint64_t keys, uint64_t voff,
                  uint64_t vlen, uint64_t n, void* stream) {
  if (!ctx || !table || !cap || (n && (!keys || !voff || !vlen))) return -EINVAL;
  if (n > cap || cap > (1ull << 40)) return -EINVAL;  // the fill counts cap * 4 words
  if (gsys_internal::no_device(ctx)) return -ENODEV;
  hipSetDevice(gsys_internal::device_of(ctx));
  hipStream_t s = (hipStream_t)stream;
  hipLaunchKernelGGL(zero_u64, dim3((uint32_t)std::min<uint64_t>((cap + 255) / 256, 65535)),
                     dim3(256), 0, s, (uint64_t*)table, cap * 4);
  if (n)
    hipLaunchKernelGGL(kv_build, dim3((uint32_t)((n + 255) / 256)), dim3(256), 0, s, (Bucket*)table,
                       cap, (const uint8_t*)keys, (const uint64_t*)voff, (const uint32_t*)vlen, n);
  return hipGetLastError() == hipSuccess ? 0 : -ENODEV;
}

uint64_t gsys_kv_io_bytes(void) { return kIoBytes; }

int gsys_kv_serve(gsys_ctx* ctx, int fd, uint64_t table, uint64_t cap, uint64_t heap, uint64_t io,
                  uint64_t io_bytes, uint64_t stop, uint64_t served, uint32_t batch, uint32_t grid,
                  uint32_t flags, uint64_t lifetime_ms, void* stream) {
  if (!ctx || !table || !cap || !heap || !stop || !served) return -EINVAL;
  if (batch == 0 || batch > kWG) return -EINVAL;
  if (gsys_internal::check_host_range(ctx, io, io_bytes)) return -EFAULT;
  if (gsys_internal::check_host_range(ctx, stop, 8)) return -EFAULT;
  uint32_t fit = (uint32_t)std::min<uint64_t>(io_bytes / kIoBytes, 0x7fffffffull);
  if (flags & ~GSYS_KV_BLOCKING) return -EINVAL;
  const void* kernel = (flags & GSYS_KV_BLOCKING) ? (const void*)kv_serve
                                                  : (const void*)kv_serve_pipelined;
  uint32_t res = gsys_internal::resident_grid(ctx, kernel, kWG, 0);
  if (!res) return -ENODEV;
  if (!grid || grid > fit) grid = fit;
  if (grid > res) grid = res;
  if (!grid) return -EINVAL;
  KvArgs A;
  if (int e = gsys_device_ctx(ctx, &A.c)) return e;
  A.tab = (const Bucket*)table;
  A.cap = cap;
  A.heap = (const uint8_t*)heap;
  A.io = io;
  A.stop = (const uint64_t*)stop;
  A.served = (unsigned long long*)served;
  A.fd = fd;
  A.batch = batch;
  A.lifetime_ticks = gsys_internal::ticks_per_ms(ctx) * (lifetime_ms ? lifetime_ms : 60000);
  void* args[] = {&A};
  const void* k = kernel;
  return gsys_internal::launch(ctx, k, grid, kWG, 0, args, (hipStream_t)stream);
}
