// Device side of gsys: issuing system calls from gfx950 kernels.
//
// A call is made at one of three granularities (section 4.1): by every
// work-item for itself, by one designated work-item for its work-group, or by
// one designated work-item for the whole kernel (section 5).  Each call has an
// ordering -- strong (synchronise the group before and after the call) or
// relaxed (before only for a producer such as write/send, after only for a
// consumer such as read/recv) -- and is blocking or non-blocking.  Work-item
// calls are implicitly strong; kernel calls can only be relaxed, because a
// kernel-wide barrier before the call can deadlock when not every work-item of
// the kernel is resident (section 4.1).  Both rules are compile-time errors
// here.
//
// Transport: a ring of 64-byte slots in fine-grained host-coherent memory
// (section 5's syscall area, claimed by ticket).  Work-item calls of one
// wavefront are coalesced: the active lanes are counted with a ballot, one
// lane takes a contiguous run of tickets with a single device-scope
// fetch-add, and each lane fills its own slot.  A request becomes visible to
// the host with a system-scope release store of READY; results come back in
// completion records that one lane per wavefront (or per work-group) polls
// with s_sleep backoff and a wall-clock watchdog, so a missing host answer
// ends the wait with -ETIMEDOUT instead of a hung kernel.
#pragma once

#include <hip/hip_runtime.h>
#include <hsa/amd_hsa_signal.h>
#include <stddef.h>
#include <stdint.h>

#include "gsys_abi.h"

namespace gsys {

enum class G { WorkItem, WorkGroup, Kernel };
enum class O { Strong, Relaxed };
enum class B { Blocking, NonBlocking };
enum class Role { Producer, Consumer };

// Role of each whitelisted call under relaxed ordering: data flows out of the
// GPU program for write/send (producers) and into it for read/recv
// (section 4.1).  mmap and openat hand back an address or a descriptor, so
// they are consumers; munmap, madvise and close act on memory or a file the
// program is done with, so they are producers (the paper issues madvise
// non-blocking and relaxed, section 7.2).
__host__ __device__ constexpr Role role_of(int nr) {
  return (nr == GSYS_NR_WRITE || nr == GSYS_NR_PWRITE64 || nr == GSYS_NR_SENDTO ||
          nr == GSYS_NR_MUNMAP || nr == GSYS_NR_MADVISE || nr == GSYS_NR_CLOSE)
             ? Role::Producer
             : Role::Consumer;
}

template <G g, O o>
struct Legal {
  // section 4.1 / section 5: work-item calls are implicitly strong, kernel
  // calls are relaxed only.
  static_assert(!(g == G::WorkItem && o == O::Relaxed),
                "work-item granularity supports only (implicit) strong ordering");
  static_assert(!(g == G::Kernel && o == O::Strong),
                "kernel granularity supports only relaxed ordering");
  static constexpr bool ok = true;
};

// A handle on an issued call.  n == 0: this lane holds no call.
struct Ticket {
  uint64_t t;         // ticket of this lane's (or the group's) request
  uint32_t head_off;  // t - first ticket of its claim group
  uint32_t n;         // size of the claim group
};

// ----------------------------------------------------------- memory helpers
// Address-space views.  Host staging, slots and registered buffers travel as
// integers or generic pointers, and accesses through those compile to flat
// instructions.  A flat access counts against the LDS counter as well as the
// memory counter, so every wait for an LDS result would also wait for each
// load still in flight over the host link, serialising a wavefront's
// prefetches.  gp() makes an access global, lp() makes it an LDS access.
template <class T>
using gptr_t = __attribute__((address_space(1))) T*;
template <class T>
using lptr_t = __attribute__((address_space(3))) T*;
template <class T>
__device__ __forceinline__ gptr_t<T> gp(uint64_t a) { return (gptr_t<T>)a; }
template <class T>
__device__ __forceinline__ gptr_t<T> gp(T* p) { return (gptr_t<T>)p; }
template <class T>
__device__ __forceinline__ lptr_t<T> lp(T* p) { return (lptr_t<T>)p; }
// 16-byte accesses use a plain vector type: uint4 is a class, and a class
// object cannot be copied through an address-space-qualified pointer.
typedef uint32_t u32x4 __attribute__((ext_vector_type(4)));
__device__ __forceinline__ u32x4 ldg16(uint64_t a) { return *gp<const u32x4>(a); }
__device__ __forceinline__ void stg16(uint64_t a, u32x4 v) { *gp<u32x4>(a) = v; }
__device__ __forceinline__ uint4 to_uint4(u32x4 v) { return make_uint4(v.x, v.y, v.z, v.w); }
__device__ __forceinline__ u32x4 to_u32x4(uint4 v) { return u32x4{v.x, v.y, v.z, v.w}; }

__device__ __forceinline__ uint64_t ld_sys(const uint64_t* p) {
  return __hip_atomic_load(gp(p), __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_SYSTEM);
}
__device__ __forceinline__ uint64_t ld_sys_acq(const uint64_t* p) {
  return __hip_atomic_load(gp(p), __ATOMIC_ACQUIRE, __HIP_MEMORY_SCOPE_SYSTEM);
}
__device__ __forceinline__ int64_t ld_sys_i64(const int64_t* p) {
  return __hip_atomic_load(gp(p), __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_SYSTEM);
}
__device__ __forceinline__ void st_sys(uint64_t* p, uint64_t v) {
  __hip_atomic_store(gp(p), v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_SYSTEM);
}
__device__ __forceinline__ void st_sys_rel(uint64_t* p, uint64_t v) {
  __hip_atomic_store(gp(p), v, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_SYSTEM);
}
__device__ __forceinline__ void fence_release_sys() { __builtin_amdgcn_fence(__ATOMIC_RELEASE, ""); }
__device__ __forceinline__ void fence_acquire_sys() { __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, ""); }

__device__ __forceinline__ uint32_t lane_id() {
  return __builtin_amdgcn_mbcnt_hi(~0u, __builtin_amdgcn_mbcnt_lo(~0u, 0u));
}
__device__ __forceinline__ uint64_t bcast64(uint64_t v, uint32_t src) {
  uint32_t lo = __builtin_amdgcn_readlane((uint32_t)v, src);
  uint32_t hi = __builtin_amdgcn_readlane((uint32_t)(v >> 32), src);
  return ((uint64_t)hi << 32) | lo;
}
__device__ __forceinline__ uint64_t active_mask() { return __ballot(1); }
__device__ __forceinline__ uint32_t first_lane(uint64_t m) { return (uint32_t)__ffsll((long long)m) - 1u; }

// Exponential backoff with s_sleep and a wall-clock watchdog
// (wall_clock64 runs at a constant 100 MHz on gfx9).
struct Waiter {
  uint64_t deadline;
  uint32_t n, cap;
  __device__ explicit Waiter(const gsys_dev_ctx& c)
      : deadline(c.timeout_ticks ? wall_clock64() + c.timeout_ticks : ~0ull),
        n(1), cap(c.sleep_max ? c.sleep_max : 16) {}
  // false once the watchdog expired
  __device__ bool pause() {
    for (uint32_t i = 0; i < n; ++i) __builtin_amdgcn_s_sleep(4);
    if (n < cap) n <<= 1;
    return wall_clock64() < deadline;
  }
};

// ---------------------------------------------------------------- doorbell
// With a doorbell (c.doorbell != 0) the host's idle pollers block on an HSA
// interrupt signal instead of spinning, and c.sleepers counts them.  The
// signal's handle is the address of its amd_signal_t.  Raising it takes
// three steps: store a value never stored before (the ticket + 1; the host's
// waits compare against the value they last saw), store the event id in the
// event's mailbox slot, and, once that store has completed, send an
// interrupt message; the driver finds the signalled mailbox slot and wakes
// the threads waiting on the event.  Only stores reach host memory: no
// read-modify-write crosses the host link.  The context checked at set-up
// that both the signal and the mailbox are mapped for this GPU.
__device__ __forceinline__ void raise_doorbell(uint64_t h, uint64_t t) {
  __hip_atomic_store(gp<int64_t>(h + offsetof(amd_signal_t, value)), (int64_t)(t + 1),
                     __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_SYSTEM);
  const uint64_t mb = *gp<const uint64_t>(h + offsetof(amd_signal_t, event_mailbox_ptr));
  if (mb) {
    const uint32_t id = *gp<const uint32_t>(h + offsetof(amd_signal_t, event_id));
    __hip_atomic_store(gp<uint64_t>(mb), (uint64_t)id, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_SYSTEM);
    fence_release_sys();  // the mailbox store has completed before the message
    __builtin_amdgcn_s_sendmsg(1 /* interrupt */, __builtin_amdgcn_readfirstlane(id));
  }
}

// After publishing ticket t (every lane that published calls this; `lead`
// is one of them).  The sequentially consistent fence orders this
// wavefront's READY stores before the sleeper load; a poller counts itself
// before its last look at the ring, so either it sees the request or the
// load here sees it counted.
__device__ __forceinline__ void ring_doorbell(const gsys_dev_ctx& c, uint64_t t, bool lead) {
  if (!c.doorbell) return;
  __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "");
  if (lead && ld_sys(c.sleepers) != 0) raise_doorbell(c.doorbell, t);
}

// ------------------------------------------------------------ ring protocol
// Wait until slot t mod D is free for ticket t.  A fresh ring holds
// FREE(t) for every t < D; later laps wait for the previous occupant to be
// freed (by the GPU waiter for blocking calls, by the host for non-blocking
// ones).  Each lane checks its own slot with one relaxed system-scope load,
// so a full ring back-pressures exactly the callers that would overwrite a
// live slot (section 5: if the slot is not free, the call is delayed).
__device__ __forceinline__ int wait_slot_free(const gsys_dev_ctx& c, uint64_t t) {
  if (t <= c.ring_mask) return 0;
  const uint64_t* ctl = &c.ring[t & c.ring_mask].ctl;
  const uint64_t want = GSYS_CTL(t, GSYS_ST_FREE);
  uint64_t v = ld_sys(ctl);
  if (v == want) return 0;
  Waiter w(c);
  for (;;) {
    if (!w.pause()) return GSYS_ETIMEDOUT_RET;
    v = ld_sys(ctl);
    if (v == want) return 0;
  }
}

// Fill slot t and hand it to the host (FREE -> POPULATING -> READY).
__device__ __forceinline__ void publish(const gsys_dev_ctx& c, uint64_t t, uint16_t nr,
                                        uint8_t flags, uint32_t grp_n, uint32_t grp_off,
                                        uint64_t a0, uint64_t a1, uint64_t a2, uint64_t a3,
                                        uint64_t a4, uint64_t a5) {
  gsys_slot* s = c.ring + (t & c.ring_mask);
  gptr_t<uint64_t> w = gp(reinterpret_cast<uint64_t*>(s));
  st_sys(&s->ctl, GSYS_CTL(t, GSYS_ST_POPULATING));
  const uint64_t hdr = (uint64_t)nr | ((uint64_t)flags << 16) | ((uint64_t)grp_n << 24) |
                       ((uint64_t)grp_off << 32);
  w[1] = hdr;
  w[2] = a0; w[3] = a1; w[4] = a2; w[5] = a3; w[6] = a4; w[7] = a5;
  st_sys_rel(&s->ctl, GSYS_CTL(t, GSYS_ST_READY));
}

// Poll the completion record of claim group `head` until `n` members are done.
// Returns 0, -ETIMEDOUT, or -EOVERFLOW if the record was reused by a later lap.
// Polls use relaxed system-scope loads (they bypass the caches and cost no
// cache maintenance); the caller issues one acquire fence after success.
__device__ __forceinline__ int poll_group(const gsys_dev_ctx& c, uint64_t head, uint32_t n) {
  const uint64_t* st = &c.comp[head & c.comp_mask].stamp;
  const uint64_t want = GSYS_STAMP(head, n);
  uint64_t v = ld_sys(st);
  if (v == want) return 0;
  Waiter w(c);
  for (;;) {
    if (v == want) return 0;
    if ((v >> 8) > head) return GSYS_EOVERFLOW_RET;
    if (!w.pause()) return GSYS_ETIMEDOUT_RET;
    v = ld_sys(st);
  }
}

__device__ __forceinline__ int64_t read_ret(const gsys_dev_ctx& c, uint64_t t) {
  return ld_sys_i64(&c.comp[t & c.comp_mask].ret);
}

// The result of a non-blocking call's ticket t, which may be collected long
// after the call.  Its slot was freed by the host, so later laps reuse the
// slot, and ticket t + C (C is a multiple of D: the same slot) writes the
// same completion record.  The slot's control word is read after the result
// (the agent-scope acquire waits for the result's load to return first): if
// it already names ticket t + C or a later one, the record may hold that
// ticket's result, and the wait reports -EOVERFLOW instead.  (A blocking
// call's record cannot be lapped: its slot is freed only after this read.)
__device__ __forceinline__ int64_t read_ret_late(const gsys_dev_ctx& c, uint64_t t) {
  const int64_t r = read_ret(c, t);
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");
  const uint64_t ctl = ld_sys(&c.ring[t & c.ring_mask].ctl);
  return GSYS_CTL_TICKET(ctl) > t + c.comp_mask ? (int64_t)GSYS_EOVERFLOW_RET : r;
}

// Blocking calls: the GPU frees the slot once it has the result (section 5).
// The result was read before (the workgroup-scope release waits for this
// wavefront's outstanding loads); nothing written here needs to reach the
// host before the FREE mark, so no system-scope write-back is needed.
__device__ __forceinline__ void free_slot(const gsys_dev_ctx& c, uint64_t t) {
  gsys_slot* s = c.ring + (t & c.ring_mask);
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "workgroup");
  st_sys(&s->ctl, GSYS_CTL(t + c.ring_mask + 1, GSYS_ST_FREE));
}

// Wave-level wait for the tickets held by the active lanes.  Lanes may hold
// tickets of different claim groups; one lane polls each distinct group.
// Returns this lane's result (or the wait's error code).
__device__ inline int64_t wave_wait(const gsys_dev_ctx& c, const Ticket& tk, bool free_after) {
  int64_t ret = GSYS_NOT_WAITED;
  bool pending = tk.n != 0;
  const uint64_t head = tk.t - tk.head_off;
  int err = 0;
  for (;;) {
    uint64_t m = __ballot(pending);
    if (!m) break;
    uint32_t src = first_lane(m);
    uint64_t h = bcast64(head, src);
    uint32_t n = __builtin_amdgcn_readlane(tk.n, src);
    int e = 0;
    if (lane_id() == src) e = poll_group(c, h, n);
    e = __builtin_amdgcn_readlane(e, src);
    if (pending && head == h) {
      pending = false;
      err = e;
    }
  }
  if (tk.n != 0) {
    fence_acquire_sys();
    if (err == 0) {
      // free_after: a blocking call's wait (it frees the slot itself)
      ret = free_after ? read_ret(c, tk.t) : read_ret_late(c, tk.t);
      if (free_after) free_slot(c, tk.t);
    } else {
      ret = err;
    }
  }
  return ret;
}

// ------------------------------------------------------------- public calls
struct Args6 {
  uint64_t a[6];
};

// Work-item granularity: every active lane issues its own call.  Implicitly
// strong: its prior writes are released at system scope before the call and
// results are acquired after it.
template <B b>
__device__ inline int64_t call_wi(const gsys_dev_ctx& c, uint16_t nr, const Args6& a,
                                  Ticket* out = nullptr) {
  (void)Legal<G::WorkItem, O::Strong>::ok;
  const uint64_t m = active_mask();
  const uint32_t n = (uint32_t)__popcll(m);
  const uint32_t rank = __builtin_amdgcn_mbcnt_hi((uint32_t)(m >> 32),
                                                  __builtin_amdgcn_mbcnt_lo((uint32_t)m, 0u));
  const uint32_t leader = first_lane(m);
  uint64_t base = 0;
  if (lane_id() == leader)
    base = __hip_atomic_fetch_add(gp(c.tail), (unsigned long long)n, __ATOMIC_RELAXED,
                                  __HIP_MEMORY_SCOPE_AGENT);
  base = bcast64(base, leader);
  Ticket tk{base + rank, rank, n};
  const int err = wait_slot_free(c, tk.t);
  if (__ballot(err != 0)) {
    // A slot stayed busy until the watchdog fired.  Nothing is published:
    // the tickets stay claimed, so a drain of this context reports the loss.
    if (out) *out = Ticket{0, 0, 0};
    return GSYS_ETIMEDOUT_RET;
  }
  const uint8_t fl = (uint8_t)((b == B::Blocking ? GSYS_F_BLOCKING : 0u) | GSYS_F_STRONG |
                               (role_of(nr) == Role::Producer ? GSYS_F_PRODUCER : 0u) |
                               (GSYS_GRAN_WI << GSYS_F_GRAN_SHIFT));
  // implicit strong ordering: the READY store is a system-scope release, so
  // every write this wavefront made before the call is visible to the host
  // before the request is
  publish(c, tk.t, nr, fl, n, rank, a.a[0], a.a[1], a.a[2], a.a[3], a.a[4], a.a[5]);
  ring_doorbell(c, tk.t, lane_id() == leader);
  if (out) *out = tk;
  if constexpr (b == B::Blocking) {
    return wave_wait(c, tk, true);
  } else {
    return 0;
  }
}

// Wait for a non-blocking work-item call (all active lanes call this).
__device__ inline int64_t wait_wi(const gsys_dev_ctx& c, const Ticket& tk) {
  return wave_wait(c, tk, false);
}

// Work-group granularity.  Every work-item of the group must call this (it
// contains work-group barriers when the ordering needs them); local thread 0
// is the designated caller and its arguments are the call's arguments
// (section 5).  Returns the call's result to every lane that waited for it:
// all lanes when a barrier follows the call, only the caller's wavefront for
// a blocking relaxed producer, nobody for non-blocking calls (GSYS_NOT_WAITED;
// the ticket goes to *out on thread 0).
template <O o, B b>
__device__ inline int64_t call_wg(const gsys_dev_ctx& c, uint16_t nr, uint8_t extra_flags,
                                  const Args6& a, Ticket* out = nullptr) {
  (void)Legal<G::WorkGroup, o>::ok;
  __shared__ int64_t s_ret;
  const bool producer = role_of(nr) == Role::Producer;
  const bool barrier_before = (o == O::Strong) || producer;
  const bool barrier_after = (o == O::Strong) || !producer;
  if (barrier_before) {
    fence_release_sys();  // every wavefront makes its writes visible to the host
    __syncthreads();
  }
  if (!barrier_before && threadIdx.x < 64) {
    // a relaxed consumer call has no group barrier before it, so only the
    // caller's wavefront may have written memory the call reads (a
    // descriptor list, say): each of its work-items releases its writes at
    // system scope before work-item 0 publishes
    fence_release_sys();
    __builtin_amdgcn_wave_barrier();
  }
  Ticket tk{0, 0, 0};
  int64_t ret = GSYS_NOT_WAITED;
  if (threadIdx.x == 0) {
    uint64_t t = __hip_atomic_fetch_add(gp(c.tail), 1ull, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    int err = wait_slot_free(c, t);
    if (err) {
      ret = err;
    } else {
      const uint8_t fl = (uint8_t)((b == B::Blocking ? GSYS_F_BLOCKING : 0u) |
                                   (o == O::Strong ? GSYS_F_STRONG : 0u) |
                                   (producer ? GSYS_F_PRODUCER : 0u) | extra_flags |
                                   (GSYS_GRAN_WG << GSYS_F_GRAN_SHIFT));
      publish(c, t, nr, fl, 1, 0, a.a[0], a.a[1], a.a[2], a.a[3], a.a[4], a.a[5]);
      ring_doorbell(c, t, true);
      tk = Ticket{t, 0, 1};
      if constexpr (b == B::Blocking) {
        int e = poll_group(c, t, 1);
        fence_acquire_sys();
        if (e == 0) {
          ret = read_ret(c, t);
          free_slot(c, t);
        } else {
          ret = e;
        }
      } else {
        ret = 0;
      }
    }
    if (out) *out = tk;
  }
  if (barrier_after) {
    if (threadIdx.x == 0) s_ret = ret;
    __syncthreads();
    ret = s_ret;
    fence_acquire_sys();
    // thread 0 may write s_ret again in the next call before any barrier of
    // that call: every work-item takes its copy first
    __syncthreads();
    if constexpr (b == B::NonBlocking) ret = GSYS_NOT_WAITED;
  } else if constexpr (b == B::Blocking) {
    // weak-block: only the caller's wavefront waits (section 6).
    if (threadIdx.x < 64) ret = bcast64((uint64_t)ret, 0);
  }
  return ret;
}

// Wait for a non-blocking work-group call: thread 0 polls, then the group
// synchronises.  Every work-item of the group calls this.
__device__ inline int64_t wait_wg(const gsys_dev_ctx& c, const Ticket& tk_thread0) {
  __shared__ int64_t s_ret;
  if (threadIdx.x == 0) {
    int64_t r = GSYS_NOT_WAITED;
    if (tk_thread0.n) {
      int e = poll_group(c, tk_thread0.t, 1);
      fence_acquire_sys();
      r = e ? (int64_t)e : read_ret_late(c, tk_thread0.t);
    }
    s_ret = r;
  }
  __syncthreads();
  fence_acquire_sys();
  const int64_t r = s_ret;
  __syncthreads();  // s_ret is rewritten by the next wait before any barrier
  return r;
}

// Per-launch state of one kernel-granularity call site; zero it before each
// launch.
struct KState {
  unsigned int elect;        // consumer calls: the first arriver takes it
  unsigned int arrived;      // producer calls: arrivals; the last arriver calls
  unsigned long long ticket; // ticket + 1 once published, KS_FAILED on failure
};
constexpr unsigned long long KS_FAILED = ~0ull;

// Kernel granularity, relaxed only.  Every work-item of every work-group calls
// this.  Consumer calls: the first work-group to arrive is the caller, and
// every work-group waits for the result before going on (the barrier after).
// Producer calls: every work-group releases its writes and arrives; the last
// one to arrive is the caller, and nobody else waits (the barrier before).
// The caller's arguments come from `make_args`, evaluated by local thread 0
// of the caller work-group after `prepare` ran on all of its work-items
// (e.g. to build a descriptor list).  Non-blocking: returns 0 (GSYS_NOT_WAITED
// outside the caller for producers) and the ticket through *out.
template <B b, class Prepare, class MakeArgs>
__device__ inline int64_t call_kernel(const gsys_dev_ctx& c, KState* ks, uint16_t nr,
                                      uint8_t extra_flags, Prepare prepare, MakeArgs make_args,
                                      Ticket* out = nullptr) {
  (void)Legal<G::Kernel, O::Relaxed>::ok;
  __shared__ int s_caller;
  __shared__ int64_t s_ret;
  __shared__ unsigned long long s_t1;  // ticket + 1, 0 = none
  const bool producer = role_of(nr) == Role::Producer;
  const unsigned int nwg = gridDim.x * gridDim.y * gridDim.z;
  if (producer) fence_release_sys();
  __syncthreads();
  if (threadIdx.x == 0) {
    int caller;
    if (producer) {
      caller = __hip_atomic_fetch_add(gp(&ks->arrived), 1u, __ATOMIC_ACQ_REL,
                                      __HIP_MEMORY_SCOPE_AGENT) == nwg - 1;
    } else {
      unsigned int exp = 0;
      caller = __hip_atomic_compare_exchange_strong(gp(&ks->elect), &exp, 1u, __ATOMIC_ACQ_REL,
                                                    __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    }
    s_caller = caller;
    s_t1 = 0;
    s_ret = GSYS_NOT_WAITED;
  }
  __syncthreads();
  const bool caller = s_caller != 0;
  if (caller) {
    prepare();
    fence_release_sys();
    __syncthreads();
    if (threadIdx.x == 0) {
      Args6 a = make_args();
      uint64_t t = __hip_atomic_fetch_add(gp(c.tail), 1ull, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
      int err = wait_slot_free(c, t);
      if (err) {
        s_ret = err;
      } else {
        const uint8_t fl = (uint8_t)((b == B::Blocking ? GSYS_F_BLOCKING : 0u) |
                                     (producer ? GSYS_F_PRODUCER : 0u) | extra_flags |
                                     (GSYS_GRAN_KERNEL << GSYS_F_GRAN_SHIFT));
        publish(c, t, nr, fl, 1, 0, a.a[0], a.a[1], a.a[2], a.a[3], a.a[4], a.a[5]);
        ring_doorbell(c, t, true);
        s_t1 = t + 1;
        s_ret = 0;
      }
      if (!producer)
        __hip_atomic_store(gp(&ks->ticket), s_t1 ? s_t1 : KS_FAILED, __ATOMIC_RELEASE,
                           __HIP_MEMORY_SCOPE_AGENT);
    }
    __syncthreads();
  } else if (!producer) {
    // learn the caller's ticket; the caller is resident because it arrived first
    if (threadIdx.x == 0) {
      Waiter w(c);
      unsigned long long v;
      for (;;) {
        v = __hip_atomic_load(gp(&ks->ticket), __ATOMIC_ACQUIRE, __HIP_MEMORY_SCOPE_AGENT);
        if (v) break;
        if (!w.pause()) { v = KS_FAILED; break; }
      }
      if (v == KS_FAILED) {
        s_ret = GSYS_ETIMEDOUT_RET;
      } else {
        s_t1 = v;
        s_ret = 0;
      }
    }
    __syncthreads();
  }
  const unsigned long long t1 = s_t1;
  if (out) *out = t1 ? Ticket{t1 - 1, 0, 1} : Ticket{0, 0, 0};
  if constexpr (b == B::NonBlocking) {
    return s_ret;
  } else {
    if (producer) {
      // weak-block: only the caller's wavefront waits
      int64_t ret = GSYS_NOT_WAITED;
      if (caller && threadIdx.x < 64) {
        ret = s_ret;
        if (t1) {
          int e = 0;
          if (threadIdx.x == 0) e = poll_group(c, t1 - 1, 1);
          e = __builtin_amdgcn_readlane(e, 0);
          fence_acquire_sys();
          ret = e ? (int64_t)e : read_ret(c, t1 - 1);
          if (e == 0 && threadIdx.x == 0) free_slot(c, t1 - 1);
        }
      }
      return ret;
    }
    // consumer: every work-group waits for the result
    __syncthreads();
    if (threadIdx.x == 0 && t1) {
      int e = poll_group(c, t1 - 1, 1);
      fence_acquire_sys();
      // the caller frees the slot after its own read; a work-group that
      // reads after that takes the lap-checked read
      int64_t r = e ? (int64_t)e : caller ? read_ret(c, t1 - 1) : read_ret_late(c, t1 - 1);
      if (caller && e == 0) free_slot(c, t1 - 1);
      s_ret = r;
    }
    __syncthreads();
    fence_acquire_sys();
    return s_ret;
  }
}

// Wait for a non-blocking kernel call from every work-group (consumer side).
__device__ inline int64_t wait_kernel(const gsys_dev_ctx& c, const Ticket& tk) {
  __shared__ int64_t s_ret;
  if (threadIdx.x == 0) {
    int64_t r = GSYS_NOT_WAITED;
    if (tk.n) {
      int e = poll_group(c, tk.t, 1);
      fence_acquire_sys();
      r = e ? (int64_t)e : read_ret_late(c, tk.t);
    }
    s_ret = r;
  }
  __syncthreads();
  fence_acquire_sys();
  const int64_t r = s_ret;
  __syncthreads();  // s_ret is rewritten by the next wait before any barrier
  return r;
}

// ============================================================= public API
// What a user kernel calls.  Every call names its granularity G, ordering O
// and blocking B (section 4.1); work-item calls are strong only and kernel
// calls relaxed only, both checked at compile time.  Under relaxed ordering
// the call's role decides which side of it synchronises the group: write,
// pwrite, sendto, munmap, madvise and close are producers (the group's
// writes are released before the call), read, pread, recvfrom, mmap and
// openat consumers (the group waits for the result after it).
//
//  G::WorkItem   every active work-item makes its own call with its own
//                arguments; the calls of a wavefront share one claim on the
//                ring (section 5 gives each work-item its own slot).
//  G::WorkGroup  every work-item of the work-group makes the call together;
//                work-item 0 is the designated caller and its arguments are
//                the call's (section 5).  Under relaxed consumer ordering
//                only work-item 0's wavefront may write memory the call reads.
//  G::Kernel     every work-item of the launch makes the call together; the
//                designated caller is the first work-group to arrive
//                (consumer) or the last (producer), and its work-item 0's
//                arguments are the call's.  Each such call needs its own
//                call site: gsys_call uses site 0 of the context's
//                kernel-call sites, gsys_call_site any of them; gsys_launch
//                clears them all before every launch.
//
// Blocking calls return the call's result (>= 0) or -errno to every
// work-item that waits for it: all of them for work-item calls and for
// group calls with a barrier after them; only the caller's wavefront for a
// relaxed blocking producer (the paper's weak-block: only the caller waits).
// Non-blocking calls return at once (0, or GSYS_NOT_WAITED where the caller
// did not issue) and hand back a Ticket through `tk` (work-item 0 of the
// caller work-group for group calls; each work-item for work-item calls);
// gsys_wait<G> then returns the result, from the same launch or a later one.
// The result is kept until C newer tickets have been claimed (C = the
// completion records, max(4 x ring slots, 65536)); a wait after that
// returns -EOVERFLOW.  A non-blocking call whose ticket is never waited for
// is still serviced; the host's gsys_wait drains it.

// The kernel-call sites a launch may use (see gsys_launch).
__device__ __forceinline__ KState* kernel_site(const gsys_dev_ctx& c, uint32_t site) {
  return reinterpret_cast<KState*>(c.ksites) + (site < c.n_ksites ? site : 0);
}

template <G g, O o, B b>
__device__ inline int64_t gsys_call(const gsys_dev_ctx& c, uint16_t nr, const Args6& a,
                                    Ticket* tk = nullptr) {
  (void)Legal<g, o>::ok;
  if constexpr (g == G::WorkItem) {
    return call_wi<b>(c, nr, a, tk);
  } else if constexpr (g == G::WorkGroup) {
    return call_wg<o, b>(c, nr, 0, a, tk);
  } else {
    return call_kernel<b>(c, kernel_site(c, 0), nr, 0, [] {}, [&] { return a; }, tk);
  }
}

template <G g, O o, B b>
__device__ inline int64_t gsys_call(const gsys_dev_ctx& c, uint16_t nr, uint64_t a0,
                                    uint64_t a1 = 0, uint64_t a2 = 0, uint64_t a3 = 0,
                                    uint64_t a4 = 0, uint64_t a5 = 0) {
  return gsys_call<g, o, b>(c, nr, Args6{{a0, a1, a2, a3, a4, a5}});
}

// A kernel-granularity call at call site `site`; every work-item of the
// launch passes the same site.  A site at or past the context's n_ksites
// makes no call and returns -EINVAL (sites are never shared by accident).
template <O o, B b>
__device__ inline int64_t gsys_call_site(const gsys_dev_ctx& c, uint32_t site, uint16_t nr,
                                         const Args6& a, Ticket* tk = nullptr) {
  (void)Legal<G::Kernel, o>::ok;
  if (site >= c.n_ksites) return GSYS_EINVAL_RET;
  return call_kernel<b>(c, kernel_site(c, site), nr, 0, [] {}, [&] { return a; }, tk);
}

// The result of a non-blocking call, by the same work-items that made it.
template <G g>
__device__ inline int64_t gsys_wait(const gsys_dev_ctx& c, const Ticket& tk) {
  if constexpr (g == G::WorkItem) return wait_wi(c, tk);
  else if constexpr (g == G::WorkGroup) return wait_wg(c, tk);
  else return wait_kernel(c, tk);
}

// Typed wrappers: the call number fixes the role; arguments are the
// system call's own (addresses are device views of registered buffers).
#define GSYS_DEFAULT_ORDER (g == G::Kernel ? O::Relaxed : O::Strong)
template <G g, O o = GSYS_DEFAULT_ORDER, B b = B::Blocking>
__device__ inline int64_t read(const gsys_dev_ctx& c, int fd, uint64_t buf, uint64_t count,
                               Ticket* tk = nullptr) {
  return gsys_call<g, o, b>(c, GSYS_NR_READ, Args6{{(uint64_t)(int64_t)fd, buf, count, 0, 0, 0}}, tk);
}
template <G g, O o = GSYS_DEFAULT_ORDER, B b = B::Blocking>
__device__ inline int64_t write(const gsys_dev_ctx& c, int fd, uint64_t buf, uint64_t count,
                                Ticket* tk = nullptr) {
  return gsys_call<g, o, b>(c, GSYS_NR_WRITE, Args6{{(uint64_t)(int64_t)fd, buf, count, 0, 0, 0}}, tk);
}
template <G g, O o = GSYS_DEFAULT_ORDER, B b = B::Blocking>
__device__ inline int64_t pread(const gsys_dev_ctx& c, int fd, uint64_t buf, uint64_t count,
                                uint64_t off, Ticket* tk = nullptr) {
  return gsys_call<g, o, b>(c, GSYS_NR_PREAD64, Args6{{(uint64_t)(int64_t)fd, buf, count, off, 0, 0}}, tk);
}
template <G g, O o = GSYS_DEFAULT_ORDER, B b = B::Blocking>
__device__ inline int64_t pwrite(const gsys_dev_ctx& c, int fd, uint64_t buf, uint64_t count,
                                 uint64_t off, Ticket* tk = nullptr) {
  return gsys_call<g, o, b>(c, GSYS_NR_PWRITE64, Args6{{(uint64_t)(int64_t)fd, buf, count, off, 0, 0}}, tk);
}
// addr: a struct sockaddr_in of addr_len bytes in a registered buffer
template <G g, O o = GSYS_DEFAULT_ORDER, B b = B::Blocking>
__device__ inline int64_t sendto(const gsys_dev_ctx& c, int fd, uint64_t buf, uint64_t len,
                                 int flags, uint64_t addr, uint64_t addr_len, Ticket* tk = nullptr) {
  return gsys_call<g, o, b>(c, GSYS_NR_SENDTO, Args6{{(uint64_t)(int64_t)fd, buf, len, (uint64_t)(int64_t)flags, addr, addr_len}}, tk);
}
// src_addr: 0, or room for a struct sockaddr_in in a registered buffer
template <G g, O o = GSYS_DEFAULT_ORDER, B b = B::Blocking>
__device__ inline int64_t recvfrom(const gsys_dev_ctx& c, int fd, uint64_t buf, uint64_t len,
                                   int flags, uint64_t src_addr, Ticket* tk = nullptr) {
  return gsys_call<g, o, b>(c, GSYS_NR_RECVFROM, Args6{{(uint64_t)(int64_t)fd, buf, len, (uint64_t)(int64_t)flags, src_addr, 0}}, tk);
}
template <G g, O o = GSYS_DEFAULT_ORDER, B b = B::Blocking>
__device__ inline int64_t mmap(const gsys_dev_ctx& c, uint64_t addr, uint64_t len, int prot,
                               int flags, int fd, uint64_t off, Ticket* tk = nullptr) {
  return gsys_call<g, o, b>(c, GSYS_NR_MMAP, Args6{{addr, len, (uint64_t)(int64_t)prot, (uint64_t)(int64_t)flags, (uint64_t)(int64_t)fd, off}}, tk);
}
template <G g, O o = GSYS_DEFAULT_ORDER, B b = B::Blocking>
__device__ inline int64_t munmap(const gsys_dev_ctx& c, uint64_t addr, uint64_t len,
                                 Ticket* tk = nullptr) {
  return gsys_call<g, o, b>(c, GSYS_NR_MUNMAP, Args6{{addr, len, 0, 0, 0, 0}}, tk);
}
template <G g, O o = GSYS_DEFAULT_ORDER, B b = B::Blocking>
__device__ inline int64_t madvise(const gsys_dev_ctx& c, uint64_t addr, uint64_t len, int advice,
                                  Ticket* tk = nullptr) {
  return gsys_call<g, o, b>(c, GSYS_NR_MADVISE, Args6{{addr, len, (uint64_t)(int64_t)advice, 0, 0, 0}}, tk);
}
// path: GSYS_PATH_MAX bytes (NUL-terminated) in a registered buffer
template <G g, O o = GSYS_DEFAULT_ORDER, B b = B::Blocking>
__device__ inline int64_t openat(const gsys_dev_ctx& c, int dirfd, uint64_t path, int flags,
                                 uint32_t mode, Ticket* tk = nullptr) {
  return gsys_call<g, o, b>(c, GSYS_NR_OPENAT, Args6{{(uint64_t)(int64_t)dirfd, path, (uint64_t)(int64_t)flags, mode, 0, 0}}, tk);
}
template <G g, O o = GSYS_DEFAULT_ORDER, B b = B::Blocking>
__device__ inline int64_t close(const gsys_dev_ctx& c, int fd, Ticket* tk = nullptr) {
  return gsys_call<g, o, b>(c, GSYS_NR_CLOSE, Args6{{(uint64_t)(int64_t)fd, 0, 0, 0, 0, 0}}, tk);
}
#undef GSYS_DEFAULT_ORDER

}  // namespace gsys
