// Test hooks of the gsys library, in a library of their own that only tests
// load (libgsys_testing.so, linked against libgsys.so).  They let CPU-only
// tests drive the host service pool through exactly the protocol the GPU
// uses, from host threads, and inject faults.  The context is reached through
// internal accessors of libgsys.so (gsys_internal::pool, doorbell,
// ring_host, no_device).
#include <errno.h>
#include <stdint.h>
#include <string.h>
#include <time.h>

#include <algorithm>
#include <thread>
#include <vector>

#include "gsys.h"
#include "gsys_testing.h"
#include "host_pool.hpp"
#include "testing_access.hpp"

namespace {

uint64_t now_ns() {
  timespec ts;
  clock_gettime(CLOCK_MONOTONIC, &ts);
  return (uint64_t)ts.tv_sec * 1000000000ull + (uint64_t)ts.tv_nsec;
}

}  // namespace

namespace {

struct EmuShared {
  gsys_dev_ctx d;
  uint64_t timeout_ns;
  gsys_host::Doorbell* db;
};

// after publishing, as the GPU does: fence, read the sleeper count, ring
void emu_ring(const EmuShared& e) {
  if (!e.db) return;
  __atomic_thread_fence(__ATOMIC_SEQ_CST);
  if (__atomic_load_n(e.d.sleepers, __ATOMIC_RELAXED)) e.db->ring();
}

// claim n tickets, then wait until each of their slots is free for this lap
uint64_t emu_claim(const EmuShared& e, uint32_t n, int* err) {
  uint64_t t = __atomic_fetch_add((uint64_t*)e.d.tail, (uint64_t)n, __ATOMIC_RELAXED);
  const uint64_t t0 = now_ns();
  for (uint32_t i = 0; i < n && !*err; ++i) {
    const uint64_t* ctl = &e.d.ring[(t + i) & e.d.ring_mask].ctl;
    while (__atomic_load_n(ctl, __ATOMIC_ACQUIRE) != GSYS_CTL(t + i, GSYS_ST_FREE)) {
      if (now_ns() - t0 > e.timeout_ns) {
        *err = -ETIMEDOUT;
        break;
      }
      std::this_thread::yield();
    }
  }
  return t;
}

void emu_publish(const EmuShared& e, uint64_t t, uint16_t nr, uint8_t flags, uint32_t n,
                 uint32_t off, const uint64_t* a) {
  gsys_slot* s = e.d.ring + (t & e.d.ring_mask);
  __atomic_store_n(&s->ctl, GSYS_CTL(t, GSYS_ST_POPULATING), __ATOMIC_RELAXED);
  s->nr = nr;
  s->flags = flags;
  s->grp_n = (uint8_t)n;
  s->grp_off = off;
  for (int i = 0; i < 6; ++i) s->args[i] = a[i];
  __atomic_store_n(&s->ctl, GSYS_CTL(t, GSYS_ST_READY), __ATOMIC_RELEASE);
}

int emu_wait(const EmuShared& e, uint64_t head, uint32_t n) {
  const uint64_t want = GSYS_STAMP(head, n);
  const uint64_t* st = &e.d.comp[head & e.d.comp_mask].stamp;
  const uint64_t t0 = now_ns();
  for (;;) {
    uint64_t v = __atomic_load_n(st, __ATOMIC_ACQUIRE);
    if (v == want) return 0;
    if ((v >> 8) > head) return -EOVERFLOW;
    if (now_ns() - t0 > e.timeout_ns) return -ETIMEDOUT;
    std::this_thread::yield();
  }
}

}  // namespace

extern "C" {

int gsys_test_emulate(gsys_ctx* c, uint32_t threads, uint64_t per, uint32_t group, uint32_t mode,
                      int fd, uint64_t buf_dev, uint64_t list_dev, uint32_t len, const uint64_t* offs,
                      int64_t* rets, uint64_t timeout_ns) {
  if (!c || !gsys_internal::no_device(c) || !threads || !group || group > 64 || !offs || !rets) return -EINVAL;
  EmuShared e;
  gsys_device_ctx(c, &e.d);
  e.timeout_ns = timeout_ns ? timeout_ns : 10000000000ull;
  e.db = gsys_internal::doorbell(c);
  const bool blocking = mode & GSYS_EMU_BLOCKING;
  const bool list = mode & GSYS_EMU_LIST;
  std::vector<int> errs(threads, 0);
  std::vector<std::thread> th;
  for (uint32_t w = 0; w < threads; ++w) {
    th.emplace_back([&, w] {
      uint64_t k = (uint64_t)w * per;
      const uint64_t end = k + per;
      while (k < end && !errs[w]) {
        const uint32_t n = (uint32_t)std::min<uint64_t>(group, end - k);
        int err = 0;
        if (list) {
          gsys_iodesc* L = (gsys_iodesc*)(list_dev + 16 * k);
          for (uint32_t i = 0; i < n; ++i)
            L[i] = gsys_iodesc{offs[k + i], (uint32_t)(i * len), (int32_t)len};
          uint64_t t = emu_claim(e, 1, &err);
          if (err) { errs[w] = err; break; }
          uint64_t a[6] = {(uint64_t)(int64_t)fd, (uint64_t)L, n, buf_dev + k * len, 0, 0};
          emu_publish(e, t, GSYS_NR_PREAD64,
                      (uint8_t)(GSYS_F_LIST | (blocking ? GSYS_F_BLOCKING : 0) |
                                (GSYS_GRAN_WG << GSYS_F_GRAN_SHIFT)),
                      1, 0, a);
          emu_ring(e);
          err = emu_wait(e, t, 1);
          if (err) { errs[w] = err; break; }
          for (uint32_t i = 0; i < n; ++i) rets[k + i] = __atomic_load_n(&L[i].len_ret, __ATOMIC_ACQUIRE);
          if (blocking)
            __atomic_store_n(&e.d.ring[t & e.d.ring_mask].ctl,
                             GSYS_CTL(t + e.d.ring_mask + 1, GSYS_ST_FREE), __ATOMIC_RELEASE);
        } else {
          uint64_t t = emu_claim(e, n, &err);
          if (err) { errs[w] = err; break; }
          for (uint32_t i = 0; i < n; ++i) {
            uint64_t a[6] = {(uint64_t)(int64_t)fd, buf_dev + (k + i) * len, len, offs[k + i], 0, 0};
            emu_publish(e, t + i, GSYS_NR_PREAD64,
                        (uint8_t)((blocking ? GSYS_F_BLOCKING : 0) | GSYS_F_STRONG), n, i, a);
          }
          emu_ring(e);
          err = emu_wait(e, t, n);
          if (err) { errs[w] = err; break; }
          for (uint32_t i = 0; i < n; ++i) {
            rets[k + i] = __atomic_load_n(&e.d.comp[(t + i) & e.d.comp_mask].ret, __ATOMIC_ACQUIRE);
            if (blocking)
              __atomic_store_n(&e.d.ring[(t + i) & e.d.ring_mask].ctl,
                               GSYS_CTL(t + i + e.d.ring_mask + 1, GSYS_ST_FREE), __ATOMIC_RELEASE);
          }
        }
        k += n;
      }
    });
  }
  for (auto& t : th) t.join();
  for (int x : errs)
    if (x) return x;
  return 0;
}

int gsys_test_raw_call(gsys_ctx* c, uint16_t nr, uint8_t flags, const uint64_t* args6, int64_t* ret,
                       uint64_t timeout_ns) {
  if (!c || !gsys_internal::no_device(c) || !args6 || !ret) return -EINVAL;
  EmuShared e;
  gsys_device_ctx(c, &e.d);
  e.timeout_ns = timeout_ns ? timeout_ns : 10000000000ull;
  e.db = gsys_internal::doorbell(c);
  int err = 0;
  uint64_t t = emu_claim(e, 1, &err);
  if (err) return err;
  emu_publish(e, t, nr, flags, 1, 0, args6);
  emu_ring(e);
  err = emu_wait(e, t, 1);
  if (err) return err;
  *ret = __atomic_load_n(&e.d.comp[t & e.d.comp_mask].ret, __ATOMIC_ACQUIRE);
  if (flags & GSYS_F_BLOCKING)
    __atomic_store_n(&e.d.ring[t & e.d.ring_mask].ctl, GSYS_CTL(t + e.d.ring_mask + 1, GSYS_ST_FREE),
                     __ATOMIC_RELEASE);
  return 0;
}

int64_t gsys_test_claim_only(gsys_ctx* c, uint32_t n) {
  if (!c || !gsys_internal::no_device(c)) return -EINVAL;
  gsys_dev_ctx d;
  gsys_device_ctx(c, &d);  // a CPU-only context's ticket counter is host memory
  return (int64_t)__atomic_fetch_add((uint64_t*)d.tail, (uint64_t)n, __ATOMIC_ACQ_REL);
}

int gsys_test_unregister_now(gsys_ctx* c, uint32_t id) {
  if (!c) return -EINVAL;
  return gsys_internal::pool(c)->remove_buffer(id);
}

int gsys_test_inject(gsys_ctx* c, uint16_t nr, int32_t err, uint32_t count) {
  if (!c || err <= 0 || err > 4095) return -EINVAL;
  gsys_internal::pool(c)->inject(nr, err, count);
  return 0;
}

int gsys_test_ring_ctl(gsys_ctx* c, uint64_t* out, uint64_t max) {
  if (!c || !out) return -EINVAL;
  uint64_t D = 0;
  const gsys_slot* ring = gsys_internal::ring_host(c, &D);
  const uint64_t n = std::min<uint64_t>(max, D);
  for (uint64_t i = 0; i < n; ++i) out[i] = __atomic_load_n(&ring[i].ctl, __ATOMIC_ACQUIRE);
  return (int)n;
}

}  // extern "C"
