// The host service pool under ThreadSanitizer.  Host threads drive the pool
// through the GPU's slot protocol (gsys_test_emulate: wave-coalesced claims,
// group completions, descriptor-list calls, blocking and non-blocking),
// with and without coalescing, while two more threads keep changing the fd
// table and the registered-buffer table that the pollers read without
// locks, and a third makes calls into an unregistered range (whose
// validation scans the whole buffer table).  A last phase turns the
// doorbell on: pollers that find nothing for 20 us block, and a sparse
// caller keeps arriving around their decision to block (the backstop is
// raised to 30 s, so a lost wake-up shows as a time-out).  Every result is
// checked against the file's bytes.  A final phase unregisters and frees
// descriptor-list buffers while list calls run over them: the pool reads and
// writes those lists from user space, so AddressSanitizer reports any use
// after the free if a service thread could still hold the list when
// unregistering returned.  Exits 0 when all checks pass; ThreadSanitizer
// turns any data race into a non-zero exit.
//
// Build: g++ -fsanitize=thread over this file, native/gsys_test_hooks.cpp,
// capi.cpp and host_pool.cpp (host code only; contexts use
// GSYS_CFG_NO_DEVICE and make no HIP calls).
#include <errno.h>
#include <fcntl.h>
#include <stdint.h>
#include <stdio.h>
#include <stdlib.h>
#include <string.h>
#include <unistd.h>

#include <atomic>
#include <string>
#include <thread>
#include <vector>

#include "gsys.h"
#include "gsys_testing.h"

namespace {

constexpr uint64_t kFile = 4u << 20;
constexpr uint32_t kItem = 4096;

uint8_t pattern(uint64_t i) { return (uint8_t)((i * 2654435761u) >> 13); }

int fail(const char* what, long a = 0, long b = 0) {
  fprintf(stderr, "FAIL %s (%ld, %ld)\n", what, a, b);
  return 1;
}

struct Phase {
  const char* name;
  uint32_t threads, group, mode, K, T;
  bool sequential;  // consecutive offsets, so coalesced bundles merge
  bool doorbell;
};

int run_phase(const std::string& path, const Phase& ph) {
  gsys_config cfg;
  memset(&cfg, 0, sizeof cfg);
  cfg.abi_version = GSYS_ABI_VERSION;
  cfg.ring_slots = 4096;  // completion records (4D) outlast slow waiters under a sanitizer
  cfg.service_threads = 4;
  cfg.coalesce_max = ph.K;
  cfg.coalesce_window_ns = ph.T;
  cfg.flags = GSYS_CFG_NO_DEVICE | GSYS_CFG_NO_PIN | GSYS_CFG_LEDGER |
              (ph.doorbell ? GSYS_CFG_DOORBELL : 0u);
  cfg.doorbell_idle_us = 20;
  gsys_ctx* ctx = nullptr;
  if (int e = gsys_init(&cfg, &ctx)) return fail("gsys_init", e);
  const int fd = open(path.c_str(), O_RDONLY);
  const int fd2 = open(path.c_str(), O_RDONLY);
  if (fd < 0 || fd2 < 0) return fail("open");
  if (gsys_allow_fd(ctx, fd, GSYS_FD_READ)) return fail("allow_fd");
  // registered first, so that dropping it moves the last live entry into
  // its slot: the pollers' lock-free lookups see entries move under them
  const uint64_t churn_base = 1ull << 46;  // a device range no call uses
  std::vector<uint8_t> dummy(1 << 16);
  uint32_t churn_id = 0;
  if (gsys_register_buffer(ctx, churn_base, dummy.data(), dummy.size(), GSYS_BUF_HOST, &churn_id))
    return fail("register");
  const uint64_t n = (uint64_t)ph.threads * 256;
  void* host = nullptr;
  uint64_t dev = 0;
  uint32_t id = 0;
  void* lhost = nullptr;
  uint64_t ldev = 0;
  uint32_t lid = 0;
  if (gsys_host_alloc(ctx, n * kItem, &host, &dev, &id)) return fail("host_alloc");
  if (gsys_host_alloc(ctx, n * 16, &lhost, &ldev, &lid)) return fail("host_alloc lists");
  std::vector<uint64_t> offs(n);
  for (uint64_t k = 0; k < n; ++k)
    offs[k] = ph.sequential ? (k * kItem) % kFile : ((k * 7919u) % (kFile / kItem)) * kItem;
  std::vector<int64_t> rets(n, -12345);

  // the tables the pollers read without locks change all the time
  std::atomic<bool> done{false};
  std::thread fd_churn([&] {
    for (uint32_t i = 0; !done.load(); ++i) gsys_allow_fd(ctx, fd2, (i & 1) ? GSYS_FD_READ : 0);
  });
  std::thread buf_churn([&] {
    uint32_t bid = churn_id;
    while (!done.load()) {
      gsys_test_unregister_now(ctx, bid);
      if (gsys_register_buffer(ctx, churn_base, dummy.data(), dummy.size(), GSYS_BUF_HOST, &bid))
        break;
    }
  });
  // calls into no registered range: their validation scans the whole
  // table, the slot being rewritten included, and must fail with -EFAULT
  std::atomic<int> bad{0};
  std::thread prober([&] {
    for (uint32_t i = 0; !done.load(); ++i) {
      if (ph.doorbell) usleep(i % 97);  // sparse: the pollers go idle in between
      const uint64_t a[6] = {(uint64_t)fd, 1ull << 47, kItem, 0, 0, 0};
      int64_t r = 0;
      if (gsys_test_raw_call(ctx, GSYS_NR_PREAD64, GSYS_F_BLOCKING, a, &r, 10000000000ull) ||
          r != -EFAULT)
        bad.store(1);
    }
  });
  const int rc = gsys_test_emulate(ctx, ph.threads, 256, ph.group, ph.mode, fd, dev, ldev, kItem,
                                   offs.data(), rets.data(), 60000000000ull);
  done.store(true);
  fd_churn.join();
  buf_churn.join();
  prober.join();
  if (rc) return fail(ph.name, rc);
  if (bad.load()) return fail("unregistered range not refused");
  if (gsys_wait(ctx, 10000000000ull)) return fail("gsys_wait");
  if (ph.doorbell) {
    // calls after pauses long enough for every poller to block
    for (int i = 0; i < 50; ++i) {
      usleep(300);
      const uint64_t a[6] = {(uint64_t)fd, dev, kItem, (uint64_t)i * kItem, 0, 0};
      int64_t r = 0;
      if (gsys_test_raw_call(ctx, GSYS_NR_PREAD64, GSYS_F_BLOCKING, a, &r, 10000000000ull) ||
          r != kItem)
        return fail("call after a pause", i, (long)r);
      for (uint32_t b = 0; b < kItem; ++b)
        if (((const uint8_t*)host)[b] != pattern((uint64_t)i * kItem + b))
          return fail("byte after a pause", i, (long)b);
    }
  }
  const uint8_t* h = (const uint8_t*)host;
  for (uint64_t k = ph.doorbell ? 1 : 0; k < n; ++k) {  // the pause calls reused buffer 0
    if (rets[k] != kItem) return fail("ret", (long)k, (long)rets[k]);
    for (uint32_t b = 0; b < kItem; ++b)
      if (h[k * kItem + b] != pattern(offs[k] + b)) return fail("byte", (long)k, (long)b);
  }
  gsys_stats st;
  if (gsys_stats_get(ctx, &st, 0)) return fail("stats");
  if (ph.doorbell && st.doorbell_sleeps == 0) return fail("no poller blocked");
  std::vector<uint64_t> led(6 * (st.claimed + 1));
  const int64_t m = gsys_ledger(ctx, led.data(), st.claimed + 1, 0);
  if ((uint64_t)m != st.claimed) return fail("ledger", (long)m, (long)st.claimed);
  for (int64_t i = 0; i < m; ++i)
    if (led[6 * i] != (uint64_t)i) return fail("ledger order", (long)i, (long)led[6 * i]);
  if (gsys_shutdown(ctx, 5000000000ull)) return fail("shutdown");
  close(fd);
  close(fd2);
  printf("%s ok: %lu calls, %lu tickets\n", ph.name, (unsigned long)n,
         (unsigned long)st.claimed);
  return 0;
}

// List calls whose descriptor lists are unregistered and freed while the
// calls are in flight.  Four callers keep issuing blocking list preads of
// 64 items, each with its own list (a call writes its results back into its
// list) in one registered block at a fixed device address; a churner
// replaces the host memory behind that address: it fills a fresh block,
// drops the old registration (the grace period only), frees the old memory
// and registers the fresh block.  A call sees either a whole list (every
// item read) or no registration (-EFAULT), never freed memory.
int run_list_free_phase(const std::string& path) {
  gsys_config cfg;
  memset(&cfg, 0, sizeof cfg);
  cfg.abi_version = GSYS_ABI_VERSION;
  cfg.ring_slots = 4096;
  cfg.service_threads = 4;
  cfg.flags = GSYS_CFG_NO_DEVICE | GSYS_CFG_NO_PIN;
  gsys_ctx* ctx = nullptr;
  if (int e = gsys_init(&cfg, &ctx)) return fail("gsys_init", e);
  const int fd = open(path.c_str(), O_RDONLY);
  if (fd < 0 || gsys_allow_fd(ctx, fd, GSYS_FD_READ)) return fail("open / allow_fd");
  constexpr uint32_t kN = 64, kLen = 512;
  void* host = nullptr;
  uint64_t dev = 0;
  uint32_t id = 0;
  if (gsys_host_alloc(ctx, 8ull * kN * kLen, &host, &dev, &id)) return fail("host_alloc");
  constexpr uint32_t kCallers = 4;
  const uint64_t list_dev = 1ull << 45;  // the lists' device address (any unused range)
  const uint64_t block = kCallers * kN * sizeof(gsys_iodesc);
  auto fresh = [&]() {
    gsys_iodesc* L = new gsys_iodesc[kCallers * kN];
    for (uint32_t i = 0; i < kCallers * kN; ++i)
      L[i] = gsys_iodesc{(uint64_t)(i % kN) * kLen, (i % kN) * kLen, (int32_t)kLen};
    return L;
  };
  gsys_iodesc* cur = fresh();
  uint32_t lid = 0;
  if (gsys_register_buffer(ctx, list_dev, cur, block, GSYS_BUF_HOST, &lid))
    return fail("register list");
  std::atomic<bool> done{false};
  std::atomic<int> bad{0};
  std::atomic<uint64_t> whole{0}, refused{0};
  std::vector<std::thread> callers;
  for (uint32_t t = 0; t < kCallers; ++t)
    callers.emplace_back([&, t] {
      const uint64_t a[6] = {(uint64_t)fd, list_dev + t * kN * sizeof(gsys_iodesc), kN,
                             dev + (uint64_t)t * 2 * kN * kLen, 0, 0};
      for (int i = 0; i < 400 && !bad.load(); ++i) {
        int64_t r = 0;
        if (gsys_test_raw_call(ctx, GSYS_NR_PREAD64, GSYS_F_BLOCKING | GSYS_F_LIST, a, &r,
                               30000000000ull)) {
          bad.store(1);
        } else if (r == (int64_t)kN * kLen) {
          whole.fetch_add(1);
        } else if (r == -EFAULT) {
          refused.fetch_add(1);
        } else {
          bad.store(2);
        }
      }
    });
  std::thread churner([&] {
    while (!done.load()) {
      gsys_iodesc* next = fresh();
      if (gsys_test_unregister_now(ctx, lid)) { bad.store(3); break; }
      delete[] cur;  // no service thread may touch it any more
      cur = next;
      if (gsys_register_buffer(ctx, list_dev, cur, block, GSYS_BUF_HOST, &lid)) {
        bad.store(4);
        break;
      }
    }
  });
  for (auto& c : callers) c.join();
  done.store(true);
  churner.join();
  if (bad.load()) return fail("list calls while freeing lists", bad.load());
  if (!whole.load()) return fail("no list call saw a whole list");
  if (gsys_wait(ctx, 10000000000ull)) return fail("gsys_wait");
  // with nothing outstanding the public call may drop and free it
  if (gsys_unregister_buffer(ctx, lid)) return fail("unregister when quiet");
  delete[] cur;
  if (gsys_shutdown(ctx, 5000000000ull)) return fail("shutdown");
  close(fd);
  printf("lists freed in flight ok: %lu whole, %lu refused\n", (unsigned long)whole.load(),
         (unsigned long)refused.load());
  return 0;
}

}  // namespace

int main(int argc, char** argv) {
  if (argc < 2) return fail("usage: pool_tsan_driver <tmp dir>");
  const std::string path = std::string(argv[1]) + "/pool_tsan.bin";
  {
    std::vector<uint8_t> data(kFile);
    for (uint64_t i = 0; i < kFile; ++i) data[i] = pattern(i);
    FILE* f = fopen(path.c_str(), "wb");
    if (!f || fwrite(data.data(), 1, kFile, f) != kFile) return fail("write file");
    fclose(f);
  }
  const Phase phases[] = {
      {"wavefront groups, blocking", 6, 64, GSYS_EMU_BLOCKING, 1, 0, false, false},
      {"small groups, non-blocking", 6, 8, 0, 1, 0, false, false},
      {"list calls, blocking", 4, 16, GSYS_EMU_LIST | GSYS_EMU_BLOCKING, 1, 0, false, false},
      {"list calls, non-blocking", 4, 32, GSYS_EMU_LIST, 1, 0, true, false},
      {"coalesced bundles", 6, 64, GSYS_EMU_BLOCKING, 8, 2000, true, false},
      {"doorbell", 4, 8, GSYS_EMU_BLOCKING, 1, 0, false, true},
  };
  setenv("GSYS_DOORBELL_BACKSTOP_US", "30000000", 1);
  for (const Phase& ph : phases)
    if (int e = run_phase(path, ph)) return e;
  if (int e = run_list_free_phase(path)) return e;
  unlink(path.c_str());
  return 0;
}
