// Host read capacity: how fast `threads` host threads copy a list of file
// ranges into memory with pread, with no GPU work at all.  The word search's
// host side makes exactly these copies (section 7.1: the CPU services the
// chunk reads whose bytes the GPU scans), so this rate bounds the file scan
// beside the host link.
#include <errno.h>
#include <time.h>
#include <unistd.h>

#include <atomic>
#include <thread>
#include <vector>

#include "gsys.h"

namespace {

uint64_t now_ns() {
  timespec t;
  clock_gettime(CLOCK_MONOTONIC, &t);
  return (uint64_t)t.tv_sec * 1000000000ull + (uint64_t)t.tv_nsec;
}

}  // namespace

int gsys_host_pread_rate(const int* fds, const uint64_t* offs, const uint32_t* lens, uint64_t n,
                         uint8_t* dst, uint64_t slot_bytes, uint64_t n_slots, uint32_t threads,
                         uint32_t reps, double* out_gbps) {
  if (!fds || !offs || !lens || !dst || !out_gbps || !n || !n_slots || !threads || !reps ||
      threads > 1024)
    return -EINVAL;
  for (uint64_t i = 0; i < n; ++i)
    if (lens[i] > slot_bytes) return -EINVAL;
  double best = 0.0;
  for (uint32_t r = 0; r < reps; ++r) {
    std::atomic<uint64_t> next{0}, bytes{0};
    std::atomic<int> err{0};
    auto work = [&] {
      uint64_t mine = 0;
      for (;;) {
        const uint64_t i = next.fetch_add(1, std::memory_order_relaxed);
        if (i >= n) break;
        const ssize_t k = pread(fds[i], dst + (i % n_slots) * slot_bytes, lens[i], (off_t)offs[i]);
        if (k < 0) {
          int z = 0;
          err.compare_exchange_strong(z, -errno);
          break;
        }
        mine += (uint64_t)k;
      }
      bytes.fetch_add(mine, std::memory_order_relaxed);
    };
    const uint64_t t0 = now_ns();
    std::vector<std::thread> ts;
    ts.reserve(threads);
    for (uint32_t t = 0; t < threads; ++t) ts.emplace_back(work);
    for (auto& t : ts) t.join();
    const uint64_t dt = now_ns() - t0;
    if (err.load()) return err.load();
    const double gbps = (double)bytes.load() / (double)(dt ? dt : 1);
    if (gbps > best) best = gbps;
  }
  *out_gbps = best;
  return 0;
}
