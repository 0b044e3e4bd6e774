// Host read capacity: how fast `threads` host threads copy a list of file
// ranges into memory with pread, with no GPU work at all.  The word search's
// host side makes exactly these copies (section 7.1: the CPU services the
// chunk reads whose bytes the GPU scans), so this rate bounds the file scan
// beside the host link.  Like the pool's pollers, each thread reads through
// its own open file description of every file (a re-open of
// /proc/self/fd/N), so the threads do not share a description's reference
// count.
#include <errno.h>
#include <fcntl.h>
#include <stdio.h>
#include <time.h>
#include <unistd.h>

#include <algorithm>
#include <atomic>
#include <thread>
#include <unordered_map>
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
  // every thread's own description of every file, opened before any timing
  // (the pool's pollers keep theirs for the life of the context)
  std::vector<int> distinct;
  {
    std::unordered_map<int, int> seen;
    for (uint64_t i = 0; i < n; ++i)
      if (seen.emplace(fds[i], 0).second) distinct.push_back(fds[i]);
  }
  std::vector<std::unordered_map<int, int>> own(threads);
  int open_err = 0;
  for (uint32_t t = 0; t < threads && !open_err; ++t)
    for (int fd : distinct) {
      char path[32];
      snprintf(path, sizeof path, "/proc/self/fd/%d", fd);
      const int c = fd < 0 ? -1 : open(path, O_RDONLY | O_CLOEXEC);
      if (c < 0 && fd >= 0 && (errno == EMFILE || errno == ENFILE)) {
        own[t].emplace(fd, -1);  // out of descriptors: the caller's own, as a poller does
        continue;
      }
      if (c < 0) {
        open_err = fd < 0 || errno == ENOENT ? -EBADF : -errno;
        break;
      }
      own[t].emplace(fd, c);
    }
  auto close_all = [&] {
    for (auto& m : own)
      for (const auto& kv : m)
        if (kv.second >= 0) close(kv.second);
  };
  if (open_err) {
    close_all();
    return open_err;
  }
  // ranges are claimed in runs (up to 256, as a work-group's list call
  // carries), small enough that every thread gets several
  const uint64_t run = std::max<uint64_t>(1, std::min<uint64_t>(256, n / (8ull * threads)));
  double best = 0.0;
  for (uint32_t r = 0; r < reps; ++r) {
    std::atomic<uint64_t> next{0}, bytes{0};
    std::atomic<int> err{0};
    auto work = [&](uint32_t t) {
      const std::unordered_map<int, int>& mine_fds = own[t];
      int last_fd = -1, last_own = -1;
      uint64_t mine = 0;
      for (;;) {
        const uint64_t i0 = next.fetch_add(run, std::memory_order_relaxed);
        if (i0 >= n || err.load(std::memory_order_relaxed)) break;
        const uint64_t i1 = std::min(n, i0 + run);
        for (uint64_t i = i0; i < i1; ++i) {
          if (fds[i] != last_fd) {
            last_fd = fds[i];
            last_own = mine_fds.at(fds[i]);
            if (last_own < 0) last_own = fds[i];
          }
          const ssize_t k = pread(last_own, dst + (i % n_slots) * slot_bytes, lens[i],
                                  (off_t)offs[i]);
          if (k < 0) {
            int z = 0;
            err.compare_exchange_strong(z, -errno);
            break;
          }
          mine += (uint64_t)k;
        }
      }
      bytes.fetch_add(mine, std::memory_order_relaxed);
    };
    const uint64_t t0 = now_ns();
    std::vector<std::thread> ts;
    ts.reserve(threads);
    for (uint32_t t = 0; t < threads; ++t) ts.emplace_back(work, t);
    for (auto& t : ts) t.join();
    const uint64_t dt = now_ns() - t0;
    if (err.load()) {
      close_all();
      return err.load();
    }
    const double gbps = (double)bytes.load() / (double)(dt ? dt : 1);
    if (gbps > best) best = gbps;
  }
  close_all();
  *out_gbps = best;
  return 0;
}
