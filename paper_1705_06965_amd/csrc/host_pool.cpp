// Host service pool (see host_pool.hpp).
#include "host_pool.hpp"

#include <errno.h>
#include <fcntl.h>
#include <netinet/in.h>
#include <pthread.h>
#include <sched.h>
#include <stdio.h>
#include <string.h>
#include <sys/mman.h>
#include <sys/socket.h>
#include <sys/stat.h>
#include <sys/syscall.h>
#include <linux/openat2.h>
#include <time.h>
#include <unistd.h>
#include <immintrin.h>

#include <algorithm>

static_assert(sizeof(gsys_slot) == 64, "slot must be one 64-byte line");
static_assert(sizeof(gsys_comp) == 16, "completion record is 16 bytes");
static_assert(sizeof(gsys_iodesc) == 16, "io descriptor is 16 bytes");
static_assert(sizeof(gsys_netdesc) == 32, "net descriptor is 32 bytes");
static_assert(GSYS_NR_READ == SYS_read && GSYS_NR_WRITE == SYS_write &&
                  GSYS_NR_MMAP == SYS_mmap && GSYS_NR_MUNMAP == SYS_munmap &&
                  GSYS_NR_PREAD64 == SYS_pread64 && GSYS_NR_PWRITE64 == SYS_pwrite64 &&
                  GSYS_NR_MADVISE == SYS_madvise && GSYS_NR_SENDTO == SYS_sendto &&
                  GSYS_NR_RECVFROM == SYS_recvfrom && GSYS_NR_CLOSE == SYS_close &&
                  GSYS_NR_OPENAT == SYS_openat,
              "call numbers are the host's system-call numbers");

namespace gsys_host {

namespace {

constexpr uint8_t kPermMask = 0xF;  // GSYS_FD_READ | WRITE | SOCK | DIR
constexpr uint8_t kOwned = 0x40;    // opened by a GPU openat: the pool closes it
constexpr uint8_t kRegular = 0x80;  // fd refers to a regular file (transfers may merge)
// Slot state used by the pool only: taken by its owner's scan, not yet
// started; another poller may still take it (see host_pool.hpp).
constexpr uint32_t kQueued = 5u;
// A poller with nothing to do spins this long before it naps between polls
// (20 us asked; with the default timer slack a nap lasts ~70 us).
constexpr uint64_t kSpinNs = 5000000;

inline uint64_t now_ns() {
  timespec ts;
  clock_gettime(CLOCK_MONOTONIC, &ts);
  return (uint64_t)ts.tv_sec * 1000000000ull + (uint64_t)ts.tv_nsec;
}

inline uint64_t ld_acq(const uint64_t* p) { return __atomic_load_n(p, __ATOMIC_ACQUIRE); }
inline void st_rel(uint64_t* p, uint64_t v) { __atomic_store_n(p, v, __ATOMIC_RELEASE); }

inline int hist_bucket(uint64_t n) {
  if (n <= 1) return 0;
  if (n == 2) return 1;
  if (n <= 4) return 2;
  if (n <= 8) return 3;
  if (n <= 16) return 4;
  if (n <= 32) return 5;
  if (n <= 64) return 6;
  return 7;
}

inline uint64_t mix64(uint64_t x) {
  x ^= x >> 33;
  x *= 0xff51afd7ed558ccdull;
  x ^= x >> 33;
  return x;
}

bool loopback_v4(const uint8_t* a, uint64_t len) {
  if (len < sizeof(sockaddr_in)) return false;
  sockaddr_in sa;
  memcpy(&sa, a, sizeof sa);
  return sa.sin_family == AF_INET && ntohl(sa.sin_addr.s_addr) == INADDR_LOOPBACK;
}

}  // namespace

Pool::Pool(gsys_slot* ring, gsys_comp* comp, uint64_t D, uint64_t C, uint64_t* retired_lo,
           const gsys_config& cfg)
    : ring_(ring), comp_(comp), D_(D), C_(C), retired_lo_(retired_lo), fdperm_(65536),
      fdgen_(65536) {
  // the CPUs this process may run on (a container's share, not the machine)
  cpu_set_t allowed;
  CPU_ZERO(&allowed);
  if (sched_getaffinity(0, sizeof allowed, &allowed) == 0)
    for (int c = 0; c < CPU_SETSIZE; ++c)
      if (CPU_ISSET(c, &allowed)) cpus_.push_back(c);
  if (cpus_.empty()) {
    const long n = sysconf(_SC_NPROCESSORS_ONLN);
    for (long c = 0; c < std::max(1L, n); ++c) cpus_.push_back((int)c);
  }
  const int ncpu = (int)cpus_.size();
  P_ = cfg.service_threads ? (int)cfg.service_threads : std::max(1, ncpu - 1);
  stripe_ = cfg.stripe ? cfg.stripe : 8;
  K_ = cfg.coalesce_max ? cfg.coalesce_max : 1;
  T_ns_ = cfg.coalesce_window_ns;
  if (K_ > 1 && stripe_ < K_) stripe_ = K_;
  if (stripe_ > 64) stripe_ = 64;
  if (K_ > 64) K_ = 64;
  first_cpu_ = cfg.first_cpu;
  pin_ = !(cfg.flags & GSYS_CFG_NO_PIN);
  ledger_on_ = (cfg.flags & GSYS_CFG_LEDGER) != 0;
  ledger_cap_ = cfg.ledger_capacity ? cfg.ledger_capacity : (1u << 20);
  for (auto& p : fdperm_) p.store(0);
  for (auto& g : fdgen_) g.store(0);
  copy_fds_ = !(cfg.flags & GSYS_CFG_SHARED_FDS);
  owned_ = std::vector<std::atomic<uint64_t>>((size_t)P_);
  for (int i = 0; i < P_; ++i) ledger_.push_back(std::make_unique<LedgerShard>());
  for (int i = 0; i <= P_; ++i) ctr_.push_back(std::make_unique<Counters>());
  for (int i = 0; i < P_; ++i) owned_[(size_t)i].store((uint64_t)i);
  {
    const char* e = getenv("GSYS_ARENA_HUGEPAGE");
    arena_huge_ = !(e && *e == '0');
    const char* st = getenv("GSYS_STEAL");
    steal_on_ = !(st && *st == '0');

  }
  fdcopies_.resize((size_t)P_);
}

Pool::~Pool() { stop_and_join(); }

void Pool::start() {
  stop_.store(false);
  next_stripe_.store((uint64_t)P_);
  for (int i = 0; i < P_; ++i) threads_.emplace_back([this, i] { poller(i); });
}

void Pool::stop_and_join() {
  stop_.store(true);
  if (db_) db_->ring();  // blocked pollers see the stop flag at once
  for (auto& t : threads_)
    if (t.joinable()) t.join();
  threads_.clear();
}

int Pool::allow_fd(int fd, uint32_t perms) {
  if (fd < 0 || fd >= (int)fdperm_.size()) return -EBADF;
  uint8_t v = (uint8_t)(perms & kPermMask);
  if (v) {
    struct stat st;
    if (fstat(fd, &st) != 0) return -errno;
    if ((v & GSYS_FD_DIR) && !S_ISDIR(st.st_mode)) return -ENOTDIR;
    if (S_ISREG(st.st_mode)) v |= kRegular;
  }
  fdgen_[fd].fetch_add(1, std::memory_order_acq_rel);
  fdperm_[fd].store(v, std::memory_order_release);
  return 0;
}

thread_local Pool::FdCopies* Pool::tls_copies_ = nullptr;
thread_local Pool::Counters* Pool::tls_ctr_ = nullptr;

namespace {
// A new open file description of the file behind `fd`, with its access mode
// and status flags; -1 if that is not possible.
int reopen_same(int fd) {
  const int fl = fcntl(fd, F_GETFL);
  if (fl < 0) return -1;
  char path[48];
  snprintf(path, sizeof path, "/proc/self/fd/%d", fd);
  const int keep = O_ACCMODE | O_APPEND | O_DIRECT | O_DSYNC | O_SYNC | O_NOATIME | O_NONBLOCK;
  return open(path, (fl & keep) | O_CLOEXEC);
}
}  // namespace

int Pool::fd_for(int64_t fd) {
  FdCopies* pc = tls_copies_;
  if (!pc || !copy_fds_ || fd < 0 || fd >= (int64_t)fdperm_.size() ||
      !(fdperm_[fd].load(std::memory_order_relaxed) & kRegular))
    return (int)fd;
  const uint32_t g = fdgen_[fd].load(std::memory_order_acquire);
  FdCopies::Ent* slot = nullptr;
  for (FdCopies::Ent& e : pc->e)
    if (e.src == (int)fd) {
      if (e.gen == g) return e.fd >= 0 ? e.fd : (int)fd;
      slot = &e;
      break;
    }
  if (!slot) slot = &pc->e[pc->next++ % FdCopies::kEnts];
  if (slot->fd >= 0) close(slot->fd);
  slot->src = (int)fd;
  slot->gen = g;
  slot->fd = reopen_same((int)fd);
  return slot->fd >= 0 ? slot->fd : (int)fd;
}

bool Pool::fd_ok(int64_t fd, uint32_t need) const {
  if (fd < 0 || fd >= (int64_t)fdperm_.size()) return false;
  uint8_t p = fdperm_[fd].load(std::memory_order_acquire);
  return (p & need) == need && (p & kPermMask) != 0;
}

int Pool::add_buffer(uint64_t dev, uint8_t* host, uint64_t bytes, uint32_t kind, uint32_t* id) {
  if (!bytes || (kind != GSYS_BUF_HOST && kind != GSYS_BUF_DEVICE)) return -EINVAL;
  if (kind == GSYS_BUF_HOST && !host) return -EINVAL;
  std::lock_guard<std::mutex> g(bufmu_);
  int n = nbufs_.load();
  if (n >= kMaxBufs) return -ENOSPC;
  for (int i = 0; i < n; ++i) {
    const Buf b = bufs_[i].load();
    if (dev < b.dev + b.bytes && b.dev < dev + bytes) return -EEXIST;
  }
  bufgen_.fetch_add(1, std::memory_order_acq_rel);  // odd: writers active
  bufs_[n].store(Buf{dev, host, bytes, kind, next_id_});
  nbufs_.store(n + 1, std::memory_order_release);
  bufgen_.fetch_add(1, std::memory_order_acq_rel);
  if (id) *id = next_id_;
  ++next_id_;
  return 0;
}

int Pool::remove_buffer(uint32_t id) {
  {
    std::lock_guard<std::mutex> g(bufmu_);
    int n = nbufs_.load();
    int i = 0;
    while (i < n && bufs_[i].id.load(std::memory_order_relaxed) != id) ++i;
    if (i == n) return -ENOENT;
    bufgen_.fetch_add(1, std::memory_order_acq_rel);
    bufs_[i].store(bufs_[n - 1].load());
    nbufs_.store(n - 1, std::memory_order_release);
    bufgen_.fetch_add(1, std::memory_order_acq_rel);
  }
  // Grace period.  A poller marks itself serving (a sequentially consistent
  // increment) before it looks up any address, so either it looks after the
  // entry went away, or the check below sees it serving and waits until it
  // has moved on.  No call a poller makes blocks (sockets are MSG_DONTWAIT,
  // files regular or opened non-blocking), so the wait is short.
  std::atomic_thread_fence(std::memory_order_seq_cst);
  for (int p = 0; p < P_; ++p) {
    const std::atomic<uint64_t>& sv = ctr_[(size_t)p]->serving;
    const uint64_t v = sv.load(std::memory_order_acquire);
    if (!(v & 1)) continue;
    while (sv.load(std::memory_order_acquire) == v) _mm_pause();
  }
  return 0;
}

// Host address of [dev, dev + len) if it lies inside one registered host
// buffer (or inside the arena, whose device address is its host address).
uint8_t* Pool::translate(uint64_t dev, uint64_t len, bool) {
  if (len > (1ull << 40) || dev + len < dev) return nullptr;
  if (arena_ && dev >= (uint64_t)arena_ && dev + len <= (uint64_t)arena_ + arena_bytes_)
    return (uint8_t*)dev;
  for (;;) {
    uint64_t g1 = bufgen_.load(std::memory_order_acquire);
    if (g1 & 1) {
      _mm_pause();
      continue;
    }
    uint8_t* r = nullptr;
    int n = nbufs_.load(std::memory_order_acquire);
    for (int i = 0; i < n; ++i) {
      const Buf b = bufs_[i].load();
      if (dev >= b.dev && dev + len <= b.dev + b.bytes) {
        r = b.kind == GSYS_BUF_HOST ? b.host + (dev - b.dev) : nullptr;
        break;
      }
    }
    std::atomic_thread_fence(std::memory_order_acquire);
    if (bufgen_.load(std::memory_order_relaxed) == g1) return r;
  }
}

void Pool::note_errno(int64_t ret) {
  if (ret >= 0) return;
  bump(ctr().err, 1);
  int b;
  switch ((int)-ret) {
    case EPERM: b = 0; break;
    case EBADF: b = 1; break;
    case EFAULT: b = 2; break;
    case EINVAL: b = 3; break;
    case EAGAIN: b = 4; break;
    case ESHUTDOWN: b = 5; break;
    case ETIMEDOUT: b = 6; break;
    default: b = 7;
  }
  bump(ctr().ehist[b], 1);
}

// Execute one request (a descriptor list goes to exec_list).
int64_t Pool::execute(const gsys_slot& s, uint64_t* calls, uint64_t* merged) {
  if (inj_left_.load(std::memory_order_acquire) && s.nr == inj_nr_.load(std::memory_order_relaxed)) {
    // an injected fault fails the whole request before anything runs
    uint32_t left = inj_left_.load(std::memory_order_acquire);
    while (left && !inj_left_.compare_exchange_weak(left, left - 1, std::memory_order_acq_rel))
      ;
    if (left) {
      const int64_t e = -(int64_t)inj_err_.load(std::memory_order_relaxed);
      if (s.flags & GSYS_F_LIST) note_errno(e);  // single calls are counted by the caller
      return e;
    }
  }
  if (s.flags & GSYS_F_LIST) return exec_list(s, calls, merged);
  const uint64_t* a = s.args;
  int64_t r;
  switch (s.nr) {
    case GSYS_NR_PREAD64:
    case GSYS_NR_READ: {
      if (!fd_ok((int64_t)a[0], GSYS_FD_READ)) return -EBADF;
      if (a[2] > (1ull << 31)) return -EINVAL;
      uint8_t* h = translate(a[1], a[2], true);
      if (!h) return -EFAULT;
      ssize_t n = s.nr == GSYS_NR_PREAD64 ? pread(fd_for((int64_t)a[0]), h, a[2], (off_t)a[3])
                                          : read((int)a[0], h, a[2]);
      ++*calls;
      r = n < 0 ? -(int64_t)errno : (int64_t)n;
      if (r > 0) bump(ctr().in, (uint64_t)r);
      return r;
    }
    case GSYS_NR_PWRITE64:
    case GSYS_NR_WRITE: {
      if (!fd_ok((int64_t)a[0], GSYS_FD_WRITE)) return -EBADF;
      if (a[2] > (1ull << 31)) return -EINVAL;
      uint8_t* h = translate(a[1], a[2], false);
      if (!h) return -EFAULT;
      ssize_t n = s.nr == GSYS_NR_PWRITE64 ? pwrite(fd_for((int64_t)a[0]), h, a[2], (off_t)a[3])
                                           : write((int)a[0], h, a[2]);
      ++*calls;
      r = n < 0 ? -(int64_t)errno : (int64_t)n;
      if (r > 0) bump(ctr().out, (uint64_t)r);
      return r;
    }
    case GSYS_NR_SENDTO: {
      if (!fd_ok((int64_t)a[0], GSYS_FD_SOCK)) return -EBADF;
      if (a[3] & ~(uint64_t)MSG_DONTWAIT) return -EINVAL;
      if (a[2] > 65507) return -EINVAL;
      uint8_t* h = translate(a[1], a[2], false);
      uint8_t* addr = translate(a[4], a[5], false);
      if (!h || !addr) return -EFAULT;
      if (!loopback_v4(addr, a[5])) return -EINVAL;
      ssize_t n = sendto((int)a[0], h, a[2], (int)a[3] | MSG_DONTWAIT, (const sockaddr*)addr,
                         (socklen_t)a[5]);
      ++*calls;
      r = n < 0 ? -(int64_t)errno : (int64_t)n;
      if (r > 0) bump(ctr().out, (uint64_t)r);
      return r;
    }
    case GSYS_NR_RECVFROM: {
      if (!fd_ok((int64_t)a[0], GSYS_FD_SOCK)) return -EBADF;
      if (a[3] & ~(uint64_t)MSG_DONTWAIT) return -EINVAL;
      if (a[2] > 65536) return -EINVAL;
      uint8_t* h = translate(a[1], a[2], true);
      if (!h) return -EFAULT;
      sockaddr_in from;
      socklen_t fl = sizeof from;
      // A poller never blocks inside the kernel: recvfrom is always
      // MSG_DONTWAIT and an empty socket answers -EAGAIN.
      ssize_t n = recvfrom((int)a[0], h, a[2], MSG_DONTWAIT, (sockaddr*)&from, &fl);
      ++*calls;
      r = n < 0 ? -(int64_t)errno : (int64_t)n;
      if (r >= 0 && a[4]) {
        uint8_t* out = translate(a[4], sizeof from, true);
        if (out) memcpy(out, &from, sizeof from);
      }
      if (r > 0) bump(ctr().in, (uint64_t)r);
      return r;
    }
    case GSYS_NR_MMAP: {
      // anonymous private memory at a fixed address inside the arena
      const uint64_t addr = a[0], len = a[1];
      if (!arena_ || (addr & 4095) || !len || (len & 4095)) return -EINVAL;
      if (addr < (uint64_t)arena_ || addr + len > (uint64_t)arena_ + arena_bytes_) return -EFAULT;
      if (a[2] & ~(uint64_t)(PROT_READ | PROT_WRITE)) return -EINVAL;
      if ((a[3] & ~(uint64_t)MAP_FIXED) != (uint64_t)(MAP_PRIVATE | MAP_ANONYMOUS)) return -EINVAL;
      if ((int64_t)a[4] != -1 || a[5] != 0) return -EINVAL;
      void* m = mmap((void*)addr, len, (int)a[2], MAP_PRIVATE | MAP_ANONYMOUS | MAP_FIXED, -1, 0);
      ++*calls;
      if (m == MAP_FAILED) return -(int64_t)errno;
      // Arena policy: back 2 MiB-aligned ranges with transparent huge pages
      // where the kernel allows it (one fault per 2 MiB instead of 512).  A
      // hint only: contents and the call's result are unchanged.
      if (arena_huge_ && ((uint64_t)m & ((2ull << 20) - 1)) == 0 && len >= (2ull << 20))
        madvise(m, len, MADV_HUGEPAGE);
      return (int64_t)(uint64_t)m;
    }
    case GSYS_NR_MUNMAP: {
      // inside the arena an unmap returns the range to the reservation
      const uint64_t addr = a[0], len = a[1];
      if (!arena_ || (addr & 4095) || !len) return -EINVAL;
      if (addr < (uint64_t)arena_ || addr + len > (uint64_t)arena_ + arena_bytes_) return -EFAULT;
      void* m = mmap((void*)addr, (len + 4095) & ~4095ull, PROT_NONE,
                     MAP_PRIVATE | MAP_ANONYMOUS | MAP_FIXED | MAP_NORESERVE, -1, 0);
      ++*calls;
      return m == MAP_FAILED ? -(int64_t)errno : 0;
    }
    case GSYS_NR_MADVISE: {
      const uint64_t addr = a[0], len = a[1];
      if (a[2] != (uint64_t)MADV_DONTNEED) return -EINVAL;
      if (!arena_ || (addr & 4095)) return -EINVAL;
      if (addr < (uint64_t)arena_ || addr + len > (uint64_t)arena_ + arena_bytes_) return -EFAULT;
      int rc = madvise((void*)addr, len, MADV_DONTNEED);
      ++*calls;
      return rc ? -(int64_t)errno : 0;
    }
    case GSYS_NR_OPENAT: {
      // a file beneath an allowed directory; the new fd belongs to the pool
      const int64_t dfd = (int64_t)a[0];
      if (!fd_ok(dfd, GSYS_FD_DIR)) return -EBADF;
      const uint8_t dperm = fdperm_[dfd].load(std::memory_order_acquire);
      const uint8_t* path = translate(a[1], GSYS_PATH_MAX, false);
      if (!path) return -EFAULT;
      if (!memchr(path, 0, GSYS_PATH_MAX)) return -ENAMETOOLONG;
      const uint64_t fl = a[2];
      const uint64_t ok_fl = O_ACCMODE | O_CREAT | O_TRUNC | O_APPEND;
      if ((fl & ~ok_fl) || (fl & O_ACCMODE) == O_ACCMODE) return -EINVAL;
      const bool writes = (fl & O_ACCMODE) != O_RDONLY || (fl & (O_CREAT | O_TRUNC));
      if (writes && !(dperm & GSYS_FD_WRITE)) return -EPERM;
      if (!writes && !(dperm & GSYS_FD_READ)) return -EPERM;
      struct open_how how;
      memset(&how, 0, sizeof how);
      // O_NONBLOCK: opening a FIFO must not block a poller (regular files
      // ignore the flag)
      how.flags = fl | O_CLOEXEC | O_NONBLOCK;
      how.mode = (fl & O_CREAT) ? (a[3] & 0666) : 0;
      how.resolve = RESOLVE_BENEATH | RESOLVE_NO_MAGICLINKS;
      const long nfd = syscall(SYS_openat2, (int)dfd, (const char*)path, &how, sizeof how);
      ++*calls;
      if (nfd < 0) return -(int64_t)errno;
      if (nfd >= (long)fdperm_.size()) {
        close((int)nfd);
        return -EMFILE;
      }
      uint8_t v = kOwned;
      if ((fl & O_ACCMODE) != O_WRONLY) v |= GSYS_FD_READ;
      if ((fl & O_ACCMODE) != O_RDONLY) v |= GSYS_FD_WRITE;
      struct stat st;
      if (fstat((int)nfd, &st) == 0 && S_ISREG(st.st_mode)) v |= kRegular;
      fdgen_[nfd].fetch_add(1, std::memory_order_acq_rel);
      fdperm_[nfd].store(v, std::memory_order_release);
      return (int64_t)nfd;
    }
    case GSYS_NR_CLOSE: {
      // only what a GPU openat opened; the fd is revoked before it is closed
      const int64_t fd = (int64_t)a[0];
      if (fd < 0 || fd >= (int64_t)fdperm_.size()) return -EBADF;
      uint8_t p = fdperm_[fd].load(std::memory_order_acquire);
      if (!(p & kOwned) || !fdperm_[fd].compare_exchange_strong(p, 0, std::memory_order_acq_rel))
        return -EBADF;
      fdgen_[fd].fetch_add(1, std::memory_order_acq_rel);
      ++*calls;
      return close((int)fd) ? -(int64_t)errno : 0;
    }
    default:
      bump(ctr().rej, 1);
      return -EPERM;
  }
}

void Pool::close_owned() {
  for (size_t fd = 0; fd < fdperm_.size(); ++fd) {
    uint8_t p = fdperm_[fd].load(std::memory_order_acquire);
    if ((p & kOwned) && fdperm_[fd].compare_exchange_strong(p, 0, std::memory_order_acq_rel)) {
      fdgen_[fd].fetch_add(1, std::memory_order_acq_rel);
      close((int)fd);
    }
  }
}

// A descriptor-list request: the group's calls run in list order on this
// thread.  File transfers adjacent both in the file and in memory are merged
// into one call and the result is split back over the descriptors.  Returns
// the bytes moved once the list has run (each descriptor's len_ret holds its
// own result, errors included), or -errno when the list is refused before any
// descriptor runs.
int64_t Pool::exec_list(const gsys_slot& s, uint64_t* calls, uint64_t* merged) {
  const uint64_t* a = s.args;
  const int64_t fd = (int64_t)a[0];
  const uint64_t count = a[2];
  const uint64_t base = a[3];
  if (count > (1ull << 24)) return -EINVAL;
  uint64_t total = 0;
  if (s.nr == GSYS_NR_PREAD64 || s.nr == GSYS_NR_PWRITE64) {
    const bool rd = s.nr == GSYS_NR_PREAD64;
    if (!fd_ok(fd, rd ? GSYS_FD_READ : GSYS_FD_WRITE)) return -EBADF;
    gsys_iodesc* d = (gsys_iodesc*)translate(a[1], count * sizeof(gsys_iodesc), true);
    if (!d && count) return -EFAULT;
    const bool mergeable = (fdperm_[fd].load(std::memory_order_relaxed) & kRegular) != 0;
    const int xfd = fd_for(fd);
    uint64_t i = 0;
    while (i < count) {
      const uint64_t off = d[i].off;
      const uint64_t boff = d[i].buf_off;
      int64_t len = d[i].len_ret;
      uint64_t j = i + 1;
      if (len >= 0 && mergeable) {
        uint64_t run = (uint64_t)len;
        while (j < count && d[j].len_ret >= 0 && d[j].off == off + run &&
               (uint64_t)d[j].buf_off == boff + run && run + (uint64_t)d[j].len_ret <= (1ull << 30)) {
          run += (uint64_t)d[j].len_ret;
          ++j;
        }
        len = (int64_t)run;
      }
      int64_t r;
      uint8_t* h = len >= 0 ? translate(base + boff, (uint64_t)len, rd) : nullptr;
      if (len < 0) {
        r = -EINVAL;
      } else if (!h) {
        r = -EFAULT;
      } else {
        ssize_t n = rd ? pread(xfd, h, (size_t)len, (off_t)off)
                       : pwrite(xfd, h, (size_t)len, (off_t)off);
        ++*calls;
        r = n < 0 ? -(int64_t)errno : (int64_t)n;
      }
      if (j > i + 1) *merged += j - i - 1;
      // split the result back over the merged descriptors
      uint64_t prefix = 0;
      for (uint64_t k = i; k < j; ++k) {
        const int64_t lk = d[k].len_ret;
        int64_t rk;
        if (r < 0) {
          rk = r;
        } else {
          const int64_t left = r - (int64_t)prefix;
          rk = left <= 0 ? 0 : (left < lk ? left : lk);
        }
        prefix += (uint64_t)(lk > 0 ? lk : 0);
        d[k].len_ret = (int32_t)rk;
        if (rk > 0) total += (uint64_t)rk;
        note_errno(rk);
      }
      i = j;
    }
    if (rd) bump(ctr().in, total);
    else bump(ctr().out, total);
  } else if (s.nr == GSYS_NR_RECVFROM || s.nr == GSYS_NR_SENDTO) {
    if (!fd_ok(fd, GSYS_FD_SOCK)) return -EBADF;
    if (a[4] & ~(uint64_t)MSG_DONTWAIT) return -EINVAL;
    gsys_netdesc* d = (gsys_netdesc*)translate(a[1], count * sizeof(gsys_netdesc), true);
    if (!d && count) return -EFAULT;
    const bool rx = s.nr == GSYS_NR_RECVFROM;
    // Runs of valid descriptors go to the kernel together (recvmmsg /
    // sendmmsg, up to kBatch datagrams per call) with the same per-datagram
    // results as one call each; an invalid descriptor gets its own error
    // and ends the run.  A receive list stops at the first -EAGAIN: the
    // socket is drained, later receive descriptors report -EAGAIN.
    constexpr uint32_t kBatch = 64;
    mmsghdr mm[kBatch];
    iovec iov[kBatch];
    sockaddr_in from[kBatch];
    uint64_t idx[kBatch];
    bool drained = false;
    auto finish = [&](uint64_t i, int64_t r) {
      d[i].len_ret = (int32_t)r;
      if (r > 0) total += (uint64_t)r;
      if (r != -EAGAIN) note_errno(r);
    };
    uint64_t i = 0;
    while (i < count) {
      // gather the next run of valid descriptors
      uint32_t n = 0;
      while (i < count && n < kBatch) {
        const int32_t len = d[i].len_ret;
        uint8_t* h = len >= 0 ? translate(base + d[i].buf_off, (uint64_t)len, true) : nullptr;
        int64_t bad = 0;
        if (len < 0 || len > 65507) bad = -EINVAL;
        else if (!h) bad = -EFAULT;
        else if (!rx && !loopback_v4(d[i].addr, d[i].addr_len)) bad = -EINVAL;
        else if (rx && drained) bad = -EAGAIN;
        if (bad) {
          if (n) break;  // run the batch first, then this descriptor
          finish(i++, bad);
          continue;
        }
        iov[n].iov_base = h;
        iov[n].iov_len = (size_t)len;
        memset(&mm[n], 0, sizeof mm[n]);
        mm[n].msg_hdr.msg_iov = &iov[n];
        mm[n].msg_hdr.msg_iovlen = 1;
        if (rx) {
          mm[n].msg_hdr.msg_name = &from[n];
          mm[n].msg_hdr.msg_namelen = sizeof from[n];
        } else {
          mm[n].msg_hdr.msg_name = d[i].addr;
          mm[n].msg_hdr.msg_namelen = (socklen_t)d[i].addr_len;
        }
        idx[n++] = i++;
      }
      // run it; a partial batch continues from the first datagram not done
      uint32_t k = 0;
      while (k < n) {
        const int m = rx ? recvmmsg((int)fd, mm + k, n - k, MSG_DONTWAIT, nullptr)
                         : sendmmsg((int)fd, mm + k, n - k, (int)a[4] | MSG_DONTWAIT);
        ++*calls;
        if (m < 0) {
          const int64_t e = -(int64_t)errno;
          if (rx && e == -EAGAIN) {
            drained = true;
            for (; k < n; ++k) finish(idx[k], -EAGAIN);
          } else {
            finish(idx[k++], e);  // this datagram failed; the rest try again
          }
          continue;
        }
        if (m > 1) *merged += (uint64_t)(m - 1);
        for (int q = 0; q < m; ++q, ++k) {
          if (rx) {
            memcpy(d[idx[k]].addr, &from[k], sizeof from[k]);
            d[idx[k]].addr_len = mm[k].msg_hdr.msg_namelen;
          }
          finish(idx[k], (int64_t)mm[k].msg_len);
        }
        if (rx && k < n) {
          // fewer datagrams than asked: the socket had no more
          drained = true;
          for (; k < n; ++k) finish(idx[k], -EAGAIN);
        }
      }
    }
    if (rx) bump(ctr().in, total);
    else bump(ctr().out, total);
  } else {
    bump(ctr().rej, 1);
    return -EPERM;
  }
  // the list ran: its result is the bytes moved; each descriptor holds its
  // own result (a negative call result means the list did not run at all)
  return (int64_t)total;
}

// Post the result (section 5): the return value goes to the slot's argument
// field and to the ticket's completion record; a blocking slot becomes
// FINISHED (the GPU frees it), a non-blocking one becomes FREE for the next
// lap.  Then the claim group's completion count goes up by one.
void Pool::complete(uint64_t t, gsys_slot* s, int64_t ret, StampAcc* acc) {
  const uint8_t flags = s->flags;
  const uint64_t head = t - s->grp_off;
  gsys_comp* c = &comp_[t & (C_ - 1)];
  __atomic_store_n(&c->ret, ret, __ATOMIC_RELAXED);
  if (flags & GSYS_F_BLOCKING) {
    __atomic_store_n((int64_t*)&s->args[0], ret, __ATOMIC_RELAXED);
    st_rel(&s->ctl, GSYS_CTL(t, GSYS_ST_FINISHED));
  } else {
    st_rel(&s->ctl, GSYS_CTL(t + D_, GSYS_ST_FREE));
  }
  if (!acc) {
    add_stamp(head, 1);
    return;
  }
  if (acc->k && acc->head != head) flush_stamp(*acc);
  acc->head = head;
  ++acc->k;
}

void Pool::add_stamp(uint64_t head, uint32_t k) {
  // release: the results posted before are visible to whoever sees the count
  uint64_t* stp = &comp_[head & (C_ - 1)].stamp;
  uint64_t v = __atomic_load_n(stp, __ATOMIC_ACQUIRE);
  for (;;) {
    const uint64_t vh = v >> 8;
    if (vh > head) break;  // lapped by a later group (the waiter reports -EOVERFLOW)
    const uint64_t nv = vh == head ? v + k : GSYS_STAMP(head, k);
    if (__atomic_compare_exchange_n(stp, &v, nv, false, __ATOMIC_ACQ_REL, __ATOMIC_ACQUIRE)) break;
  }
}

void Pool::serve_bundle(Req* rq, int n, int poller, StampAcc* acc) {
  // serving (odd) before any address lookup: see remove_buffer
  ctr().serving.fetch_add(1, std::memory_order_seq_cst);
  const uint64_t t0 = now_ns();
  uint64_t tprev = t0;
  uint64_t calls = 0, merged = 0;
  int i = 0;
  while (i < n) {
    gsys_slot& s = *rq[i].s;
    // counts held back for another group are posted before this request runs
    if (acc && acc->k && acc->head != rq[i].t - s.grp_off) flush_stamp(*acc);
    // Coalesced bundle: fold single pread/pwrite requests that continue the
    // previous one in the file and in memory into one call.
    int j = i + 1;
    if (n > 1 && !(s.flags & GSYS_F_LIST) &&
        (s.nr == GSYS_NR_PREAD64 || s.nr == GSYS_NR_PWRITE64)) {
      uint64_t run = s.args[2];
      while (j < n) {
        const gsys_slot& u = *rq[j].s;
        if ((u.flags & GSYS_F_LIST) || u.nr != s.nr || u.args[0] != s.args[0] ||
            u.args[1] != s.args[1] + run || u.args[3] != s.args[3] + run ||
            run + u.args[2] > (1ull << 30))
          break;
        run += u.args[2];
        ++j;
      }
      const bool regular =
          (int64_t)s.args[0] >= 0 && (int64_t)s.args[0] < (int64_t)fdperm_.size() &&
          (fdperm_[s.args[0]].load(std::memory_order_relaxed) & kRegular);
      if (j > i + 1 && regular) {
        // Field by field: the control word stays out of the copy, since
        // stealing pollers may still be trying to claim it atomically.
        gsys_slot big{};
        big.nr = s.nr;
        big.flags = s.flags;
        big.grp_n = s.grp_n;
        big.grp_off = s.grp_off;
        memcpy(big.args, s.args, sizeof big.args);
        big.args[2] = run;
        int64_t r = execute(big, &calls, &merged);
        merged += (uint64_t)(j - i - 1);
        uint64_t prefix = 0;
        for (int k = i; k < j; ++k) {
          const int64_t lk = (int64_t)rq[k].s->args[2];
          int64_t rk = r < 0 ? r : std::max<int64_t>(0, std::min<int64_t>(lk, r - (int64_t)prefix));
          prefix += (uint64_t)lk;
          note_errno(rk);
          if (ledger_on_) {
            const uint64_t te = now_ns();
            record(poller, {rq[k].t, rq[k].s->nr, (uint64_t)rk,
                            mix64(rq[k].s->args[0] ^ mix64(rq[k].s->args[1] ^ mix64(rq[k].s->args[3]))),
                            tprev, (te << 8) | (uint64_t)(poller & 0xff)});
          }
          complete(rq[k].t, rq[k].s, rk, acc);
        }
        i = j;
        continue;
      }
      j = i + 1;
    }
    int64_t r = execute(s, &calls, &merged);
    if (!(s.flags & GSYS_F_LIST)) note_errno(r);
    if (ledger_on_) {
      const uint64_t te = now_ns();
      record(poller, {rq[i].t, s.nr, (uint64_t)r,
                      mix64(s.args[0] ^ mix64(s.args[1] ^ mix64(s.args[3]))), tprev,
                      (te << 8) | (uint64_t)(poller & 0xff)});
      tprev = te;
    }
    complete(rq[i].t, rq[i].s, r, acc);
    ++i;
  }
  Counters& k = ctr();
  bump(k.requests, (uint64_t)n);
  bump(k.calls, calls);
  bump(k.merged, merged);
  bump(k.bundles, 1);
  bump(k.bhist[hist_bucket((uint64_t)n)], 1);
  bump(k.ns, now_ns() - t0);
  k.serviced.fetch_add((uint64_t)n, std::memory_order_release);
  k.serving.fetch_add(1, std::memory_order_release);
}

// Advance the retire watermark: ticket lo has retired once its slot has been
// freed for a later lap (the ticket in the control word only grows).
void Pool::retire_scan() {
  if (retire_busy_.test_and_set(std::memory_order_acquire)) return;
  uint64_t lo = __atomic_load_n(retired_lo_, __ATOMIC_RELAXED);
  const uint64_t lo0 = lo;
  for (uint64_t k = 0; k < D_; ++k) {
    const uint64_t c = ld_acq(&ring_[lo & (D_ - 1)].ctl);
    if (GSYS_CTL_TICKET(c) < lo + D_) break;
    ++lo;
  }
  if (lo != lo0) st_rel(retired_lo_, lo);
  retire_busy_.clear(std::memory_order_release);
}

// Ticket t's request was taken by a poller (PROCESSING / FINISHED for this
// lap) or has already been freed for a later lap.
static inline bool taken(uint64_t c, uint64_t t) {
  const uint64_t ct = GSYS_CTL_TICKET(c);
  const uint32_t st = GSYS_CTL_STATE(c);
  return ct > t ||
         (ct == t && (st == GSYS_ST_PROCESSING || st == GSYS_ST_FINISHED || st == kQueued));
}

void Pool::poller(int idx) {
  tls_copies_ = &fdcopies_[(size_t)idx];
  tls_ctr_ = ctr_[(size_t)idx].get();
  if (pin_) {
    // poller i runs on allowed CPU number first + i (mod the allowed count)
    const size_t first = first_cpu_ >= 0 ? (size_t)first_cpu_ : 1;
    cpu_set_t set;
    CPU_ZERO(&set);
    CPU_SET(cpus_[(first + (size_t)idx) % cpus_.size()], &set);
    pthread_setaffinity_np(pthread_self(), sizeof set, &set);
  }
  const uint32_t S = stripe_;
  const uint64_t full = S >= 64 ? ~0ull : ((1ull << S) - 1);
  std::vector<Req> rq(S);
  uint64_t s = (uint64_t)idx;
  uint64_t done = 0;
  uint64_t idle = 0;
  uint64_t idle_since = 0;
  bool woken = false;  // back from the doorbell and nothing found yet
  bool napping = false;  // idle longer than kSpinNs (no doorbell)
  // Nothing in this poller's stripe is READY (a peek: nothing is taken).
  auto stripe_quiet = [&]() {
    const uint64_t t0 = s * S;
    for (uint32_t i = 0; i < S; ++i) {
      if ((done >> i) & 1) continue;
      const uint64_t t = t0 + i;
      if (ld_acq(&ring_[t & (D_ - 1)].ctl) == GSYS_CTL(t, GSYS_ST_READY)) return false;
    }
    return true;
  };
  // Serve one READY or QUEUED request of another poller's stripe or of one of
  // the next two unowned stripes; false if there is none.
  auto steal = [&]() {
    auto try_stripe = [&](uint64_t st) {
      if (st == s) return false;
      for (uint32_t i = 0; i < S; ++i) {
        const uint64_t t = st * S + i;
        gsys_slot* sl = &ring_[t & (D_ - 1)];
        uint64_t c = ld_acq(&sl->ctl);
        if (c != GSYS_CTL(t, GSYS_ST_READY) && c != GSYS_CTL(t, kQueued)) continue;
        if (__atomic_compare_exchange_n(&sl->ctl, &c, GSYS_CTL(t, GSYS_ST_PROCESSING), false,
                                        __ATOMIC_ACQ_REL, __ATOMIC_ACQUIRE)) {
          Req r{t, sl};
          serve_bundle(&r, 1, idx);
          return true;
        }
      }
      return false;
    };
    for (int p = 0; p < P_; ++p)
      if (p != idx && try_stripe(owned_[(size_t)p].load(std::memory_order_relaxed))) return true;
    const uint64_t nx = next_stripe_.load(std::memory_order_relaxed);
    return try_stripe(nx) || try_stripe(nx + 1);
  };
  while (!stop_.load(std::memory_order_relaxed)) {
    int n = 0;
    auto scan = [&](void) {
      const uint64_t t0 = s * S;
      for (uint32_t i = 0; i < S && n < (int)S; ++i) {
        if ((done >> i) & 1) continue;
        const uint64_t t = t0 + i;
        gsys_slot* sl = &ring_[t & (D_ - 1)];
        uint64_t c = ld_acq(&sl->ctl);
        if (c != GSYS_CTL(t, GSYS_ST_READY)) {
          if (taken(c, t)) done |= 1ull << i;  // served by another poller
          continue;
        }
        if (__atomic_compare_exchange_n(&sl->ctl, &c, GSYS_CTL(t, kQueued), false,
                                        __ATOMIC_ACQ_REL, __ATOMIC_ACQUIRE)) {
          rq[n++] = Req{t, sl};
          done |= 1ull << i;
        }
      }
    };
    scan();
    if (n && K_ > 1 && done != full && (uint32_t)n < K_ && T_ns_) {
      // coalescing window (section 5): wait for more requests to bundle
      const uint64_t deadline = now_ns() + T_ns_;
      while ((uint32_t)n < K_ && done != full && now_ns() < deadline) {
        _mm_pause();
        scan();
      }
    }
    if (n) {
      woken = false;
      // a queued request is served by whoever moves it to PROCESSING
      auto start = [](const Req& q) {
        uint64_t c = GSYS_CTL(q.t, kQueued);
        return __atomic_compare_exchange_n(&q.s->ctl, &c, GSYS_CTL(q.t, GSYS_ST_PROCESSING), false,
                                           __ATOMIC_ACQ_REL, __ATOMIC_ACQUIRE);
      };
      StampAcc acc;
      if (K_ > 1) {
        // requests in ticket order; bundles of at most K of those still here
        std::sort(rq.begin(), rq.begin() + n, [](const Req& x, const Req& y) { return x.t < y.t; });
        for (int i = 0; i < n; i += (int)K_) {
          const int e = std::min<int>((int)K_, n - i);
          int m = 0;
          for (int k = i; k < i + e; ++k)
            if (start(rq[k])) rq[i + m++] = rq[k];
          if (m) serve_bundle(&rq[i], m, idx, &acc);
        }
      } else {
        for (int i = 0; i < n; ++i)
          if (start(rq[i])) serve_bundle(&rq[i], 1, idx, &acc);
      }
      flush_stamp(acc);
      idle = 0;
      napping = false;
    }
    if (done == full) {
      // the next unowned stripe goes to whichever poller finishes first, so
      // long requests (group calls) spread evenly over the pool
      s = next_stripe_.fetch_add(1, std::memory_order_relaxed);
      owned_[(size_t)idx].store(s, std::memory_order_relaxed);
      done = 0;
      continue;
    }
    if (!n) {
      ++idle;
      bump(ctr().idle, 1);
      if ((idle & 63) == 0) retire_scan();
      if (steal_on_ && (idle & 255) == 0 && steal()) {
        woken = false;
        idle = 0;
        napping = false;
        continue;
      }
      if (idle == 1) idle_since = now_ns();
      if (db_) {
        // A poller woken for a request of another stripe blocks again at
        // once; the idle period applies after real work (bursts).
        if (woken || ((idle & 63) == 0 && now_ns() - idle_since >= db_idle_ns_)) {
          // Sleep protocol.  Read the doorbell, count this poller as a
          // sleeper (sequentially consistent), then look at the stripe once
          // more.  A publisher stores READY, fences, then reads the count:
          // either it sees this poller counted and raises the doorbell
          // (changing the value read here), or its READY store came first
          // and the look below finds the request.
          retire_scan();
          const uint64_t seen = db_->value();
          __atomic_fetch_add(sleepers_, 1, __ATOMIC_SEQ_CST);
          woken = false;
          if (stripe_quiet() && !stop_.load(std::memory_order_relaxed)) {
            db_->wait(seen, db_backstop_ns_);
            bump(ctr().sleeps, 1);
            woken = true;
          }
          __atomic_fetch_sub(sleepers_, 1, __ATOMIC_SEQ_CST);
          idle = 0;
        } else {
          _mm_pause();
        }
      } else {
        if (!napping && (idle & 63) == 0 && now_ns() - idle_since >= kSpinNs) napping = true;
        if (napping) {
          // idle for a while: give the core back in short naps
          timespec ts{0, 20000};
          nanosleep(&ts, nullptr);
        } else {
          _mm_pause();
        }
      }
    }
  }
  // the copies are closed by the thread that used them
  for (FdCopies::Ent& e : fdcopies_[(size_t)idx].e) {
    if (e.fd >= 0) close(e.fd);
    e = FdCopies::Ent{};
  }
  tls_copies_ = nullptr;
  tls_ctr_ = nullptr;
}

uint64_t Pool::poison_outstanding(uint64_t claimed) {
  // runs after the pollers stopped: every request still READY (or taken
  // but never completed) is answered with -ESHUTDOWN so that GPU waiters
  // return instead of waiting for the watchdog
  uint64_t lo = __atomic_load_n(retired_lo_, __ATOMIC_RELAXED);
  uint64_t n = 0;
  for (uint64_t t = lo; t < claimed; ++t) {
    gsys_slot* sl = &ring_[t & (D_ - 1)];
    uint64_t c = ld_acq(&sl->ctl);
    if (c == GSYS_CTL(t, GSYS_ST_READY) || c == GSYS_CTL(t, GSYS_ST_PROCESSING) ||
        c == GSYS_CTL(t, kQueued)) {
      complete(t, sl, -ESHUTDOWN);
      bump(ctr().ehist[5], 1);
      ++n;
    }
  }
  ctr().serviced.fetch_add(n, std::memory_order_release);
  return n;
}

void Pool::stats(gsys_stats* o, int reset) {
  gsys_stats sum;
  memset(&sum, 0, sizeof sum);
  for (auto& cp : ctr_) {
    const Counters& c = *cp;
    auto rd = [](const std::atomic<uint64_t>& a) { return a.load(std::memory_order_relaxed); };
    sum.requests += rd(c.requests);
    sum.host_calls += rd(c.calls);
    sum.bytes_in += rd(c.in);
    sum.bytes_out += rd(c.out);
    sum.errors += rd(c.err);
    sum.rejected += rd(c.rej);
    sum.bundles += rd(c.bundles);
    sum.merged += rd(c.merged);
    sum.idle_polls += rd(c.idle);
    sum.service_ns += rd(c.ns);
    sum.doorbell_sleeps += rd(c.sleeps);
    for (int i = 0; i < 8; ++i) {
      sum.bundle_hist[i] += rd(c.bhist[i]);
      sum.errno_hist[i] += rd(c.ehist[i]);
    }
  }
  // counters only grow: a reset keeps the sums as the new zero
  std::lock_guard<std::mutex> g(stmu_);
  memset(o, 0, sizeof *o);
  o->requests = sum.requests - base_.requests;
  o->host_calls = sum.host_calls - base_.host_calls;
  o->bytes_in = sum.bytes_in - base_.bytes_in;
  o->bytes_out = sum.bytes_out - base_.bytes_out;
  o->errors = sum.errors - base_.errors;
  o->rejected = sum.rejected - base_.rejected;
  o->bundles = sum.bundles - base_.bundles;
  o->merged = sum.merged - base_.merged;
  o->idle_polls = sum.idle_polls - base_.idle_polls;
  o->service_ns = sum.service_ns - base_.service_ns;
  o->doorbell_sleeps = sum.doorbell_sleeps - base_.doorbell_sleeps;
  for (int i = 0; i < 8; ++i) {
    o->bundle_hist[i] = sum.bundle_hist[i] - base_.bundle_hist[i];
    o->errno_hist[i] = sum.errno_hist[i] - base_.errno_hist[i];
  }
  if (reset) base_ = sum;
  o->retired_lo = __atomic_load_n(retired_lo_, __ATOMIC_ACQUIRE);
}

void Pool::record(int poller, const LedgerRec& r) {
  // At most ledger_cap_ records between resets: a shard takes capacity from
  // the shared count 256 records at a time.
  LedgerShard& sh = *ledger_[(size_t)poller];
  std::lock_guard<std::mutex> g(sh.mu);
  const uint64_t ep = ledger_epoch_.load(std::memory_order_acquire);
  if (sh.epoch != ep) {
    sh.epoch = ep;
    sh.quota = 0;
  }
  if (!sh.quota) {
    constexpr uint64_t kBlock = 256;
    const uint64_t got = ledger_n_.fetch_add(kBlock, std::memory_order_relaxed);
    if (got >= ledger_cap_) return;
    sh.quota = std::min<uint64_t>(kBlock, ledger_cap_ - got);
  }
  --sh.quota;
  sh.recs.push_back(r);
}

int64_t Pool::ledger(uint64_t* out, uint64_t max, int reset) {
  std::vector<LedgerRec> v;
  for (auto& sh : ledger_) {
    std::lock_guard<std::mutex> g(sh->mu);
    v.insert(v.end(), sh->recs.begin(), sh->recs.end());
    if (reset) sh->recs.clear();
  }
  if (reset) {
    // a shard notices the new epoch (under its lock) and drops its quota
    ledger_epoch_.fetch_add(1, std::memory_order_acq_rel);
    ledger_n_.store(0, std::memory_order_relaxed);
  }
  std::sort(v.begin(), v.end(), [](const LedgerRec& x, const LedgerRec& y) { return x.ticket < y.ticket; });
  const uint64_t n = std::min<uint64_t>(max, v.size());
  if (out) {
    for (uint64_t i = 0; i < n; ++i) {
      out[6 * i] = v[i].ticket;
      out[6 * i + 1] = v[i].nr;
      out[6 * i + 2] = v[i].ret;
      out[6 * i + 3] = v[i].digest;
      out[6 * i + 4] = v[i].t_start;
      out[6 * i + 5] = v[i].t_end_poller;
    }
  }
  return (int64_t)n;
}

}  // namespace gsys_host
