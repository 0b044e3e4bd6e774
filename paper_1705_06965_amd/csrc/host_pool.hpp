// Host service pool: the CPU side that executes GPU-issued system calls.
//
// The paper dispatches each request from a GPU interrupt to a kernel
// work-queue task that scans the requesting wavefront's slots, moves every
// ready slot to processing, executes the call and writes the result back
// (section 5).  Here P pinned user-space threads poll the slot ring instead
// (section 3 treats interrupts versus polling as orthogonal; section 9 names
// the user-mode service thread of earlier GPU file and network systems).
// Tickets are dealt to pollers in stripes of `stripe` consecutive tickets;
// a poller that has serviced every ticket of its stripe takes the next
// unowned stripe.  A wavefront's 64 work-item calls are thus serviced by
// several threads at once, long group calls spread evenly over the pool, and
// a kernel-granularity call is one unit of work for one thread (section 6,
// Fig. 5).
//
// Exactly-once: a poller takes a request only by compare-and-swap of the
// slot's control word from READY to PROCESSING (section 5).
//
// Work stealing: an owner's scan moves every READY request of its stripe to
// QUEUED, a host-only state (the GPU never looks at it), and serves them one
// after another, moving each to PROCESSING first.  A poller that has found
// nothing to do for a while serves a READY or QUEUED request of another
// poller's stripe (or of the next unowned stripes) the same way, so a short
// call never waits behind the long calls queued ahead of it.  Whoever moves a
// request to PROCESSING serves it; an owner skips a queued request that was
// taken, and counts a request of its stripe that is no longer READY for this
// lap as done.  GSYS_STEAL=0 in the environment turns stealing off.
//
// Nothing a poller writes per request is shared with another poller but the
// request's own slot and completion record: statistics and ledger records
// go to per-poller blocks, and a poller serving several members of one
// claim group in a row counts them in the group's record with one update.
//
// Coalescing (section 4.2, section 5): with K > 1 a poller that finds a ready
// request waits up to T ns for more ready requests of its stripe, up to K,
// and executes them as one bundle, folding transfers that are adjacent both
// in the file and in memory into one call.
#pragma once

#include <atomic>
#include <cstdint>
#include <memory>
#include <mutex>
#include <thread>
#include <vector>

#include "gsys.h"

namespace gsys_host {

struct Buf {
  uint64_t dev;
  uint8_t* host;
  uint64_t bytes;
  uint32_t kind;
  uint32_t id;
};

// A registered buffer's slot in the table.  Pollers read it without the
// table's mutex, under the generation seqlock, so every field is an atomic
// read and written with relaxed order (the generation orders them).
struct BufSlot {
  std::atomic<uint64_t> dev{0}, host{0}, bytes{0};
  std::atomic<uint32_t> kind{0}, id{0};
  Buf load() const {
    return Buf{dev.load(std::memory_order_relaxed),
               reinterpret_cast<uint8_t*>(host.load(std::memory_order_relaxed)),
               bytes.load(std::memory_order_relaxed), kind.load(std::memory_order_relaxed),
               id.load(std::memory_order_relaxed)};
  }
  void store(const Buf& b) {
    dev.store(b.dev, std::memory_order_relaxed);
    host.store(reinterpret_cast<uint64_t>(b.host), std::memory_order_relaxed);
    bytes.store(b.bytes, std::memory_order_relaxed);
    kind.store(b.kind, std::memory_order_relaxed);
    id.store(b.id, std::memory_order_relaxed);
  }
};

// How an idle poller blocks until the GPU announces new requests (an HSA
// interrupt signal on a device context, a condition variable in CPU-only
// contexts).  Every publisher that sees a non-zero sleeper count after its
// READY store raises the doorbell, which stores a value never stored before.
class Doorbell {
 public:
  virtual ~Doorbell() = default;
  virtual uint64_t value() = 0;
  // return once the value differs from `seen` or `timeout_ns` has passed
  virtual void wait(uint64_t seen, uint64_t timeout_ns) = 0;
  // raise it from the host (wakes every blocked poller)
  virtual void ring() = 0;
};

struct LedgerRec {
  uint64_t ticket, nr, ret, digest, t_start, t_end_poller;  // t_end << 8 | poller
};

class Pool {
 public:
  // Memory is owned by the caller (the C-ABI layer).
  Pool(gsys_slot* ring, gsys_comp* comp, uint64_t D, uint64_t C, uint64_t* retired_lo,
       const gsys_config& cfg);
  ~Pool();
  void start();
  void stop_and_join();

  // whitelist
  int allow_fd(int fd, uint32_t perms);
  // Close every fd a GPU openat opened and is still open (after the pollers
  // stopped).
  void close_owned();
  int add_buffer(uint64_t dev, uint8_t* host, uint64_t bytes, uint32_t kind, uint32_t* id);
  // Drop a registration.  Returns once no service thread can still use the
  // buffer: every poller that was serving requests when the entry went away
  // has finished them (later requests no longer find it).
  int remove_buffer(uint32_t id);
  void set_arena(uint8_t* base, uint64_t bytes) { arena_ = base; arena_bytes_ = bytes; }
  // Answer the next `count` single requests of call `nr` with -err.
  void inject(uint16_t nr, int32_t err, uint32_t count) {
    inj_nr_.store(nr, std::memory_order_relaxed);
    inj_err_.store(err, std::memory_order_relaxed);
    inj_left_.store(count, std::memory_order_release);
  }
  // Before start(): idle pollers count themselves in *sleepers (a word the
  // publishers can read) and block on `db`; `idle_ns` of finding nothing
  // comes first, `backstop_ns` bounds each block.
  void set_doorbell(Doorbell* db, uint64_t* sleepers, uint64_t idle_ns, uint64_t backstop_ns) {
    db_ = db;
    sleepers_ = sleepers;
    db_idle_ns_ = idle_ns;
    db_backstop_ns_ = backstop_ns;
  }

  // servicing
  // requests completed so far (each completion is visible to the caller)
  uint64_t serviced() const {
    uint64_t n = 0;
    for (const auto& c : ctr_) n += c->serviced.load(std::memory_order_acquire);
    return n;
  }
  // Complete every request still READY with -ESHUTDOWN (called after the
  // pollers stopped).  `claimed` bounds the tickets examined.
  uint64_t poison_outstanding(uint64_t claimed);
  void retire_scan();

  // true if [dev, dev + len) lies inside one registered host buffer
  bool host_range(uint64_t dev, uint64_t len) { return translate(dev, len, false) != nullptr; }

  void stats(gsys_stats* out, int reset);
  int64_t ledger(uint64_t* out, uint64_t max, int reset);

 private:
  struct Req {
    uint64_t t;
    gsys_slot* s;
  };
  // Completions of one claim group that a poller has posted but not yet
  // counted in the group's completion record.  A group is done only when all
  // its members are, so a poller that serves several members in a row counts
  // them with one update of the shared record instead of one each.
  struct StampAcc {
    uint64_t head = ~0ull;
    uint32_t k = 0;
  };
  void poller(int idx);
  void serve_bundle(Req* rq, int n, int poller, StampAcc* acc = nullptr);
  int64_t execute(const gsys_slot& s, uint64_t* calls, uint64_t* merged);
  int64_t exec_list(const gsys_slot& s, uint64_t* calls, uint64_t* merged);
  // Post one request's result; its group count goes to *acc (flushed when
  // the group changes) or, without acc, straight to the completion record.
  void complete(uint64_t t, gsys_slot* s, int64_t ret, StampAcc* acc = nullptr);
  void add_stamp(uint64_t head, uint32_t k);
  void flush_stamp(StampAcc& acc) {
    if (acc.k) add_stamp(acc.head, acc.k);
    acc.k = 0;
  }
  void record(int poller, const LedgerRec& r);
  uint8_t* translate(uint64_t dev, uint64_t len, bool need_host_write);
  bool fd_ok(int64_t fd, uint32_t need) const;
  // The descriptor a positional call on regular file `fd` should use: this
  // poller's own open file description of it (see FdCopies), or `fd`.
  int fd_for(int64_t fd);
  void note_errno(int64_t ret);

  gsys_slot* ring_;
  gsys_comp* comp_;
  uint64_t D_, C_;
  uint64_t* retired_lo_;
  int P_;
  uint32_t stripe_, K_, T_ns_;
  int first_cpu_;
  std::vector<int> cpus_;  // CPUs in this process's affinity mask, ascending
  bool pin_;
  bool ledger_on_;
  uint64_t ledger_cap_;

  std::vector<std::thread> threads_;
  std::atomic<bool> stop_{false};
  std::atomic<uint64_t> next_stripe_{0};  // stripes are taken in order by whichever poller is free
  std::vector<std::atomic<uint64_t>> owned_;  // each poller's current stripe (for stealing)
  std::atomic_flag retire_busy_ = ATOMIC_FLAG_INIT;

  std::vector<std::atomic<uint8_t>> fdperm_;
  // Bumped by every allow_fd on an fd number: a poller's copy made under an
  // older generation is re-opened before use.
  std::vector<std::atomic<uint32_t>> fdgen_;
  bool copy_fds_ = true;

 public:
  // A poller's private open file descriptions of allowed regular files.
  // Many threads calling pread on one description all update its reference
  // count in the kernel; with one description per thread the host's pread
  // rate rose from ~10 M/s to ~16 M/s (15 threads, 4 KiB, tmpfs).
  struct FdCopies {
    struct Ent {
      int src = -1;
      uint32_t gen = 0;
      int fd = -1;  // -1: re-opening failed, the caller's fd is used
    };
    static constexpr int kEnts = 8;
    Ent e[kEnts];
    uint32_t next = 0;
  };

 private:
  std::vector<FdCopies> fdcopies_;
  static thread_local FdCopies* tls_copies_;

  // buffer table: seqlock-protected fixed array
  static constexpr int kMaxBufs = 512;
  BufSlot bufs_[kMaxBufs];
  std::atomic<int> nbufs_{0};
  std::atomic<uint64_t> bufgen_{0};
  std::mutex bufmu_;
  uint32_t next_id_ = 1;

  uint8_t* arena_ = nullptr;
  uint64_t arena_bytes_ = 0;
  bool arena_huge_ = true;  // hint MADV_HUGEPAGE on 2 MiB-aligned arena mappings
  bool steal_on_ = true;    // idle pollers serve other stripes' requests

  // fault injection (test hook)
  std::atomic<uint32_t> inj_left_{0};
  std::atomic<uint32_t> inj_nr_{0};
  std::atomic<int32_t> inj_err_{0};

  Doorbell* db_ = nullptr;
  uint64_t* sleepers_ = nullptr;
  uint64_t db_idle_ns_ = 0, db_backstop_ns_ = 0;

  // Statistics: one block of counters per poller (only that poller writes
  // it) and one for every other thread; stats() sums them.  Pollers never
  // write a cache line another poller writes: shared counters cost each
  // request several contended read-modify-writes.
  struct alignas(64) Counters {
    std::atomic<uint64_t> requests{0}, calls{0}, in{0}, out{0}, err{0}, rej{0}, bundles{0},
        merged{0}, idle{0}, ns{0}, sleeps{0};
    std::atomic<uint64_t> serviced{0};  // completed requests, release-incremented
    // odd while this poller serves requests (it may hold host addresses of
    // registered buffers); remove_buffer waits for it to move on
    std::atomic<uint64_t> serving{0};
    std::atomic<uint64_t> bhist[8] = {}, ehist[8] = {};
  };
  std::vector<std::unique_ptr<Counters>> ctr_;  // P pollers, then the others
  static thread_local Counters* tls_ctr_;
  Counters& ctr() { return tls_ctr_ ? *tls_ctr_ : *ctr_.back(); }
  static void bump(std::atomic<uint64_t>& a, uint64_t v) { a.fetch_add(v, std::memory_order_relaxed); }
  std::mutex stmu_;
  gsys_stats base_{};  // sums at the last reset

  // The ledger in one shard per poller: a poller appends to its own shard
  // under that shard's lock, which only the reader also takes, so recording
  // does not make the pollers wait for each other.
  struct alignas(64) LedgerShard {
    std::mutex mu;
    std::vector<LedgerRec> recs;
    uint64_t quota = 0;  // records this shard may still add
    uint64_t epoch = 0;  // reset generation the quota belongs to
  };
  std::vector<std::unique_ptr<LedgerShard>> ledger_;
  // capacity handed out to the shards in blocks (since the last reset)
  std::atomic<uint64_t> ledger_n_{0};
  std::atomic<uint64_t> ledger_epoch_{0};
};

}  // namespace gsys_host
