// C ABI of libgsys.so: context set-up and tear-down, whitelist registration,
// launches and the drain call.  See include/gsys.h for the contract.
#include <errno.h>
#include <linux/futex.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#include <stdio.h>
#include <sys/mman.h>
#include <sys/syscall.h>
#include <time.h>
#include <unistd.h>

#include <hip/hip_runtime.h>
#include <hsa/amd_hsa_signal.h>
#include <hsa/hsa.h>
#include <hsa/hsa_ext_amd.h>

#include <algorithm>
#include <atomic>
#include <map>
#include <mutex>
#include <thread>
#include <vector>

#include "gsys.h"
#include "host_pool.hpp"
#include "kernels.hpp"
#include "testing_access.hpp"

namespace {

// Pollers block on a futex word.  In CPU-only contexts the emulated callers
// raise it directly; device contexts put a relay thread in front of it.
class FutexDoorbell : public gsys_host::Doorbell {
 public:
  uint64_t value() override { return v_.load(std::memory_order_acquire); }
  void wait(uint64_t seen, uint64_t timeout_ns) override {
    // the kernel blocks only while the word still holds `seen`
    timespec ts{(time_t)(timeout_ns / 1000000000ull), (long)(timeout_ns % 1000000000ull)};
    syscall(SYS_futex, reinterpret_cast<uint32_t*>(&v_), FUTEX_WAIT_PRIVATE, (uint32_t)seen, &ts,
            nullptr, 0);
  }
  void ring() override {
    v_.fetch_add(1, std::memory_order_acq_rel);
    syscall(SYS_futex, reinterpret_cast<uint32_t*>(&v_), FUTEX_WAKE_PRIVATE, INT32_MAX, nullptr,
            nullptr, 0);
  }

 private:
  std::atomic<uint32_t> v_{0};
  static_assert(sizeof(std::atomic<uint32_t>) == 4, "futex word");
};

// Device contexts: the GPU raises an HSA interrupt signal (it stores
// ticket + 1 into it; the host's own values have bit 62 set, so no value
// repeats).  One relay thread waits on the signal and raises the pollers'
// futex word: the runtime's wait polls for a while before it blocks, and
// that cost is paid by one thread instead of by every poller.  The relay
// reads the signal's new value before it raises the word, so a poller that
// read the word after a raise is covered by the relay's next wait.
class HsaDoorbell final : public FutexDoorbell {
 public:
  HsaDoorbell(hsa_signal_t s, uint64_t ticks_per_s) : s_(s), hz_(ticks_per_s) {
    relay_ = std::thread([this] { relay(); });
  }
  ~HsaDoorbell() override {
    stop_.store(true, std::memory_order_release);
    hsa_signal_store_screlease(s_, (hsa_signal_value_t)((1ull << 62) | ++n_));
    relay_.join();
  }

 private:
  void relay() {
    hsa_signal_value_t v = hsa_signal_load_scacquire(s_);
    while (!stop_.load(std::memory_order_acquire)) {
      hsa_signal_wait_scacquire(s_, HSA_SIGNAL_CONDITION_NE, v, hz_ / 10 /* 100 ms */,
                                HSA_WAIT_STATE_BLOCKED);
      const hsa_signal_value_t nv = hsa_signal_load_scacquire(s_);
      if (nv != v) {
        v = nv;
        ring();
      }
    }
  }
  hsa_signal_t s_;
  uint64_t hz_;
  std::atomic<uint64_t> n_{0};
  std::atomic<bool> stop_{false};
  std::thread relay_;
};

}  // namespace

struct gsys_ctx {
  gsys_config cfg;
  bool no_device = false;
  int device = 0;
  uint64_t D = 0, C = 0;
  gsys_slot* ring = nullptr;       // host view
  gsys_comp* comp = nullptr;       // host view
  // host-coherent page: [0] retired_lo, [32] the ticket counter of NO_DEVICE
  // contexts, [64] sleeping pollers, [96..97] serving control words; each
  // group on its own 256-byte line
  uint64_t* host_words = nullptr;
  gsys_slot* ring_dev = nullptr;
  gsys_comp* comp_dev = nullptr;
  uint64_t* retired_lo_dev = nullptr;
  unsigned long long* dev_words = nullptr;  // [0] tail, [32..63] kernel-call state
  // kernel-granularity call sites of user kernels (gsys_launch clears them)
  unsigned long long* ksites = nullptr;
  gsys_host::Pool* pool = nullptr;
  hipStream_t aux = nullptr;
  std::mutex mu;
  std::map<void*, std::pair<uint64_t, uint32_t>> host_allocs;  // host ptr -> (bytes, id)
  uint8_t* arena = nullptr;
  uint64_t arena_bytes = 0;
  uint64_t timeout_ticks = 0;
  uint64_t wall_khz = 100000;
  uint32_t sleep_max = 16;
  uint32_t grid_override = 0;
  int cu_count = 0;
  // graph forms: per key, an instantiated chain of kernel nodes
  struct Graph {
    hipGraph_t graph;
    hipGraphExec_t exec;
    std::vector<hipGraphNode_t> nodes;
  };
  std::map<uint64_t, Graph> graphs;
  // doorbell (GSYS_CFG_DOORBELL)
  gsys_host::Doorbell* db = nullptr;
  uint64_t* sleepers_dev = nullptr;  // host_words[64] as the GPU sees it
  bool hsa_up = false;
  bool sig_live = false;
  hsa_signal_t sig{0};
};

namespace {

uint64_t now_ns() {
  timespec ts;
  clock_gettime(CLOCK_MONOTONIC, &ts);
  return (uint64_t)ts.tv_sec * 1000000000ull + (uint64_t)ts.tv_nsec;
}

uint64_t env_u64(const char* name, uint64_t dflt) {
  const char* v = getenv(name);
  if (!v || !*v) return dflt;
  return strtoull(v, nullptr, 0);
}

bool is_pow2(uint64_t x) { return x && !(x & (x - 1)); }

// fine-grained, host-coherent pinned memory visible to the GPU
int host_coherent(gsys_ctx* c, uint64_t bytes, void** host, void** dev) {
  if (c->no_device) {
    void* p = nullptr;
    if (posix_memalign(&p, 4096, bytes)) return -ENOMEM;
    memset(p, 0, bytes);
    *host = p;
    *dev = p;
    return 0;
  }
  void* p = nullptr;
  if (hipHostMalloc(&p, bytes, hipHostMallocCoherent | hipHostMallocMapped | hipHostMallocPortable) !=
      hipSuccess)
    return -ENOMEM;
  void* d = nullptr;
  if (hipHostGetDevicePointer(&d, p, 0) != hipSuccess) {
    hipHostFree(p);
    return -ENODEV;
  }
  memset(p, 0, bytes);
  *host = p;
  *dev = d;
  return 0;
}

void host_coherent_free(gsys_ctx* c, void* host) {
  if (!host) return;
  if (c->no_device) free(host);
  else hipHostFree(host);
}

uint64_t claimed_tickets(gsys_ctx* c) {
  if (c->no_device) return __atomic_load_n(&c->host_words[32], __ATOMIC_ACQUIRE);
  unsigned long long v = 0;
  hipSetDevice(c->device);
  if (hipMemcpyAsync(&v, c->dev_words, sizeof v, hipMemcpyDeviceToHost, c->aux) != hipSuccess)
    return 0;
  hipStreamSynchronize(c->aux);
  return v;
}

// The HIP device's HSA agent (matched by PCI location).
struct AgentFind {
  uint32_t bdf, domain;
  hsa_agent_t agent;
  bool found;
};

hsa_status_t find_agent(hsa_agent_t a, void* data) {
  AgentFind* f = (AgentFind*)data;
  hsa_device_type_t t;
  if (hsa_agent_get_info(a, HSA_AGENT_INFO_DEVICE, &t) != HSA_STATUS_SUCCESS ||
      t != HSA_DEVICE_TYPE_GPU)
    return HSA_STATUS_SUCCESS;
  uint32_t bdf = ~0u, dom = ~0u;
  hsa_agent_get_info(a, (hsa_agent_info_t)HSA_AMD_AGENT_INFO_BDFID, &bdf);
  hsa_agent_get_info(a, (hsa_agent_info_t)HSA_AMD_AGENT_INFO_DOMAIN, &dom);
  if (bdf == f->bdf && dom == f->domain) {
    f->agent = a;
    f->found = true;
    return HSA_STATUS_INFO_BREAK;
  }
  return HSA_STATUS_SUCCESS;
}

// true if the runtime reports [p, p + len) inside one allocation that
// `agent` may access at the same address the host uses
bool gpu_maps(hsa_agent_t agent, const void* p, uint64_t len) {
  hsa_amd_pointer_info_t pi;
  memset(&pi, 0, sizeof pi);
  pi.size = sizeof pi;
  uint32_t n = 0;
  hsa_agent_t* acc = nullptr;
  if (hsa_amd_pointer_info(p, &pi, malloc, &n, &acc) != HSA_STATUS_SUCCESS) return false;
  bool ok = false;
  for (uint32_t i = 0; i < n; ++i) ok = ok || acc[i].handle == agent.handle;
  free(acc);
  const uint64_t base = (uint64_t)pi.agentBaseAddress, a = (uint64_t)p;
  return ok && pi.sizeInBytes && pi.agentBaseAddress == pi.hostBaseAddress && a >= base &&
         a + len <= base + pi.sizeInBytes;
}

// An interrupt signal whose block and event mailbox this GPU may write.
int make_hsa_doorbell(gsys_ctx* c, const hipDeviceProp_t& prop) {
  if (hsa_init() != HSA_STATUS_SUCCESS) return -ENOTSUP;
  c->hsa_up = true;
  AgentFind f{((uint32_t)prop.pciBusID << 8) | ((uint32_t)prop.pciDeviceID << 3),
              (uint32_t)prop.pciDomainID, hsa_agent_t{0}, false};
  hsa_iterate_agents(find_agent, &f);
  uint64_t hz = 0;
  if (!f.found || hsa_system_get_info(HSA_SYSTEM_INFO_TIMESTAMP_FREQUENCY, &hz) != HSA_STATUS_SUCCESS ||
      !hz)
    return -ENOTSUP;
  if (hsa_signal_create(0, 0, nullptr, &c->sig) != HSA_STATUS_SUCCESS) return -ENOTSUP;
  c->sig_live = true;
  const amd_signal_t* s = (const amd_signal_t*)c->sig.handle;
  if (s->kind != AMD_SIGNAL_KIND_USER || !s->event_mailbox_ptr || !gpu_maps(f.agent, s, sizeof *s) ||
      !gpu_maps(f.agent, (const void*)s->event_mailbox_ptr, sizeof(uint64_t)))
    return -ENOTSUP;
  c->db = new (std::nothrow) HsaDoorbell(c->sig, hz);
  return c->db ? 0 : -ENOMEM;
}

void destroy(gsys_ctx* c) {
  if (!c) return;
  if (c->pool) {
    c->pool->stop_and_join();
    c->pool->close_owned();
    delete c->pool;
    c->pool = nullptr;
  }
  delete c->db;
  c->db = nullptr;
  if (c->sig_live) hsa_signal_destroy(c->sig);
  if (c->hsa_up) hsa_shut_down();
  if (!c->no_device) {
    hipSetDevice(c->device);
    for (auto& g : c->graphs) {
      hipGraphExecDestroy(g.second.exec);
      hipGraphDestroy(g.second.graph);
    }
    if (c->aux) hipStreamDestroy(c->aux);
    if (c->dev_words) hipFree(c->dev_words);
    if (c->ksites) hipFree(c->ksites);
  }
  for (auto& kv : c->host_allocs) host_coherent_free(c, kv.first);
  c->host_allocs.clear();
  host_coherent_free(c, c->ring);
  host_coherent_free(c, c->comp);
  host_coherent_free(c, c->host_words);
  if (c->arena) munmap(c->arena, c->arena_bytes);
  delete c;
}

}  // namespace

extern "C" {

int gsys_init(const gsys_config* cfg_in, gsys_ctx** out) {
  if (!out) return -EINVAL;
  *out = nullptr;
  gsys_config cfg;
  memset(&cfg, 0, sizeof cfg);
  cfg.abi_version = GSYS_ABI_VERSION;
  cfg.first_cpu = -1;
  if (cfg_in) cfg = *cfg_in;
  if (cfg.abi_version != GSYS_ABI_VERSION) return -EINVAL;
  // environment overrides (the autotuner writes these)
  cfg.ring_slots = (uint32_t)env_u64("GSYS_RING_SLOTS", cfg.ring_slots);
  cfg.service_threads = (uint32_t)env_u64("GSYS_SERVICE_THREADS", cfg.service_threads);
  cfg.coalesce_max = (uint32_t)env_u64("GSYS_COALESCE_MAX", cfg.coalesce_max);
  cfg.coalesce_window_ns = (uint32_t)env_u64("GSYS_COALESCE_WINDOW_NS", cfg.coalesce_window_ns);
  cfg.stripe = (uint32_t)env_u64("GSYS_STRIPE", cfg.stripe);
  if (!cfg.ring_slots) cfg.ring_slots = 65536;
  if (!is_pow2(cfg.ring_slots) || cfg.ring_slots < 64 || cfg.ring_slots > (1u << 24)) return -EINVAL;
  if (cfg.stripe > 64) return -EINVAL;

  gsys_ctx* c = new (std::nothrow) gsys_ctx;
  if (!c) return -ENOMEM;
  c->cfg = cfg;
  c->no_device = (cfg.flags & GSYS_CFG_NO_DEVICE) != 0;
  c->device = cfg.device;
  c->D = cfg.ring_slots;
  // completion records: 4D, and at least 65,536 (1 MiB), so that a small
  // ring still keeps a non-blocking call's result for the next 65,535
  // tickets (a later lap of its record makes the device wait report
  // -EOVERFLOW)
  c->C = std::max<uint64_t>(4ull * c->D, 65536ull);
  c->grid_override = (uint32_t)env_u64("GSYS_PERSISTENT_GRID", 0);
  c->sleep_max = (uint32_t)env_u64("GSYS_SLEEP_MAX", cfg.sleep_max ? cfg.sleep_max : 64);
  const uint64_t tmo = cfg.device_timeout_ns ? cfg.device_timeout_ns : 30000000000ull;
  c->timeout_ticks = tmo / 10;  // 100 MHz device wall clock

  if (!c->no_device) {
    if (hipSetDevice(c->device) != hipSuccess) {
      destroy(c);
      return -ENODEV;
    }
    hipDeviceProp_t prop;
    if (hipGetDeviceProperties(&prop, c->device) != hipSuccess) {
      destroy(c);
      return -ENODEV;
    }
    c->cu_count = prop.multiProcessorCount;
    // the allocation-free serving entry point's scratch on this device
    if (int e = gsys_internal::serve_scratch_setup ? gsys_internal::serve_scratch_setup(c->device)
                                                   : -ENODEV) {
      destroy(c);
      return e;
    }
    int wall_khz = 0;
    if (hipDeviceGetAttribute(&wall_khz, hipDeviceAttributeWallClockRate, c->device) == hipSuccess &&
        wall_khz > 0) {
      c->timeout_ticks = (uint64_t)((double)tmo * 1e-9 * (double)wall_khz * 1e3);
      c->wall_khz = (uint64_t)wall_khz;
    }
    if (hipStreamCreateWithFlags(&c->aux, hipStreamNonBlocking) != hipSuccess ||
        hipMalloc((void**)&c->dev_words, 64 * sizeof(unsigned long long)) != hipSuccess ||
        hipMemset(c->dev_words, 0, 64 * sizeof(unsigned long long)) != hipSuccess ||
        hipMalloc((void**)&c->ksites, gsys_internal::kSites * 16) != hipSuccess ||
        hipMemset(c->ksites, 0, gsys_internal::kSites * 16) != hipSuccess ||
        hipDeviceSynchronize() != hipSuccess) {
      destroy(c);
      return -ENODEV;
    }
  }
  void *rh, *rd, *ch, *cd, *wh, *wd;
  int e;
  if ((e = host_coherent(c, c->D * sizeof(gsys_slot), &rh, &rd)) ||
      (c->ring = (gsys_slot*)rh, c->ring_dev = (gsys_slot*)rd, false) ||
      (e = host_coherent(c, c->C * sizeof(gsys_comp), &ch, &cd)) ||
      (c->comp = (gsys_comp*)ch, c->comp_dev = (gsys_comp*)cd, false) ||
      (e = host_coherent(c, 4096, &wh, &wd))) {
    destroy(c);
    return e;
  }
  c->host_words = (uint64_t*)wh;
  c->retired_lo_dev = (uint64_t*)wd;
  c->sleepers_dev = (uint64_t*)wd + 64;
  if (cfg.flags & GSYS_CFG_DOORBELL) {
    if (c->no_device) {
      c->db = new (std::nothrow) FutexDoorbell;
      e = c->db ? 0 : -ENOMEM;
    } else {
      hipDeviceProp_t prop;
      e = hipGetDeviceProperties(&prop, c->device) == hipSuccess ? make_hsa_doorbell(c, prop) : -ENODEV;
    }
    if (e) {
      destroy(c);
      return e;
    }
  }
  for (uint64_t i = 0; i < c->D; ++i) c->ring[i].ctl = GSYS_CTL(i, GSYS_ST_FREE);
  if (cfg.arena_bytes) {
    const uint64_t bytes = (cfg.arena_bytes + (2u << 20) - 1) & ~((2ull << 20) - 1);
    // reserve, 2 MiB aligned
    void* m = mmap(nullptr, bytes + (2u << 20), PROT_NONE,
                   MAP_PRIVATE | MAP_ANONYMOUS | MAP_NORESERVE, -1, 0);
    if (m == MAP_FAILED) {
      destroy(c);
      return -ENOMEM;
    }
    uint8_t* a = (uint8_t*)(((uint64_t)m + (2u << 20) - 1) & ~((2ull << 20) - 1));
    if (a != m) munmap(m, (size_t)(a - (uint8_t*)m));
    munmap(a + bytes, (size_t)(((uint8_t*)m + bytes + (2u << 20)) - (a + bytes)));
    c->arena = a;
    c->arena_bytes = bytes;
  }
  __atomic_thread_fence(__ATOMIC_SEQ_CST);
  c->pool = new (std::nothrow) gsys_host::Pool(c->ring, c->comp, c->D, c->C, c->host_words, cfg);
  if (!c->pool) {
    destroy(c);
    return -ENOMEM;
  }
  if (c->arena) c->pool->set_arena(c->arena, c->arena_bytes);
  if (c->db) {
    const uint64_t idle_us =
        env_u64("GSYS_DOORBELL_IDLE_US", cfg.doorbell_idle_us ? cfg.doorbell_idle_us : 200);
    // each block lasts 50 ms at most: a backstop only, the doorbell wakes
    // first (tests raise it so that a lost wake-up shows as a time-out)
    const uint64_t backstop_us = env_u64("GSYS_DOORBELL_BACKSTOP_US", 50000);
    c->pool->set_doorbell(c->db, &c->host_words[64], idle_us * 1000, backstop_us * 1000);
  }
  c->pool->start();
  *out = c;
  return 0;
}

int gsys_allow_fd(gsys_ctx* c, int fd, uint32_t perms) {
  if (!c) return -EINVAL;
  return c->pool->allow_fd(fd, perms);
}

int gsys_register_buffer(gsys_ctx* c, uint64_t dev, void* host, uint64_t bytes, uint32_t kind,
                         uint32_t* out_id) {
  if (!c) return -EINVAL;
  return c->pool->add_buffer(dev, (uint8_t*)host, bytes, kind, out_id);
}

// Outstanding tickets may still reference any buffer: claimed tickets that
// the pool has not all serviced after a short wait make a removal -EBUSY.
static int quiet_for_removal(gsys_ctx* c) {
  return gsys_wait(c, 10000000) ? -EBUSY : 0;
}

int gsys_unregister_buffer(gsys_ctx* c, uint32_t id) {
  if (!c) return -EINVAL;
  if (int e = quiet_for_removal(c)) return e;
  return c->pool->remove_buffer(id);
}

int gsys_host_alloc(gsys_ctx* c, uint64_t bytes, void** host_out, uint64_t* dev_out,
                    uint32_t* id_out) {
  if (!c || !bytes || !host_out || !dev_out) return -EINVAL;
  if (!c->no_device) hipSetDevice(c->device);
  void *h, *d;
  if (int e = host_coherent(c, bytes, &h, &d)) return e;
  uint32_t id = 0;
  if (int e = c->pool->add_buffer((uint64_t)d, (uint8_t*)h, bytes, GSYS_BUF_HOST, &id)) {
    host_coherent_free(c, h);
    return e;
  }
  {
    std::lock_guard<std::mutex> g(c->mu);
    c->host_allocs[h] = {bytes, id};
  }
  *host_out = h;
  *dev_out = (uint64_t)d;
  if (id_out) *id_out = id;
  return 0;
}

int gsys_host_free(gsys_ctx* c, void* host) {
  if (!c) return -EINVAL;
  std::lock_guard<std::mutex> g(c->mu);
  auto it = c->host_allocs.find(host);
  if (it == c->host_allocs.end()) return -ENOENT;
  if (int e = quiet_for_removal(c)) return e;
  // the memory is freed only after no service thread can still use it
  if (int e = c->pool->remove_buffer(it->second.second)) return e;
  host_coherent_free(c, host);
  c->host_allocs.erase(it);
  return 0;
}

int gsys_device_ctx(gsys_ctx* c, gsys_dev_ctx* out) {
  if (!c || !out) return -EINVAL;
  memset(out, 0, sizeof *out);
  out->ring = c->ring_dev;
  out->comp = c->comp_dev;
  out->tail = c->no_device ? (unsigned long long*)&c->host_words[32] : c->dev_words;
  out->retired_lo = c->retired_lo_dev;
  out->ring_mask = c->D - 1;
  out->comp_mask = c->C - 1;
  out->timeout_ticks = c->timeout_ticks;
  out->sleep_max = c->sleep_max;
  out->flags = c->cfg.flags;
  out->arena = (uint64_t)c->arena;
  out->arena_bytes = c->arena_bytes;
  if (c->ksites) {
    out->ksites = (uint64_t)c->ksites;
    out->n_ksites = gsys_internal::kSites;
  }
  if (c->db) {
    // CPU-only contexts: any non-zero value; the emulated callers ring c->db
    out->doorbell = c->no_device ? 1 : c->sig.handle;
    out->sleepers = c->sleepers_dev;
  }
  return 0;
}

int gsys_wait(gsys_ctx* c, uint64_t timeout_ns) {
  if (!c) return -EINVAL;
  const uint64_t want = claimed_tickets(c);
  const uint64_t t0 = now_ns();
  uint32_t spins = 0;
  while (c->pool->serviced() < want) {
    if (timeout_ns && now_ns() - t0 > timeout_ns) return -ETIMEDOUT;
    if (++spins < 1000) {
      std::this_thread::yield();
    } else {
      timespec ts{0, 20000};
      nanosleep(&ts, nullptr);
    }
  }
  c->pool->retire_scan();
  return 0;
}

int gsys_stats_get(gsys_ctx* c, gsys_stats* out, int reset) {
  if (!c || !out) return -EINVAL;
  c->pool->stats(out, reset);
  out->claimed = claimed_tickets(c);
  return 0;
}

int64_t gsys_ledger(gsys_ctx* c, uint64_t* out, uint64_t max, int reset) {
  if (!c) return -EINVAL;
  return c->pool->ledger(out, max, reset);
}

int gsys_shutdown(gsys_ctx* c, uint64_t timeout_ns) {
  if (!c) return -EINVAL;
  int rc = gsys_wait(c, timeout_ns ? timeout_ns : 1);
  c->pool->stop_and_join();
  c->pool->poison_outstanding(claimed_tickets(c));
  if (!c->no_device) {
    hipSetDevice(c->device);
    hipDeviceSynchronize();
  }
  destroy(c);
  return rc;
}

const char* gsys_strerror(int code) {
  switch (-code) {
    case 0: return "success";
    case EPERM: return "call not in the whitelist";
    case EBADF: return "file descriptor not allowed";
    case EFAULT: return "address range not registered";
    case EINVAL: return "invalid argument";
    case ENOMEM: return "out of memory";
    case ENODEV: return "HIP runtime failure";
    case EEXIST: return "overlaps a registered buffer";
    case ENOENT: return "no such registration";
    case ETIMEDOUT: return "timed out";
    case ESHUTDOWN: return "context shut down";
    case EOVERFLOW: return "completion record reused before it was read";
    case EAGAIN: return "try again";
    case EINPROGRESS: return "not waited for";
    case ENOTSUP: return "no interrupt signal mapped for the GPU (doorbell)";
    case E2BIG: return "more jobs than the allocation-free scratch holds";
    default: return strerror(-code);
  }
}

}  // extern "C"

// ----------------------------------------------------------------- internal
namespace gsys_internal {

int check_host_range(gsys_ctx* c, uint64_t dev, uint64_t bytes) {
  // the pool's table holds every registration, including gsys_host_alloc ones
  return c->pool->host_range(dev, bytes) ? 0 : -EFAULT;
}

void* kstate(gsys_ctx* c) { return c->dev_words + 32; }

uint32_t resident_grid(gsys_ctx* c, const void* kernel, uint32_t block, uint32_t lds) {
  int per_cu = 0;
  const hipError_t e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, kernel, (int)block, lds);
  if (e == hipSuccess && per_cu < 1) {
    // The runtime has answered 0 for a work-group that fills a compute unit's
    // register file exactly (16 wavefronts of 128 VGPRs).  A work-group the
    // compiler built for this size (its flat work-group size bounds its
    // registers) whose LDS fits runs alone on an idle compute unit, so one
    // per compute unit is resident.
    hipFuncAttributes a{};
    int dev = 0, lds_cu = 0;
    hipGetDevice(&dev);
    if (hipFuncGetAttributes(&a, kernel) == hipSuccess && (int)block <= a.maxThreadsPerBlock &&
        hipDeviceGetAttribute(&lds_cu, hipDeviceAttributeMaxSharedMemoryPerMultiprocessor, dev) ==
            hipSuccess &&
        (uint64_t)lds + a.sharedSizeBytes <= (uint64_t)lds_cu) {
      fprintf(stderr, "gsys: occupancy query answered 0 (block %u, LDS %u bytes): one "
              "work-group per compute unit\n", block, lds);
      return (uint32_t)c->cu_count;
    }
  }
  if (e != hipSuccess || per_cu < 1) {
    hipFuncAttributes a{};
    const hipError_t ea = hipFuncGetAttributes(&a, kernel);
    int dev = -1;
    hipGetDevice(&dev);
    fprintf(stderr,
            "gsys: no resident work-group fits (%s; block %u, LDS %u bytes; device %d; "
            "kernel: %s, %d VGPRs, %zu B private, %zu B static LDS, %d threads at most)\n",
            e != hipSuccess ? hipGetErrorString(e) : "occupancy 0", block, lds, dev,
            hipGetErrorString(ea), a.numRegs, a.localSizeBytes, a.sharedSizeBytes,
            a.maxThreadsPerBlock);
    return 0;
  }
  return (uint32_t)per_cu * (uint32_t)c->cu_count;
}

uint32_t persistent_grid_override(gsys_ctx* c) { return c->grid_override; }

uint64_t ticks_per_ms(gsys_ctx* c) { return c->wall_khz; }

int control_page(gsys_ctx* c, void** host, uint64_t* dev) {
  // words 96 and 97 of the context's host-coherent page (their own line)
  *host = c->host_words + 96;
  *dev = (uint64_t)(c->retired_lo_dev + 96);
  return 0;
}

bool no_device(gsys_ctx* c) { return c->no_device; }

gsys_host::Pool* pool(gsys_ctx* c) { return c->pool; }

gsys_host::Doorbell* doorbell(gsys_ctx* c) { return c->db; }

gsys_slot* ring_host(gsys_ctx* c, uint64_t* slots) {
  *slots = c->D;
  return c->ring;
}

int device_of(gsys_ctx* c) { return c->device; }

uint64_t hash_words(std::initializer_list<uint64_t> w) {
  uint64_t h = 0x9e3779b97f4a7c15ull;
  for (uint64_t x : w) {
    h ^= x + 0x9e3779b97f4a7c15ull + (h << 6) + (h >> 2);
    h *= 0xbf58476d1ce4e5b9ull;
  }
  return h;
}

int launch(gsys_ctx* c, const void* kernel, uint32_t grid, uint32_t block, uint32_t lds, void** args,
           hipStream_t s) {
  if (c->no_device) return -ENODEV;  // a CPU-only context launches nothing
  hipSetDevice(c->device);
  const hipError_t e = hipLaunchKernel(kernel, dim3(grid), dim3(block), args, lds, s);
  if (e != hipSuccess) {
    fprintf(stderr, "gsys: kernel launch failed: %s (grid %u, block %u, LDS %u bytes)\n",
            hipGetErrorString(e), grid, block, lds);
    return -ENODEV;
  }
  return 0;
}

int launch_graph(gsys_ctx* c, uint64_t key, const KLaunch* k, uint32_t n, hipStream_t s) {
  if (!n) return -EINVAL;
  if (c->no_device) return -ENODEV;
  hipSetDevice(c->device);
  auto params = [&](uint32_t i) {
    hipKernelNodeParams p;
    memset(&p, 0, sizeof p);
    p.func = const_cast<void*>(k[i].kernel);
    p.gridDim = k[i].grid;
    p.blockDim = k[i].block;
    p.sharedMemBytes = k[i].lds;
    p.kernelParams = k[i].args;
    return p;
  };
  std::lock_guard<std::mutex> g(c->mu);
  auto it = c->graphs.find(key);
  if (it == c->graphs.end()) {
    // a chain of kernel nodes, each depending on the one before
    gsys_ctx::Graph G;
    if (hipGraphCreate(&G.graph, 0) != hipSuccess) return -ENODEV;
    for (uint32_t i = 0; i < n; ++i) {
      const hipKernelNodeParams p = params(i);
      hipGraphNode_t node;
      const hipGraphNode_t* dep = i ? &G.nodes.back() : nullptr;
      if (hipGraphAddKernelNode(&node, G.graph, dep, i ? 1 : 0, &p) != hipSuccess) {
        hipGraphDestroy(G.graph);
        return -ENODEV;
      }
      G.nodes.push_back(node);
    }
    if (hipGraphInstantiate(&G.exec, G.graph, nullptr, nullptr, 0) != hipSuccess) {
      hipGraphDestroy(G.graph);
      return -ENODEV;
    }
    it = c->graphs.emplace(key, std::move(G)).first;
  } else {
    // the same shape again: this launch's arguments go into the nodes (the
    // runtime copies them), so a caller may reuse one argument array with
    // new values, and every replay sees its own
    if (it->second.nodes.size() != n) return -EINVAL;
    for (uint32_t i = 0; i < n; ++i) {
      const hipKernelNodeParams p = params(i);
      if (hipGraphExecKernelNodeSetParams(it->second.exec, it->second.nodes[i], &p) != hipSuccess)
        return -ENODEV;
    }
  }
  if (hipGraphLaunch(it->second.exec, s) != hipSuccess) return -ENODEV;
  return 0;
}

}  // namespace gsys_internal
