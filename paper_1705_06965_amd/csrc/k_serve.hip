// Serving form: jobs of uneven size arrive over time and are admitted while
// others are running on the GPU (continuous batching).  Job kinds:
//   scan    pread a 4 KiB-aligned range of a file in 1 MiB pieces and store
//           the FNV-1a-64 of every 4 KiB block (the pread microbenchmark's
//           call and consumer, section 6);
//   pwrite  copy bytes from an HBM pool to staging and pwrite them (a
//           producer call, section 4.1);
//   release mmap a 2 MiB block of the reserved arena, fill it with pread,
//           pwrite one page's first 64 bytes back, madvise(MADV_DONTNEED),
//           pwrite page 0's first 64 bytes (now zeros), munmap: the memory
//           hand-back of section 7.2.
// Every call is made at work-group granularity with relaxed ordering (the
// paper's choice for its case studies); scans prefetch the next piece with a
// non-blocking call.
//
// Persistent form: the host driver posts a job by raising a counter in
// host-coherent memory; resident work-groups claim tasks in job order from a
// device cursor (job, task).  A scan longer than 8 MiB is cut into 8 MiB
// tasks that different work-groups run at once (a 64 MiB scan no longer
// holds one work-group for its whole read-and-hash time); every other job
// is one task.
// The work-group that completes a job's last task publishes its result and
// marks it done with a system-scope release store.  Plain form: one
// single-work-group launch per job.
#include "gsys_device.hpp"
#include "fnv_wave.hpp"
#include "gsys.h"
#include "kernels.hpp"

#include <errno.h>
#include <stdio.h>
#include <sys/mman.h>
#include <time.h>
#include <immintrin.h>

#include <algorithm>
#include <mutex>
#include <vector>

namespace gsys_sv {

using namespace gsys;
using gsys_k::Tile;
using gsys_k::wave_fnv_t;

constexpr uint32_t kWG = 256;
constexpr uint32_t kPiece = 1u << 20;          // scan read size (256 blocks of 4 KiB)
constexpr uint32_t kBlock = 4096;
constexpr uint64_t kRelBytes = 2ull << 20;
constexpr uint64_t kSplitMiB = 8;              // persistent form: default scan task size
// Default persistent grid: work-groups waiting for work poll host memory,
// and a few hundred of them slow the host pool's calls (see gsys_serve_run).
constexpr uint32_t kServeGrid = 64;

// Per-job progress of the persistent form (device memory, one per job).
struct JobState {
  unsigned long long bytes;     // scan: bytes read by the finished tasks
  long long err;                // first -errno of a task, 0 if none
  unsigned int done;            // finished tasks
  unsigned int ntasks;          // set by the host before the launch
  unsigned long long pad;
};

// Per-job state of the allocation-free entry point: a fixed array in device
// memory (2 MiB), one copy per GPU for the life of the process.  In host
// code `scratch` only names the array; its device address on each GPU is
// looked up once by scratch_setup() and kept in scratch_dev[].
constexpr uint32_t kScratchJobs = 65536;
static __device__ __align__(256) JobState scratch[kScratchJobs];
constexpr int kMaxDevices = 64;

struct SvArgs {
  gsys_dev_ctx c;
  gsys_job* jobs;               // host-coherent job records
  const uint64_t* ctl;          // host-coherent: [0] jobs posted, [1] stop
  unsigned long long* cursor;   // device: next (job << 32 | task) to claim
  JobState* js;                 // device: per-job progress (persistent form)
  uint64_t* digests;            // device: scan digests
  const uint8_t* content;       // device: pwrite content pool
  uint64_t staging;             // host: 2 x 1 MiB per work-group
  uint64_t lifetime_ticks;
  uint64_t split;               // persistent form: scan task size (multiple of 1 MiB)
};

__host__ __device__ inline uint32_t tasks_of(uint32_t kind, uint64_t len, uint64_t split) {
  return (kind == GSYS_JOB_SCAN && len > split) ? (uint32_t)((len + split - 1) / split) : 1u;
}

// Scan `len` bytes of fd at `off`; digests of its 4 KiB blocks go to
// digests[dig0 ...].  Returns the bytes read or the first -errno.
__device__ int64_t scan_range(const SvArgs& A, int32_t fd, uint64_t off, uint64_t len,
                              uint64_t dig0, uint8_t* lds, uint64_t stg0, uint64_t stg1) {
  const uint64_t blocks = len / kBlock;
  const uint64_t pieces = (len + kPiece - 1) / kPiece;
  int64_t total = 0;
  int64_t err = 0;
  auto issue = [&](uint64_t p) {
    const uint64_t bytes = std::min<uint64_t>(kPiece, len - p * kPiece);
    Args6 a{{(uint64_t)(int64_t)fd, (p & 1) ? stg1 : stg0, bytes, off + p * kPiece, 0, 0}};
    Ticket tk{0, 0, 0};
    call_wg<O::Relaxed, B::NonBlocking>(A.c, GSYS_NR_PREAD64, 0, a, &tk);
    return tk;
  };
  Ticket tk = pieces ? issue(0) : Ticket{0, 0, 0};
  for (uint64_t p = 0; p < pieces; ++p) {
    Ticket tn{0, 0, 0};
    if (p + 1 < pieces) tn = issue(p + 1);
    const int64_t r = wait_wg(A.c, tk);
    if (r < 0 && !err) err = r;
    if (r > 0) total += r;
    const uint64_t blk = p * (kPiece / kBlock) + threadIdx.x;
    const int64_t have = r - (int64_t)threadIdx.x * kBlock;
    const uint32_t nbytes = r <= 0 || have <= 0 ? 0u : (uint32_t)std::min<int64_t>(have, kBlock);
    const uint64_t base = (p & 1) ? stg1 : stg0;
    const uint64_t row0 = base + (uint64_t)(threadIdx.x & ~63u) * kBlock;
    const uint64_t h = wave_fnv_t<256>(row0, nbytes, kBlock, lds + (threadIdx.x >> 6) * Tile<256>::kBytes);
    if (blk < blocks) A.digests[dig0 + blk] = h;
    // the buffer of piece p is refilled by piece p + 2, issued next iteration
    __syncthreads();
    tk = tn;
  }
  return err ? err : total;
}

__device__ int64_t scan_job(const SvArgs& A, const gsys_job& J, uint8_t* lds, uint64_t stg0,
                            uint64_t stg1) {
  return scan_range(A, J.fd, J.off, J.len, J.src, lds, stg0, stg1);
}

__device__ int64_t pwrite_job(const SvArgs& A, const gsys_job& J, uint64_t stg0) {
  uint8_t* dst = reinterpret_cast<uint8_t*>(stg0);
  const uint8_t* src = A.content + J.src;
  const uint64_t n16 = J.len / 16;
  if ((J.src & 15) == 0) {
    for (uint64_t i = threadIdx.x; i < n16; i += blockDim.x)
      stg16((uint64_t)dst + 16 * i, ldg16((uint64_t)src + 16 * i));
    for (uint64_t i = n16 * 16 + threadIdx.x; i < J.len; i += blockDim.x)
      gp(dst)[i] = gp(src)[i];
  } else {
    for (uint64_t i = threadIdx.x; i < J.len; i += blockDim.x) gp(dst)[i] = gp(src)[i];
  }
  Args6 a{{(uint64_t)(int64_t)J.fd, stg0, J.len, J.off, 0, 0}};
  // producer call: every lane's copy is released before it; only the
  // caller's wavefront waits for the result
  const int64_t r = call_wg<O::Relaxed, B::Blocking>(A.c, GSYS_NR_PWRITE64, 0, a);
  __syncthreads();  // the staging buffer is reused by the next job
  return r;
}

__device__ int64_t release_job(const SvArgs& A, const gsys_job& J) {
  const uint64_t addr = A.c.arena + J.len * kRelBytes;
  int64_t first = 0;
  auto note = [&](int64_t r) {
    if (r < 0 && !first) first = r;
  };
  int64_t r = call_wg<O::Relaxed, B::Blocking>(
      A.c, GSYS_NR_MMAP, 0,
      Args6{{addr, kRelBytes, PROT_READ | PROT_WRITE, MAP_PRIVATE | MAP_ANONYMOUS | MAP_FIXED,
             (uint64_t)(int64_t)-1, 0}});
  note(r);
  if (r >= 0 && (uint64_t)r != addr) note(-EFAULT);
  if (r < 0) return first;
  note(call_wg<O::Relaxed, B::Blocking>(
      A.c, GSYS_NR_PREAD64, 0, Args6{{(uint64_t)(int64_t)J.aux_fd, addr, kRelBytes, J.src, 0, 0}}));
  note(call_wg<O::Relaxed, B::Blocking>(
      A.c, GSYS_NR_PWRITE64, 0,
      Args6{{(uint64_t)(int64_t)J.fd, addr + (uint64_t)J.page * kBlock, 64, J.off, 0, 0}}));
  note(call_wg<O::Relaxed, B::Blocking>(A.c, GSYS_NR_MADVISE, 0,
                                        Args6{{addr, kRelBytes, MADV_DONTNEED, 0, 0, 0}}));
  note(call_wg<O::Relaxed, B::Blocking>(
      A.c, GSYS_NR_PWRITE64, 0, Args6{{(uint64_t)(int64_t)J.fd, addr, 64, J.off + 64, 0, 0}}));
  note(call_wg<O::Relaxed, B::Blocking>(A.c, GSYS_NR_MUNMAP, 0,
                                        Args6{{addr, kRelBytes, 0, 0, 0, 0}}));
  // producer calls are weak-block: only the caller's wavefront holds their
  // results, so the verdict is the designated caller's
  return first;
}

__device__ __forceinline__ gsys_job load_job(const SvArgs& A, uint32_t j) {
  gsys_job J;
  const uint64_t* w = reinterpret_cast<const uint64_t*>(A.jobs + j);
  uint64_t v[8];
#pragma unroll
  for (int i = 0; i < 8; ++i) v[i] = ld_sys(w + i);
  __builtin_memcpy(&J, v, sizeof J);
  return J;
}

__device__ __forceinline__ void publish_job(const SvArgs& A, uint32_t j, int64_t res) {
  gsys_job* jp = A.jobs + j;
  __hip_atomic_store((uint64_t*)&jp->result, (uint64_t)res, __ATOMIC_RELAXED,
                     __HIP_MEMORY_SCOPE_SYSTEM);
  // every output of the job (digests in HBM, file writes done by the host)
  // is complete before the host sees `done`
  __threadfence();
  st_sys_rel(&jp->done, 1);
}

// Task t of job j (persistent form).  Every task folds its result into the
// job's progress record; the work-group that finishes the last task
// publishes the job.
__device__ void run_task(const SvArgs& A, uint32_t j, uint32_t t, uint8_t* lds, uint64_t stg0,
                         uint64_t stg1) {
  __shared__ int64_t s_tres;
  fence_acquire_sys();
  const gsys_job J = load_job(A, j);
  int64_t res;
  if (J.kind == GSYS_JOB_SCAN) {
    const uint64_t o = (uint64_t)t * A.split;
    // a single-task scan is the whole job (at most `split` bytes)
    const uint64_t len = o < J.len ? std::min<uint64_t>(A.split, J.len - o) : 0;
    res = scan_range(A, J.fd, J.off + o, len, J.src + o / kBlock, lds, stg0, stg1);
  } else if (J.kind == GSYS_JOB_PWRITE) {
    res = pwrite_job(A, J, stg0);
  } else if (J.kind == GSYS_JOB_RELEASE) {
    res = release_job(A, J);
  } else {
    res = -EINVAL;
  }
  if (threadIdx.x == 0) s_tres = res;
  __syncthreads();
  if (threadIdx.x == 0) {
    JobState* st = A.js + j;
    const int64_t r = s_tres;
    if (r < 0) {
      unsigned long long z = 0;
      __hip_atomic_compare_exchange_strong((unsigned long long*)&st->err, &z,
                                           (unsigned long long)r, __ATOMIC_RELAXED,
                                           __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    } else {
      __hip_atomic_fetch_add(&st->bytes, (unsigned long long)r, __ATOMIC_RELAXED,
                             __HIP_MEMORY_SCOPE_AGENT);
    }
    const unsigned int nt = st->ntasks;
    // release this task's outputs and accounting; the last finisher acquires
    // every other task's
    const unsigned int done =
        __hip_atomic_fetch_add(&st->done, 1u, __ATOMIC_ACQ_REL, __HIP_MEMORY_SCOPE_AGENT) + 1;
    if (done == nt) {
      int64_t out = r;
      if (J.kind == GSYS_JOB_SCAN) {
        const long long e = (long long)__hip_atomic_load((unsigned long long*)&st->err,
                                                         __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        out = e ? (int64_t)e
                : (int64_t)__hip_atomic_load(&st->bytes, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
      }
      publish_job(A, j, out);
    }
  }
  __syncthreads();
}

__device__ void run_job(const SvArgs& A, uint32_t j, uint8_t* lds, uint64_t stg0, uint64_t stg1) {
  __shared__ int64_t s_res;
  fence_acquire_sys();
  const gsys_job J = load_job(A, j);
  int64_t res;
  if (J.kind == GSYS_JOB_SCAN) res = scan_job(A, J, lds, stg0, stg1);
  else if (J.kind == GSYS_JOB_PWRITE) res = pwrite_job(A, J, stg0);
  else if (J.kind == GSYS_JOB_RELEASE) res = release_job(A, J);
  else res = -EINVAL;
  if (threadIdx.x == 0) s_res = res;
  __syncthreads();
  if (threadIdx.x == 0) publish_job(A, j, s_res);
  __syncthreads();
}

__global__ __launch_bounds__(kWG) void serve_persistent(SvArgs A) {
  extern __shared__ __align__(16) uint8_t lds[];
  __shared__ int s_job;
  __shared__ unsigned int s_task;
  const uint64_t stg0 = A.staging + (uint64_t)blockIdx.x * 2 * kPiece;
  const uint64_t stg1 = stg0 + kPiece;
  const uint64_t t_end = wall_clock64() + A.lifetime_ticks;
  for (;;) {
    if (threadIdx.x == 0) {
      int got = -1;
      unsigned int task = 0;
      uint32_t idle = 0;
      for (;;) {
        unsigned long long cur =
            __hip_atomic_load(A.cursor, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        const uint32_t nj = (uint32_t)(cur >> 32);
        const uint64_t posted = ld_sys(&A.ctl[0]);
        if (nj < posted) {
          const uint32_t t = (uint32_t)cur;
          const unsigned int nt = A.js[nj].ntasks;
          const unsigned long long next = t + 1 < nt ? cur + 1 : (unsigned long long)(nj + 1) << 32;
          if (__hip_atomic_compare_exchange_strong(A.cursor, &cur, next, __ATOMIC_RELAXED,
                                                   __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT)) {
            got = (int)nj;
            task = t;
            break;
          }
          continue;
        }
        if (ld_sys(&A.ctl[1]) || wall_clock64() > t_end) break;
        const uint32_t reps = 1u << min(idle, 5u);
        for (uint32_t r = 0; r < reps; ++r) __builtin_amdgcn_s_sleep(4);
        ++idle;
      }
      s_job = got;
      s_task = task;
    }
    __syncthreads();
    const int j = s_job;
    const unsigned int t = s_task;
    __syncthreads();
    if (j < 0) break;
    run_task(A, (uint32_t)j, t, lds, stg0, stg1);
  }
}

__global__ __launch_bounds__(kWG) void serve_one(SvArgs A, uint32_t j) {
  extern __shared__ __align__(16) uint8_t lds[];
  run_job(A, j, lds, A.staging, A.staging + kPiece);
}

__global__ void zero_u32(unsigned int* p, uint32_t n) {
  const uint32_t i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) p[i] = 0;
}

// Per-job progress records of the persistent form, set from the job records
// (host-coherent memory) before the launch: nothing done, the task count.
__global__ void init_jobs(JobState* js, const gsys_job* jobs, uint32_t n, uint64_t split) {
  const uint32_t i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  const uint64_t* w = reinterpret_cast<const uint64_t*>(jobs + i);
  const uint32_t kind = (uint32_t)ld_sys(w);                            // kind | fd << 32
  const uint64_t len = ld_sys(w + 2);
  js[i] = JobState{0, 0, 0, tasks_of(kind, len, split), 0};
}

uint64_t now_ns() {
  timespec ts;
  clock_gettime(CLOCK_MONOTONIC, &ts);
  return (uint64_t)ts.tv_sec * 1000000000ull + (uint64_t)ts.tv_nsec;
}

// Host buffer bytes a job holds while it is admitted and unfinished: a scan
// task streams through its work-group's two 1 MiB staging buffers, a pwrite
// stages its bytes, a release maps one 2 MiB arena block.
uint64_t job_bytes(const gsys_job& J, uint64_t split) {
  if (J.kind == GSYS_JOB_SCAN) return (uint64_t)tasks_of(J.kind, J.len, split) * 2ull * kPiece;
  if (J.kind == GSYS_JOB_PWRITE) return (J.len + kBlock - 1) / kBlock * kBlock;
  return kRelBytes;
}

// Every job record is checked before anything is launched: the kernels copy
// and store through the records' offsets without further bounds.
int check_jobs(const gsys_job* jobs, uint32_t n, const gsys_serve_params& P, uint64_t arena_bytes) {
  for (uint32_t i = 0; i < n; ++i) {
    const gsys_job& J = jobs[i];
    if (J.kind == GSYS_JOB_SCAN) {
      if (J.len % kBlock) return -EINVAL;
      if (J.src > P.n_digests || J.len / kBlock > P.n_digests - J.src) return -EINVAL;
    } else if (J.kind == GSYS_JOB_PWRITE) {
      if (J.len > kPiece) return -EINVAL;  // one staging buffer
      if (J.src > P.content_bytes || J.len > P.content_bytes - J.src) return -EINVAL;
    } else if (J.kind == GSYS_JOB_RELEASE) {
      if (J.len >= arena_bytes / kRelBytes || J.page >= kRelBytes / kBlock) return -EINVAL;
    } else {
      return -EINVAL;
    }
  }
  return 0;
}

// The serving loop shared by both entry points.  js: per-job state of the
// persistent form (n records), ignored by the plain form.
int serve_run(gsys_ctx* ctx, gsys_serve_params* P, JobState* js, hipStream_t s) {
  const uint32_t n = P->n;
  gsys_job* jobs = (gsys_job*)P->jobs_host;
  uint64_t* ctl_h = nullptr;
  uint64_t ctl_d = 0;
  if (int e = gsys_internal::control_page(ctx, (void**)&ctl_h, &ctl_d)) return e;
  SvArgs A;
  if (int e = gsys_device_ctx(ctx, &A.c)) return e;
  A.jobs = (gsys_job*)P->jobs_dev;
  A.ctl = (const uint64_t*)ctl_d;
  A.cursor = (unsigned long long*)gsys_internal::kstate(ctx) + 8;
  A.js = js;
  {
    // scan task size in MiB (0 = never split); overridable for tuning
    const char* e = getenv("GSYS_SERVE_SPLIT_MIB");
    const uint64_t mib = e && *e ? strtoull(e, nullptr, 0) : kSplitMiB;
    A.split = mib ? (mib << 20) : ~0ull;
  }
  A.digests = (uint64_t*)P->digests;
  A.content = (const uint8_t*)P->content;
  A.staging = P->staging;
  const uint64_t tmo = P->timeout_ns ? P->timeout_ns : 120000000000ull;
  A.lifetime_ticks = gsys_internal::ticks_per_ms(ctx) * (tmo / 1000000ull + 1000);
  uint64_t* lat = P->latency_ns;
  for (uint32_t i = 0; i < n; ++i) {
    __atomic_store_n(&jobs[i].done, 0ull, __ATOMIC_RELAXED);
    lat[i] = ~0ull;  // not finished yet
  }
  P->peak_inflight_bytes = 0;
  __atomic_store_n(&ctl_h[0], 0ull, __ATOMIC_RELEASE);
  __atomic_store_n(&ctl_h[1], 0ull, __ATOMIC_RELEASE);
  hipLaunchKernelGGL(zero_u32, dim3(1), dim3(64), 0, s, (unsigned int*)A.cursor, 2u);
  const uint32_t lds = (kWG / 64) * Tile<256>::kBytes;
  if (P->form == GSYS_PERSISTENT) {
    if (n) hipLaunchKernelGGL(init_jobs, dim3((n + 255) / 256), dim3(256), 0, s, js,
                              (const gsys_job*)P->jobs_dev, n, A.split);
    if (hipGetLastError() != hipSuccess || hipStreamSynchronize(s) != hipSuccess) return -ENODEV;
    const uint32_t res = gsys_internal::resident_grid(ctx, (const void*)serve_persistent, kWG, lds);
    if (!res) return -ENODEV;
    const uint64_t fit = P->staging_bytes / (2ull * kPiece);
    uint32_t grid = P->grid ? P->grid : kServeGrid;
    if (grid > res) grid = res;
    if (grid > fit) grid = (uint32_t)fit;
    void* args[] = {&A};
    if (int e = gsys_internal::launch(ctx, (const void*)serve_persistent, grid, kWG, lds, args, s))
      return e;
  } else if (hipStreamSynchronize(s) != hipSuccess) {
    return -ENODEV;
  }
  const uint64_t t0 = now_ns();
  const uint64_t deadline = t0 + tmo;
  const uint64_t budget = P->max_inflight_bytes;
  uint32_t posted = 0, completed = 0, oldest = 0;
  uint64_t held = 0;  // buffer bytes of admitted, unfinished jobs
  int rc = 0;
  while (completed < n) {
    const uint64_t t = now_ns();
    bool progress = false;
    // Admission: a job that has arrived is posted while fewer than
    // max_inflight jobs are unfinished and its bytes fit the budget (a job
    // larger than the whole budget is admitted alone).
    while (posted < n && t0 + P->arrival_ns[posted] <= t && posted - completed < P->max_inflight) {
      const uint64_t need = job_bytes(jobs[posted], A.split);
      if (budget && held && held + need > budget) break;
      if (P->form == GSYS_PERSISTENT) {
        __atomic_store_n(&ctl_h[0], (uint64_t)posted + 1, __ATOMIC_RELEASE);
      } else {
        SvArgs B = A;
        uint32_t jj = posted;
        void* args[] = {&B, &jj};
        if (hipLaunchKernel((const void*)serve_one, dim3(1), dim3(kWG), args, lds, s) != hipSuccess) {
          rc = -ENODEV;
          break;
        }
      }
      held += need;
      if (held > P->peak_inflight_bytes) P->peak_inflight_bytes = held;
      ++posted;
      progress = true;
    }
    if (rc) break;
    const uint64_t t2 = now_ns();
    for (uint32_t i = oldest; i < posted; ++i) {
      if (lat[i] == ~0ull && __atomic_load_n(&jobs[i].done, __ATOMIC_ACQUIRE)) {
        lat[i] = t2 - (t0 + P->arrival_ns[i]);
        held -= job_bytes(jobs[i], A.split);
        ++completed;
        progress = true;
      }
    }
    while (oldest < posted && lat[oldest] != ~0ull) ++oldest;
    if (t2 > deadline) {
      rc = -ETIMEDOUT;
      break;
    }
    if (!progress) _mm_pause();
  }
  __atomic_store_n(&ctl_h[1], 1ull, __ATOMIC_RELEASE);
  const hipError_t se = hipStreamSynchronize(s);
  if (se != hipSuccess) {
    fprintf(stderr, "gsys: serving stream: %s\n", hipGetErrorString(se));
    if (!rc) rc = -ENODEV;
  }
  return rc;
}

// Argument checks shared by both entry points (no HIP call).
int check_params(gsys_ctx* ctx, const gsys_serve_params* P) {
  if (!ctx || !P || !P->jobs_dev || !P->jobs_host || !P->arrival_ns || !P->latency_ns ||
      !P->max_inflight)
    return -EINVAL;
  if (P->form != GSYS_PLAIN && P->form != GSYS_PERSISTENT) return -EINVAL;
  if ((P->n_digests && !P->digests) || (P->content_bytes && !P->content)) return -EINVAL;
  if (gsys_internal::check_host_range(ctx, P->jobs_dev, (uint64_t)P->n * sizeof(gsys_job)))
    return -EFAULT;
  if (gsys_internal::check_host_range(ctx, P->staging, P->staging_bytes)) return -EFAULT;
  if (P->staging_bytes < 2ull * kPiece) return -EINVAL;
  gsys_dev_ctx c;
  if (int e = gsys_device_ctx(ctx, &c)) return e;
  if (int e = check_jobs((const gsys_job*)P->jobs_host, P->n, *P, c.arena ? c.arena_bytes : 0))
    return e;
  return 0;
}

std::mutex scratch_mu;
JobState* scratch_dev[kMaxDevices];  // device address of `scratch` per device

}  // namespace gsys_sv

using namespace gsys_sv;

// With `device` current: look up the device address of the allocation-free
// scratch array on it (once per device).
int gsys_internal::serve_scratch_setup(int device) {
  if (device < 0 || device >= kMaxDevices) return -ENODEV;
  std::lock_guard<std::mutex> g(scratch_mu);
  if (scratch_dev[device]) return 0;
  void* p = nullptr;
  const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
  if (e != hipSuccess || !p) {
    fprintf(stderr, "gsys: no device address for the serving scratch array: %s\n",
            hipGetErrorString(e));
    return -ENODEV;
  }
  scratch_dev[device] = (JobState*)p;
  return 0;
}

int gsys_serve_run_noalloc(gsys_ctx* ctx, gsys_serve_params* P, void* stream) {
  if (int e = check_params(ctx, P)) return e;
  if (P->n > kScratchJobs) return -E2BIG;
  if (gsys_internal::no_device(ctx)) return -ENODEV;
  const int dev = gsys_internal::device_of(ctx);
  JobState* js = nullptr;
  {
    std::lock_guard<std::mutex> g(scratch_mu);
    if (dev >= 0 && dev < kMaxDevices) js = scratch_dev[dev];
  }
  if (!js) return -ENODEV;  // gsys_init found no address for it
  return serve_run(ctx, P, js, (hipStream_t)stream);
}

int gsys_serve_run(gsys_ctx* ctx, gsys_serve_params* P, void* stream) {
  if (int e = check_params(ctx, P)) return e;
  if (gsys_internal::no_device(ctx)) return -ENODEV;
  hipStream_t s = (hipStream_t)stream;
  JobState* js = nullptr;
  if (P->form == GSYS_PERSISTENT &&
      hipMalloc((void**)&js, (uint64_t)(P->n ? P->n : 1) * sizeof(JobState)) != hipSuccess)
    return -ENOMEM;
  const int rc = serve_run(ctx, P, js, s);
  if (js) (void)hipFree(js);
  return rc;
}
