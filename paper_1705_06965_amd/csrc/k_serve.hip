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
// device cursor (job, task).  A scan longer than 16 MiB is cut into 16 MiB
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
#include <vector>

namespace gsys_sv {

using namespace gsys;
using gsys_k::Tile;
using gsys_k::wave_fnv_t;

constexpr uint32_t kWG = 256;
constexpr uint32_t kPiece = 1u << 20;          // scan read size (256 blocks of 4 KiB)
constexpr uint32_t kBlock = 4096;
constexpr uint64_t kRelBytes = 2ull << 20;
constexpr uint64_t kSplitMiB = 16;             // persistent form: default scan task size
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

uint64_t now_ns() {
  timespec ts;
  clock_gettime(CLOCK_MONOTONIC, &ts);
  return (uint64_t)ts.tv_sec * 1000000000ull + (uint64_t)ts.tv_nsec;
}

}  // namespace gsys_sv

using namespace gsys_sv;

int gsys_serve_run(gsys_ctx* ctx, uint32_t form, uint64_t jobs_dev, void* jobs_host, uint32_t n,
                   const uint64_t* arrival_ns, uint32_t max_inflight, uint64_t digests,
                   uint64_t content, uint64_t staging, uint64_t staging_bytes, uint32_t grid,
                   uint64_t timeout_ns, uint64_t* latency_ns, void* stream) {
  if (!ctx || !jobs_dev || !jobs_host || !arrival_ns || !latency_ns || !max_inflight) return -EINVAL;
  if (form != GSYS_PLAIN && form != GSYS_PERSISTENT) return -EINVAL;
  if (gsys_internal::check_host_range(ctx, jobs_dev, (uint64_t)n * sizeof(gsys_job))) return -EFAULT;
  if (gsys_internal::check_host_range(ctx, staging, staging_bytes)) return -EFAULT;
  if (staging_bytes < 2ull * kPiece) return -EINVAL;
  hipStream_t s = (hipStream_t)stream;
  gsys_job* jobs = (gsys_job*)jobs_host;
  uint64_t* ctl_h = nullptr;
  uint64_t ctl_d = 0;
  if (int e = gsys_internal::control_page(ctx, (void**)&ctl_h, &ctl_d)) return e;
  SvArgs A;
  if (int e = gsys_device_ctx(ctx, &A.c)) return e;
  A.jobs = (gsys_job*)jobs_dev;
  A.ctl = (const uint64_t*)ctl_d;
  A.cursor = (unsigned long long*)gsys_internal::kstate(ctx) + 8;
  A.js = nullptr;
  {
    // scan task size in MiB (0 = never split); overridable for tuning
    const char* e = getenv("GSYS_SERVE_SPLIT_MIB");
    const uint64_t mib = e && *e ? strtoull(e, nullptr, 0) : kSplitMiB;
    A.split = mib ? (mib << 20) : ~0ull;
  }
  A.digests = (uint64_t*)digests;
  A.content = (const uint8_t*)content;
  A.staging = staging;
  const uint64_t tmo = timeout_ns ? timeout_ns : 120000000000ull;
  A.lifetime_ticks = gsys_internal::ticks_per_ms(ctx) * (tmo / 1000000ull + 1000);
  for (uint32_t i = 0; i < n; ++i) {
    __atomic_store_n(&jobs[i].done, 0ull, __ATOMIC_RELAXED);
    latency_ns[i] = ~0ull;
  }
  __atomic_store_n(&ctl_h[0], 0ull, __ATOMIC_RELEASE);
  __atomic_store_n(&ctl_h[1], 0ull, __ATOMIC_RELEASE);
  hipLaunchKernelGGL(zero_u32, dim3(1), dim3(64), 0, s, (unsigned int*)A.cursor, 2u);
  const uint32_t lds = (kWG / 64) * Tile<256>::kBytes;
  JobState* js_dev = nullptr;
  if (form == GSYS_PERSISTENT) {
    // per-job task counts, fixed before the launch
    std::vector<JobState> st(n ? n : 1);
    for (uint32_t i = 0; i < n; ++i) {
      st[i] = JobState{0, 0, 0, tasks_of(jobs[i].kind, jobs[i].len, A.split), 0};
    }
    if (hipMalloc((void**)&js_dev, st.size() * sizeof(JobState)) != hipSuccess) return -ENOMEM;
    if (hipMemcpyAsync(js_dev, st.data(), st.size() * sizeof(JobState), hipMemcpyHostToDevice,
                       s) != hipSuccess ||
        hipStreamSynchronize(s) != hipSuccess) {
      hipFree(js_dev);
      return -ENODEV;
    }
    A.js = js_dev;
    uint32_t res = gsys_internal::resident_grid(ctx, (const void*)serve_persistent, kWG, lds);
    if (!res) {
      hipFree(js_dev);
      return -ENODEV;
    }
    const uint64_t fit = staging_bytes / (2ull * kPiece);
    if (!grid) grid = kServeGrid;
    if (grid > res) grid = res;
    if (grid > fit) grid = (uint32_t)fit;
    void* args[] = {&A};
    if (int e = gsys_internal::launch(ctx, (const void*)serve_persistent, grid, kWG, lds, args, s)) {
      hipFree(js_dev);
      return e;
    }
  } else if (hipStreamSynchronize(s) != hipSuccess) {
    return -ENODEV;
  }
  const uint64_t t0 = now_ns();
  const uint64_t deadline = t0 + tmo;
  uint32_t posted = 0, completed = 0, oldest = 0;
  int rc = 0;
  std::vector<uint8_t> seen(n, 0);
  while (completed < n) {
    const uint64_t t = now_ns();
    bool progress = false;
    while (posted < n && t0 + arrival_ns[posted] <= t && posted - completed < max_inflight) {
      if (form == GSYS_PERSISTENT) {
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
      ++posted;
      progress = true;
    }
    if (rc) break;
    const uint64_t t2 = now_ns();
    for (uint32_t i = oldest; i < posted; ++i) {
      if (!seen[i] && __atomic_load_n(&jobs[i].done, __ATOMIC_ACQUIRE)) {
        seen[i] = 1;
        latency_ns[i] = t2 - (t0 + arrival_ns[i]);
        ++completed;
        progress = true;
      }
    }
    while (oldest < posted && seen[oldest]) ++oldest;
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
  if (js_dev) hipFree(js_dev);
  return rc;
}
