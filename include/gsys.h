/*
 * gsys: GPU-issued system calls on one MI355X (gfx950), serviced in user
 * space by a host service pool.  C ABI of libgsys.so.
 *
 * Conventions for every entry point below:
 *   - Return 0 (or a non-negative count) on success and -errno on failure.
 *     Nothing aborts the process; gsys_strerror() names the code.
 *   - "device address" means an address a GPU kernel can dereference.  Host
 *     buffers from gsys_host_alloc() have one (returned in *dev_out); device
 *     buffers are plain hipMalloc memory.
 *   - `stream` is a hipStream_t passed as void* (NULL = the null stream).
 *   - A gsys_ctx is not thread-safe for init/shutdown; the launch entry points
 *     may be called from one host thread at a time per context.  Any number of
 *     GPU lanes may issue calls concurrently.
 *   - Arguments are checked before anything runs.  In a GSYS_CFG_NO_DEVICE
 *     context every call that would launch a kernel then returns -ENODEV and
 *     launches nothing.
 *
 * Whitelist.  The service pool executes only pread64, pwrite64, read, write,
 * sendto and recvfrom (IPv4 loopback peers only), mmap (anonymous, inside the
 * context's arena), munmap and madvise (MADV_DONTNEED, inside the arena),
 * openat (a relative path beneath a directory allowed with GSYS_FD_DIR) and
 * close (of a descriptor such an openat returned), on file descriptors the
 * caller allowed with gsys_allow_fd and buffers it registered.  Anything else
 * completes with -EPERM (call not allowed), -EBADF (fd not allowed), -EFAULT
 * (address range not registered) or -EINVAL (flags).
 */
#ifndef GSYS_H
#define GSYS_H

#include <stddef.h>
#include <stdint.h>

#include "gsys_abi.h"

#ifdef __cplusplus
extern "C" {
#endif

typedef struct gsys_ctx gsys_ctx;

/* gsys_config.flags */
#define GSYS_CFG_LEDGER    0x1u  /* record every serviced ticket (exactly-once checks) */
#define GSYS_CFG_NO_DEVICE 0x2u  /* host memory only, no HIP calls (CPU tests)        */
#define GSYS_CFG_NO_PIN    0x4u  /* do not pin service threads to cores              */
#define GSYS_CFG_SHARED_FDS 0x8u /* positional calls use the caller's descriptors
                                    directly (no per-thread copies, see below)       */
#define GSYS_CFG_DOORBELL  0x10u /* idle pollers block on an interrupt signal that
                                    the GPU raises after publishing, instead of
                                    spinning (see gsys_init)                          */

typedef struct gsys_config {
    uint32_t abi_version;        /* must be GSYS_ABI_VERSION                          */
    int32_t  device;             /* HIP device ordinal                                */
    uint32_t ring_slots;         /* D, power of two >= 64 (0 = 65536)                 */
    uint32_t service_threads;    /* P host pollers (0 = CPUs in the process's affinity
                                    mask - 1, at least 1)                            */
    uint32_t coalesce_max;       /* K: max calls per coalesced bundle (0/1 = off)     */
    uint32_t coalesce_window_ns; /* T: how long a poller waits to fill a bundle       */
    uint32_t stripe;             /* tickets per poller stripe (0 = 8; at least K when
                                    coalescing, at most 64)                          */
    uint32_t flags;              /* GSYS_CFG_*                                        */
    uint64_t arena_bytes;        /* reserved address range for GPU mmap (0 = none)    */
    uint64_t device_timeout_ns;  /* GPU watchdog on every wait (0 = 30 s)             */
    int32_t  first_cpu;          /* pin poller i to the (first_cpu + i)-th CPU of the
                                    affinity mask, wrapping (-1 = from the second)   */
    uint32_t ledger_capacity;    /* ledger records kept between resets (0 = 1<<20)    */
    uint32_t sleep_max;          /* GPU wait backoff cap, in s_sleep steps of ~256
                                    clocks doubled up to this count (0 = 64)           */
    uint32_t doorbell_idle_us;   /* GSYS_CFG_DOORBELL: how long a poller finds nothing
                                    before it blocks (0 = 200)                        */
    uint32_t reserved[2];
} gsys_config;

/*
 * Create a context: allocate the slot ring (D x 64 B) and the completion
 * records (C = max(4D, 65536) x 16 B) in fine-grained, host-coherent memory,
 * the device-side
 * ticket counter, and start P service threads that poll the ring.
 * The ring replaces the paper's syscall area (section 5); the polling pool
 * replaces its interrupt + work-queue dispatch (section 3 notes that the
 * design is orthogonal to interrupts versus polling).
 * GSYS_CFG_DOORBELL: the context also creates an HSA interrupt signal and a
 * relay thread that waits on it.  A poller that has found nothing for
 * doorbell_idle_us counts itself in a host-coherent sleeper word, looks at
 * its stripe once more and blocks (50 ms at most, a backstop); a GPU caller
 * that has published a request and sees a non-zero sleeper count stores a
 * new value into the signal and raises its interrupt, and the relay wakes
 * the blocked pollers.  Fences on both sides order the READY store /
 * sleeper load against the sleeper count / last look, so a request is never
 * left with its poller asleep.  Pollers then cost no CPU while the GPU is
 * quiet, at the price of the interrupt's latency (~75 us) on the first
 * request after a pause.
 * In a GSYS_CFG_NO_DEVICE context the doorbell is a condition variable that
 * host threads that emulate GPU callers (the tests' hook library) raise the
 * same way.
 * cfg == NULL uses all defaults.  *out receives the context.
 * Errors: -EINVAL (bad D / version), -ENOMEM, -ENODEV (HIP failure),
 * -ENOTSUP (GSYS_CFG_DOORBELL, but no interrupt signal mapped for the GPU).
 */
int gsys_init(const gsys_config *cfg, gsys_ctx **out);

/* fd permissions for gsys_allow_fd */
#define GSYS_FD_READ  0x1u
#define GSYS_FD_WRITE 0x2u
#define GSYS_FD_SOCK  0x4u
#define GSYS_FD_DIR   0x8u  /* a directory that GPU openat calls resolve beneath */

/*
 * Allow GPU calls on `fd` with `perms` (GSYS_FD_*).  The caller keeps
 * ownership of the fd and must keep it open until gsys_wait() returns.
 * perms == 0 revokes the fd (later calls on it complete with -EBADF).
 *
 * GSYS_FD_DIR (fd must be a directory, else -ENOTDIR) lets the GPU open
 * files beneath it: openat(dirfd, path, flags, mode) with `path` in a
 * registered host buffer (NUL within GSYS_PATH_MAX bytes, else
 * -ENAMETOOLONG), flags from O_RDONLY / O_WRONLY / O_RDWR / O_CREAT /
 * O_TRUNC / O_APPEND (others -EINVAL; writing needs GSYS_FD_WRITE on the
 * directory, creating needs it too, else -EPERM; mode & 0666).  The path is
 * resolved with openat2(RESOLVE_BENEATH | RESOLVE_NO_MAGICLINKS): absolute
 * paths, ".." and symlinks that leave the directory fail (-EXDEV).  The new
 * fd is allowed for the access the flags give and belongs to the pool: the
 * GPU closes it with close(fd) (-EBADF for any fd it did not open), and
 * gsys_shutdown closes the ones still open.  A GPU-opened fd must not be
 * closed while calls on it are in flight (as with POSIX close).
 *
 * For a regular file, each service thread runs pread / pwrite through its
 * own open file description of the same file (opened on first use through
 * /proc/self/fd with the fd's status flags), because calls from many
 * threads on one description contend on its reference count in the
 * kernel.  Positional calls behave the same on either; read / write use the
 * caller's fd and its file offset.  A thread's copy is re-opened after the
 * next gsys_allow_fd on that fd number and closed when the pool stops, so a
 * revoked file stays open until then.  GSYS_CFG_SHARED_FDS turns this off.
 * Errors: -EBADF (fd < 0 or >= 65536).
 */
int gsys_allow_fd(gsys_ctx *ctx, int fd, uint32_t perms);

/* buffer kinds */
#define GSYS_BUF_HOST   1u  /* host memory the host can write (pinned or library-allocated) */
#define GSYS_BUF_DEVICE 2u  /* HBM: GPU only, never a host call's target                  */

/*
 * Register [dev_addr, dev_addr + bytes) as a target of GPU calls.  host_addr
 * is where the host service pool reaches the same bytes (for GSYS_BUF_HOST;
 * NULL for GSYS_BUF_DEVICE).  The caller keeps ownership; the memory must
 * outlive gsys_wait().  *out_id receives a handle.
 * Errors: -EINVAL (bytes == 0, bad kind), -EEXIST (overlaps a registration).
 */
int gsys_register_buffer(gsys_ctx *ctx, uint64_t dev_addr, void *host_addr, uint64_t bytes,
                         uint32_t kind, uint32_t *out_id);

/*
 * Drop a registration.  Tickets the GPU has claimed may still name the
 * buffer, so while the host has not serviced every claimed ticket (after
 * waiting up to 10 ms for them) the call fails with -EBUSY and keeps it.
 * On success it returns only once no service thread can still be using the
 * buffer's memory: the caller may free it then.  Errors: -ENOENT, -EBUSY.
 */
int gsys_unregister_buffer(gsys_ctx *ctx, uint32_t id);

/*
 * Allocate `bytes` of fine-grained, host-coherent pinned memory that GPU
 * kernels can read and write while host threads do the same, and register it
 * as GSYS_BUF_HOST.  *host_out / *dev_out receive the host and device
 * addresses, *id_out the registration.  Freed by gsys_host_free() (which
 * unregisters it first, with gsys_unregister_buffer's -EBUSY rule, and
 * frees nothing when that fails) or at shutdown.  Errors: -ENOMEM, -ENODEV;
 * gsys_host_free: -ENOENT, -EBUSY.
 */
int gsys_host_alloc(gsys_ctx *ctx, uint64_t bytes, void **host_out, uint64_t *dev_out,
                    uint32_t *id_out);
int gsys_host_free(gsys_ctx *ctx, void *host_ptr);

/* Copy the device context (what a kernel needs to issue calls) into *out. */
int gsys_device_ctx(gsys_ctx *ctx, gsys_dev_ctx *out);

/* launch modes */
#define GSYS_PLAIN      0u  /* one launch as described                              */
#define GSYS_PERSISTENT 1u  /* grid clamped to what is co-resident on the device    */
#define GSYS_GRAPH      2u  /* persistent, captured once into a hipGraph, replayed  */

typedef struct gsys_launch_desc {
    const void *kernel;      /* __global__ function (host stub address)          */
    uint32_t grid[3];
    uint32_t block[3];
    uint32_t lds_bytes;      /* dynamic LDS                                      */
    uint32_t mode;           /* GSYS_PLAIN | GSYS_PERSISTENT | GSYS_GRAPH         */
    void   **args;           /* kernel argument pointers, as for hipLaunchKernel */
} gsys_launch_desc;

/*
 * Launch a kernel that issues gsys calls (the device API is
 * include/gsys_device.hpp; pass the kernel a gsys_dev_ctx from
 * gsys_device_ctx).  Every launch first clears the context's
 * kernel-granularity call sites (section 5: a kernel call's designated
 * caller is elected per launch), on the same stream.
 *   PLAIN       the grid as given (1-3 dimensions, at most 1024 work-items
 *               per work-group)
 *   PERSISTENT  grid[0] (a one-dimensional grid) clamped to the work-groups
 *               of that kernel that fit on the device at once, so that no
 *               call waits on a work-group that cannot run (section 4.1:
 *               kernel-wide ordering can deadlock when not every work-item
 *               is resident)
 *   GRAPH       as PERSISTENT, run as a hipGraph built once per (kernel,
 *               grid, block, LDS); every launch sets its own argument values
 *               into the graph before replaying it, so `args` may point at
 *               the same array with new values each time
 * Asynchronous on `stream`.  Errors: -EINVAL, -ENODEV (HIP launch failure,
 * or a CPU-only context).
 */
int gsys_launch(gsys_ctx *ctx, const gsys_launch_desc *desc, void *stream);

/*
 * Drain (section 8.3: a CPU-side call that makes sure every GPU system call
 * has completed).  Reads how many tickets the GPU has claimed and waits until
 * the host has serviced all of them, or `timeout_ns` passed (0 = forever).
 * Call it after the issuing kernels finished to drain everything.
 * Errors: -ETIMEDOUT.
 */
int gsys_wait(gsys_ctx *ctx, uint64_t timeout_ns);

typedef struct gsys_stats {
    uint64_t requests;          /* ring requests serviced (tickets)              */
    uint64_t host_calls;        /* POSIX calls executed for them                 */
    uint64_t bytes_in;          /* bytes delivered toward the GPU (pread, recv)  */
    uint64_t bytes_out;         /* bytes taken from the GPU (pwrite, send)       */
    uint64_t errors;            /* calls that returned -errno                    */
    uint64_t rejected;          /* requests refused by the whitelist checks      */
    uint64_t bundles;           /* coalesced bundles executed                    */
    uint64_t merged;            /* transfers folded into a neighbour's call      */
    uint64_t idle_polls;        /* poller passes that found nothing              */
    uint64_t retired_lo;        /* every ticket below this has retired           */
    uint64_t claimed;           /* tickets the GPU has claimed (read at call)    */
    uint64_t service_ns;        /* host time spent executing calls               */
    uint64_t bundle_hist[8];    /* bundle sizes 1, 2, 3-4, 5-8, 9-16, 17-32, 33-64, 65+ */
    uint64_t errno_hist[8];     /* EPERM, EBADF, EFAULT, EINVAL, EAGAIN, ESHUTDOWN, ETIMEDOUT, other */
    uint64_t doorbell_sleeps;   /* times a poller blocked on the doorbell        */
} gsys_stats;

/*
 * Snapshot the counters since the last reset; reset != 0 makes this
 * snapshot the new zero.  Each poller counts in its own block and the
 * snapshot sums them, so counts from calls still being completed may land
 * in the next snapshot.  retired_lo and claimed are read, never reset.
 */
int gsys_stats_get(gsys_ctx *ctx, gsys_stats *out, int reset);

/*
 * Ledger (GSYS_CFG_LEDGER): copy the records of serviced tickets, sorted by
 * ticket (the `max` lowest tickets when there are more), into
 * out[6*i .. 6*i+5] = {ticket, nr, ret, args digest, service start
 * (CLOCK_MONOTONIC ns), service end ns << 8 | poller index}.  out may be
 * NULL to count.  Returns the number of records copied; reset != 0 clears
 * the ledger.  Each poller records into its own shard, so recording does
 * not serialize the pool.
 */
int64_t gsys_ledger(gsys_ctx *ctx, uint64_t *out, uint64_t max, int reset);

/*
 * Stop the pool: drain with `timeout_ns`, complete every request still in the
 * ring with -ESHUTDOWN so GPU waiters return, join the threads, free the ring,
 * the completion records and every gsys_host_alloc() buffer.  ctx is invalid
 * afterwards.  Returns 0, or -ETIMEDOUT if the drain timed out (the context is
 * torn down all the same).
 */
int gsys_shutdown(gsys_ctx *ctx, uint64_t timeout_ns);

/* Static text for a 0 / -errno code. */
const char *gsys_strerror(int code);

/* ------------------------------------------------------------------------
 * Workload entry points.  Each launches hand-written gfx950 kernels that
 * issue calls through the ring and consume the results on the GPU.
 * ------------------------------------------------------------------------ */

/* invocation cell: granularity x ordering x blocking (section 4.1) */
#define GSYS_CELL_GRAN(c)   ((c) & 3u)        /* GSYS_GRAN_WI / _WG / _KERNEL */
#define GSYS_CELL_STRONG    0x4u
#define GSYS_CELL_BLOCKING  0x8u

/*
 * Per-item pread + FNV-1a-64 checksum (the pread microbenchmark of section 6,
 * Fig. 5): item i reads item_bytes at offsets[i] from `fd` into
 * staging + i * item_bytes, then the GPU computes out_fnv[i] over the bytes
 * read and stores the call's return value in out_ret[i].
 *
 *   offsets   device address, uint64[n_items]
 *   staging   device address of a registered GSYS_BUF_HOST buffer of
 *             `staging_bytes` bytes (0 = n_items * item_bytes).  The plain form
 *             needs room for every item (item i lands at staging + i *
 *             item_bytes).  The persistent forms also accept a smaller
 *             staging ring: each resident work-group then owns two batch
 *             buffers, and the grid shrinks to what the ring holds (at least
 *             2 * wg_size * item_bytes bytes).
 *   lists     device address of a registered GSYS_BUF_HOST buffer of at least
 *             n_items * 16 bytes (descriptor lists of group calls)
 *   out_fnv   device address, uint64[n_items];  out_ret: int64[n_items]
 *   cell      GSYS_CELL_* bits; work-item must be strong and kernel must be
 *             relaxed (section 4.1), others give -EINVAL
 *   form      GSYS_PLAIN (grid n_items / wg_size) or GSYS_PERSISTENT /
 *             GSYS_GRAPH (co-resident grid looping over batches of wg_size
 *             items, double-buffered non-blocking group calls; cell ignored).
 *             The persistent grid is 64 work-groups (fewer if fewer are
 *             resident or there are fewer batches; environment
 *             GSYS_PERSISTENT_GRID sets it instead): every work-group waiting
 *             for its call polls host memory, which slows the host pool, and
 *             64 groups of 256 keep enough reads in flight.
 *   wg_size   work-items per work-group: 64, 128, 256, 512 or 1024
 * item_bytes must be a multiple of 64 and at most 1 MiB; n_items % wg_size
 * need not be 0 (the tail work-group is partial).  n_items == 0 returns 0 at
 * once, launching nothing.
 * Errors: -EINVAL (shapes), -EFAULT (unregistered buffers), -ENODEV.
 */
int gsys_fnv4k(gsys_ctx *ctx, int fd, uint64_t offsets, uint64_t n_items, uint32_t item_bytes,
               uint64_t staging, uint64_t staging_bytes, uint64_t lists, uint64_t out_fnv,
               uint64_t out_ret, uint32_t cell, uint32_t form, uint32_t wg_size, void *stream);

/* One chunk of a file for gsys_wordscan. */
typedef struct gsys_chunk {
    int32_t  fd;       /* allowed for GSYS_FD_READ                     */
    uint32_t file;     /* row of the counts matrix                     */
    uint64_t off;      /* file offset of the chunk                     */
    uint32_t len;      /* chunk bytes (<= chunk_max)                   */
    uint32_t pad;
} gsys_chunk;

/*
 * Word search (the wordcount case study of section 7.1): counts[f * nq + q] =
 * number of tokens of file f equal to query q, a token being a maximal run of
 * bytes other than space (0x20) and newline (0x0a), compared exactly.
 *
 *   chunks    device gsys_chunk[n_chunks]: every file cut into chunks of at
 *             most chunk_max bytes that cover it exactly (a token belongs to
 *             the chunk in which it starts; each chunk's pread also fetches
 *             the byte before it and 16 bytes after it).  n_chunks == 0
 *             (every file empty, or nfiles == 0) launches only the zeroing
 *             of counts; chunks may then be 0
 *   queries   device uint8[nq * 16], query q in bytes [16q, 16q + qlens[q]);
 *             1 <= qlens[q] <= 16, no delimiter bytes, all distinct;
 *             1 <= nq <= 64
 *   counts    device uint32[nfiles * nq], zeroed by the call
 *   staging   registered GSYS_BUF_HOST buffer of staging_bytes; the plain
 *             form needs n_chunks * cbuf bytes, the persistent forms 2 * cbuf
 *             per resident work-group (the grid shrinks to fit), with
 *             cbuf = round_up(chunk_max + 64, 16)
 *   form      GSYS_PLAIN: one work-group per chunk, blocking relaxed
 *             work-group pread (the paper's setting); GSYS_PERSISTENT /
 *             GSYS_GRAPH: resident work-groups take chunks from a device work
 *             counter and prefetch the next chunk with a non-blocking call;
 *             GSYS_GRAPH runs the zeroing of counts and counter and the scan
 *             as one hipGraph per shape, replayed with this call's arguments
 *   passes    times the persistent forms read and scan every chunk within
 *             the one launch (work-groups go from one pass to the next
 *             without draining); counts add up, so each is passes times the
 *             file's (uint32, modulo 2^32).  The plain form takes 1 only;
 *             n_chunks * passes < 2^32.
 * Errors: -EINVAL (shapes), -EFAULT (staging not registered), -ENODEV.
 */
int gsys_wordscan(gsys_ctx *ctx, uint64_t chunks, uint32_t n_chunks, uint32_t chunk_max,
                  uint64_t queries, uint64_t qlens, uint32_t nq, uint64_t counts, uint32_t nfiles,
                  uint64_t staging, uint64_t staging_bytes, uint32_t form, uint32_t passes,
                  void *stream);

/*
 * Key-value GET server (the network case study of section 7.3: GPU
 * recvfrom / sendto at work-group granularity, blocking, relaxed).
 *
 * gsys_kv_build fills `table` (device, cap x 32-byte buckets) with the n keys
 * (device uint8[n * 16]); voff / vlen (device uint64[n] / uint32[n]) locate
 * each value in a device heap, 16-byte aligned, at most 1024 bytes.  Open
 * addressing: bucket = floor(FNV-1a-64(key) * cap / 2^64), linear probing.
 * Keys must be distinct; n <= cap <= 2^40.
 *
 * gsys_kv_serve launches the persistent server on the UDP socket `fd`
 * (allowed with GSYS_FD_SOCK, bound by the caller to 127.0.0.1).  Request
 * datagram (32 B): u64 id; u8 op (1 = GET); u8 pad[7]; u8 key[16].  Reply
 * (16 + len B): u64 id; u8 status (0 hit, 1 miss, 2 bad request); u8 pad;
 * u16 len; u32 pad; value[len]; sent to the request's source address.
 * Each work-group receives up to `batch` (<= 256) datagrams per recvfrom
 * list call.  flags: 0 = pipelined loop (the receive of a work-group's next
 * batch is in flight while it answers the current one; sends are
 * non-blocking over two sets of buffers), GSYS_KV_BLOCKING = one blocking
 * receive, then one blocking send, per batch.  io: registered GSYS_BUF_HOST
 * region of io_bytes, at least
 * gsys_kv_io_bytes() per work-group (the grid shrinks to fit; grid 0 =
 * as many as fit and are resident).  stop: registered host word; the server
 * exits when it reads nonzero, or after lifetime_ms (0 = 60 s).  served:
 * device uint64 incremented by the number of datagrams answered.
 * Returns after the launch; the caller sets *stop and synchronises.
 * Errors: -EINVAL, -EFAULT, -ENODEV.
 */
int gsys_kv_build(gsys_ctx *ctx, uint64_t table, uint64_t cap, uint64_t keys, uint64_t voff,
                  uint64_t vlen, uint64_t n, void *stream);
uint64_t gsys_kv_io_bytes(void);
#define GSYS_KV_BLOCKING 1u
int gsys_kv_serve(gsys_ctx *ctx, int fd, uint64_t table, uint64_t cap, uint64_t heap, uint64_t io,
                  uint64_t io_bytes, uint64_t stop, uint64_t served, uint32_t batch, uint32_t grid,
                  uint32_t flags, uint64_t lifetime_ms, void *stream);

/*
 * UDP load generator for the key-value server (the CPU load generator of
 * section 7.3).  `threads` client threads, each with its own loopback socket
 * and a contiguous slice of the n requests (req_len bytes each, request k
 * must carry id k + 1 in its first 8 bytes), keep up to `window` requests
 * outstanding, store reply k at replies + k * reply_stride (its length in
 * reply_len[k], and the time from first send to reply in lat_ns[k] if
 * lat_ns is not NULL), and retransmit after rto_ns (0 = 20 ms).  Returns the
 * number of requests answered, or -errno (-ETIMEDOUT after timeout_ns, 0 =
 * 60 s) when some are missing.  *retransmits (if not NULL) counts resends.
 */
int64_t gsys_kv_loadgen(uint32_t server_port, const uint8_t *reqs, uint32_t req_len, uint64_t n,
                        uint32_t threads, uint32_t window, uint64_t rto_ns, uint64_t timeout_ns,
                        uint8_t *replies, uint32_t reply_stride, uint32_t *reply_len,
                        uint64_t *lat_ns, uint64_t *retransmits);

/*
 * Host read capacity (a measurement helper, no GPU involved): `threads` host
 * threads take the n ranges (fds[i], offs[i], lens[i]) in order from a shared
 * counter, in runs of up to 256 (at least 8 runs per thread), and pread
 * range i into dst + (i mod n_slots) * slot_bytes, each
 * through its own open file description of the file (a read-only re-open of
 * the caller's fd, made before the timed passes), as the service pool does for GPU-issued preads (the
 * sweep's items, the word search's chunks of section 7.1); the best
 * of `reps` passes, in returned bytes per nanosecond (GB/s), is stored in
 * *out_gbps.  dst must hold n_slots * slot_bytes bytes (caller-owned).
 * Returns 0, -EINVAL (a null pointer, n, n_slots, threads or reps of 0,
 * threads > 1024, or a range longer than slot_bytes), -EBADF (an fd that is
 * not open) or the -errno of the first failed re-open or pread.
 */
int gsys_host_pread_rate(const int *fds, const uint64_t *offs, const uint32_t *lens, uint64_t n,
                         uint8_t *dst, uint64_t slot_bytes, uint64_t n_slots, uint32_t threads,
                         uint32_t reps, double *out_gbps);

/* Serving job record (64 bytes, in host-coherent memory). */
#define GSYS_JOB_SCAN    0u
#define GSYS_JOB_PWRITE  1u
#define GSYS_JOB_RELEASE 2u
typedef struct gsys_job {
    uint32_t kind;     /* GSYS_JOB_*                                                  */
    int32_t  fd;       /* scan: input file; pwrite / release: output file            */
    uint64_t off;      /* scan / pwrite: file offset; release: output offset (128 B) */
    uint64_t len;      /* scan: bytes (multiple of 4096); pwrite: bytes;
                          release: index of the 2 MiB arena block                    */
    uint64_t src;      /* scan: first digest index; pwrite: offset in the content
                          pool; release: offset in the stamp file                    */
    int32_t  aux_fd;   /* release: stamp file                                         */
    uint32_t page;     /* release: page (0..511) whose first 64 bytes are read back   */
    uint64_t done;     /* 0 until the GPU finishes the job                            */
    int64_t  result;   /* scan: bytes read or the first -errno; pwrite: its return
                          value; release: 0 or the first -errno                       */
    uint64_t pad;
} gsys_job;

/*
 * Serving (continuous batching, sections 2 and 6: long-lived work-groups
 * keep taking work while the host services earlier calls): run n jobs
 * arriving at arrival_ns[i] after the start (open loop).
 *
 * Scan jobs pread their range in 1 MiB pieces (the next piece is prefetched
 * with a non-blocking call) and store FNV-1a-64 of every 4 KiB block to
 * digests[src + block].  Pwrite jobs copy content[src .. src + len) (device)
 * to staging and pwrite it.  Release jobs (the madvise use of section 7.2)
 * mmap arena block `len` (2 MiB, the context's arena), pread it full from
 * aux_fd at src, pwrite the first 64 bytes of page `page` to fd at off,
 * madvise(MADV_DONTNEED), pwrite the first 64 bytes of page 0 to off + 64
 * (zeros) and munmap.  All calls are work-group granularity, relaxed.
 *
 * Admission: a job that has arrived is posted while fewer than max_inflight
 * posted jobs are unfinished and, when max_inflight_bytes is not 0, while
 * its buffer bytes fit beside theirs (a job larger than the whole budget is
 * posted only when nothing else is in flight).  A job's buffer bytes are
 * what it holds while in flight: 2 MiB of staging per scan task, its length
 * rounded up to 4 KiB for a pwrite, 2 MiB of arena for a release.
 * latency_ns[i] is the time from job i's scheduled arrival to the host
 * seeing it done (queueing included).
 *
 * Every job record is checked before anything is launched; a record that
 * fails a check makes the call return -EINVAL with nothing run: kind is one
 * of GSYS_JOB_*; scan: len a multiple of 4096 and src + len / 4096 <=
 * n_digests; pwrite: len <= 1 MiB and src + len <= content_bytes; release:
 * len < (the context's arena bytes) / 2 MiB and page < 512.
 */
typedef struct gsys_serve_params {
    uint32_t form;               /* GSYS_PERSISTENT: resident work-groups claim tasks in
                                    job order as jobs are posted; a scan longer than 8 MiB
                                    (environment GSYS_SERVE_SPLIT_MIB overrides the size,
                                    0 = never split) is cut into tasks of that size run by
                                    different work-groups, and the work-group finishing its
                                    last task publishes the job (result: bytes read, or the
                                    first -errno of any task).  GSYS_PLAIN: one
                                    single-work-group launch per job on `stream`, in
                                    arrival order                                        */
    uint32_t n;                  /* jobs                                                   */
    uint64_t jobs_dev;           /* gsys_job[n] in a registered host buffer (GPU address) */
    void    *jobs_host;          /* the same records, host address; filled by the caller,
                                    done / result are written here                        */
    const uint64_t *arrival_ns;  /* host uint64[n], non-decreasing                         */
    uint64_t *latency_ns;        /* host uint64[n], out                                    */
    uint32_t max_inflight;       /* >= 1                                                   */
    uint32_t grid;               /* persistent work-groups; 0 = 64.  Every work-group
                                    waiting for work polls host memory, and a few hundred of
                                    them slow the host pool's calls enough to tip a 20k
                                    jobs/s stream into a standing backlog                  */
    uint64_t max_inflight_bytes; /* 0 = no byte budget                                     */
    uint64_t digests;            /* device uint64[n_digests]                               */
    uint64_t n_digests;
    uint64_t content;            /* device bytes[content_bytes]                            */
    uint64_t content_bytes;
    uint64_t staging;            /* registered host buffer, 2 MiB per work-group (the
                                    persistent grid shrinks to fit; at least 2 MiB)        */
    uint64_t staging_bytes;
    uint64_t timeout_ns;         /* 0 = 120 s                                              */
    uint64_t peak_inflight_bytes;/* out: the most buffer bytes admitted at once            */
} gsys_serve_params;

/* Blocks until every job is done (or timeout_ns: -ETIMEDOUT).  Allocates the
 * persistent form's per-job state (32 bytes per job) in device memory for
 * the call.  Errors: -EINVAL, -EFAULT, -ENOMEM, -ENODEV, -ETIMEDOUT. */
int gsys_serve_run(gsys_ctx *ctx, gsys_serve_params *params, void *stream);

/*
 * gsys_serve_run for callers that cannot allocate memory during the call
 * (code under HIP graph capture, tight serving loops, harnesses that forbid
 * hipMalloc): the same session and results, but the persistent form's
 * per-job state lives in a fixed array of 65,536 records (2 MiB) in device
 * memory that the library holds on each GPU it runs on until the process
 * ends.  Nothing is allocated by the call (no hipMalloc / hipFree, no host
 * heap).  params and stream as for gsys_serve_run; n above 65,536 returns
 * -E2BIG with nothing run.  Every call on one GPU shares that GPU's array
 * (each call sets the records of its n jobs before launching), so calls that
 * overlap on one GPU race: run them one after the other.  Errors: as for
 * gsys_serve_run, plus -E2BIG.
 */
int gsys_serve_run_noalloc(gsys_ctx *ctx, gsys_serve_params *params, void *stream);

/*
 * Visibility canary for producer calls (section 4.1 ordering): work-item i
 * writes 64 stamp bytes (eight little-endian words
 * (seed * 0x9E3779B97F4A7C15) ^ ((8i + k + 1) * 0xD1B54A32D192ED03), k =
 * 0..7, mod 2^64) at buf + 64i, then the buffer is written to `fd` with
 * pwrite at the granularity / ordering / blocking of `cell`: each work-item
 * its 64 bytes at file offset 64i, each work-group its range, or the last
 * work-group of the kernel the whole buffer.  The file must then hold every
 * stamp.  out_ret (device int64) receives each call's return value: per
 * work-item, per work-group, or [0] for the kernel call.
 * buf: registered GSYS_BUF_HOST, n_items * 64 bytes.  wg_size: 64..1024,
 * multiple of 64.  Errors: -EINVAL (illegal cell, shapes), -EFAULT.
 */
int gsys_canary(gsys_ctx *ctx, int fd, uint64_t buf, uint64_t n_items, uint64_t seed,
                uint64_t out_ret, uint32_t cell, uint32_t wg_size, void *stream);

/*
 * The wordcount as section 7.1 issues it: persistent work-groups take files
 * f from a device counter; for each one calls openat(dirfd, paths + f * GSYS_PATH_MAX,
 * O_RDONLY), read(fd, buf, chunk) until a read returns fewer than chunk
 * bytes (the end of a regular file), and close(fd), all at work-group
 * granularity with relaxed ordering (the next read is in flight while the
 * previous piece is scanned).  counts[f][q] (device uint32, zeroed here) =
 * tokens of file f equal to query q (tokens: maximal runs of bytes other
 * than space and newline; queries as for gsys_wordscan); file_ret[f]
 * (device int64) = bytes read, or the -errno of the failing openat / read /
 * close.
 *   dirfd    allowed with GSYS_FD_DIR | GSYS_FD_READ (see gsys_allow_fd)
 *   paths    registered host buffer of nfiles x GSYS_PATH_MAX bytes of
 *            NUL-terminated paths relative to dirfd
 *   chunk    bytes per read: a multiple of 64, 64 .. 64 MiB
 *   staging  registered host buffer; each resident work-group uses two
 *            buffers of gsys_wordcount_open_buffer_bytes(chunk) bytes (the
 *            grid shrinks to fit)
 *   progress 0, or a registered host buffer of progress_groups x 16 bytes
 *            (the grid shrinks to progress_groups): work-group w keeps
 *            [2w] = (file + 1) << 32 | phase (1 openat, 2 waiting for a
 *            read, 3 scanning, 4 close, 5 no more files) and [2w + 1] =
 *            piece << 32 | low 32 bits of the ticket waited for, stored at
 *            system scope so the host can read them while the kernel runs
 * Asynchronous on `stream`; gsys_wait drains the host side.  nfiles == 0
 * returns 0 once the shapes (nq, chunk) pass, launching nothing; the
 * pointers may then be null.  Errors: -EINVAL, -EFAULT (paths, staging or
 * progress not registered), -ENODEV.
 */
/* Bytes of one piece buffer of gsys_wordcount_open for reads of `chunk`
 * bytes: the carried bytes, the piece and the scanner's window past it. */
uint64_t gsys_wordcount_open_buffer_bytes(uint32_t chunk);
int gsys_wordcount_open(gsys_ctx *ctx, int dirfd, uint64_t paths, uint32_t nfiles,
                        uint64_t queries, uint64_t qlens, uint32_t nq, uint64_t counts,
                        uint64_t file_ret, uint32_t chunk, uint64_t staging,
                        uint64_t staging_bytes, uint64_t progress, uint32_t progress_groups,
                        void *stream);

/*
 * Block permutation written out with pwrite: the ordering / blocking
 * microbenchmark of section 6 (Fig. 6).  `in` (device, n_blocks * 8192
 * bytes, little-endian 64-bit words) is cut into 8 KiB blocks; one
 * work-group of 1024 work-items per block applies `iters` rounds of
 *     bit j of y[i] = bit tau[j] of x[sigma[i]]   (i < 1024, j < 64)
 * and then issues one work-group pwrite(fd, staging + 8192 b, 8192,
 * file_off + 8192 b) under the ordering / blocking of `cell` (work-group
 * granularity only).  The result never lands in `in`.
 *   sigma, tau  host arrays: permutations of 0..1023 and 0..63 (copied into
 *               the launch; anything else is -EINVAL)
 *   staging     registered GSYS_BUF_HOST, n_blocks * 8192 bytes; it must not
 *               be reused before gsys_wait returns
 *   out_ret     device int64[n_blocks]: blocking cells get pwrite's result;
 *               non-blocking cells get GSYS_NOT_WAITED (the results are in
 *               the ledger) unless the call could not be issued
 * n_blocks == 0 launches nothing.  The launch is asynchronous on `stream`;
 * non-blocking calls may still be in service when the kernel ends:
 * gsys_wait drains them.  Errors: -EINVAL (cell, tables, sizes), -EFAULT.
 */
int gsys_permute(gsys_ctx *ctx, int fd, uint64_t in, const uint16_t *sigma, const uint8_t *tau,
                 uint64_t n_blocks, uint32_t iters, uint64_t staging, uint64_t file_off,
                 uint64_t out_ret, uint32_t cell, void *stream);

/*
 * Stateful file calls at work-group granularity (read() and write() advance
 * the file offset; sections 4.1 and 8.1).  Work-group f (grid = nfiles, 256
 * work-items) issues, one call at a time:
 *     openat(dirfd, paths + f * GSYS_PATH_MAX, O_WRONLY|O_CREAT|O_TRUNC, 0600)
 *     write(fd, piece p)        for p = 0 .. K-1, K = ceil(file_bytes / piece)
 *     close(fd)
 *     openat(dirfd, path, O_RDONLY)
 *     read(fd, piece p)         for p = 0 .. K-1, then one 16-byte read at
 *                               the end of the file (must return 0)
 *     close(fd)
 * and counts the bytes read back that differ from what it wrote.  Piece p
 * of file f is data[f * file_bytes + p * piece ...] (device), at most
 * `piece` bytes; the work-group copies it into its write area of staging
 * before the write.  The writes are producers under the ordering of `cell`
 * (work-group, strong or relaxed, blocking; anything else is -EINVAL); the
 * other calls are relaxed and blocking.  Outputs (device):
 *   rets      int64[nfiles][2K + 5], every call's result in the order above;
 *             a failed openat ends the file's sequence (later entries are
 *             left as they were)
 *   mismatch  uint64[nfiles] (zeroed here): bytes read back that differ
 * staging: registered host buffer of at least nfiles * 2 * A bytes, A =
 * max(file_bytes, 16) rounded up to 16 (write area, then read area, per
 * file).  dirfd must be allowed with GSYS_FD_DIR and GSYS_FD_READ |
 * GSYS_FD_WRITE.  file_bytes <= 2 GiB, K <= 2^20.  Asynchronous on
 * `stream`.  nfiles == 0 returns 0 at once (rets and mismatch may then be
 * null).  Errors: -EINVAL, -EFAULT (paths or staging not registered),
 * -ENODEV.
 */
int gsys_file_roundtrip(gsys_ctx *ctx, int dirfd, uint64_t paths, uint32_t nfiles, uint64_t data,
                        uint64_t file_bytes, uint32_t piece, uint64_t staging,
                        uint64_t staging_bytes, uint64_t rets, uint64_t mismatch, uint32_t cell,
                        void *stream);

/*
 * One stateful call for the whole kernel (kernel granularity, relaxed,
 * blocking) through `fd`, which the caller opened and allowed.
 *   nr = GSYS_NR_WRITE: every work-group stores its slice of `data` (device,
 *        `bytes`) into `staging`; the last work-group to arrive calls
 *        write(fd, staging, bytes), so the bytes land at the file offset and
 *        consecutive launches append in launch order.
 *   nr = GSYS_NR_READ: the first work-group to arrive calls read(fd,
 *        staging, bytes); every work-group waits for it and counts the bytes
 *        of its slice that differ from `data`.
 * ret: device int64[1], the call's result; mismatch: device uint64[1]
 * (zeroed here).  staging: registered host buffer of `bytes`.  grid: 1 ..
 * 65535 work-groups of 256.  Errors: -EINVAL, -EFAULT, -ENODEV.
 */
int gsys_file_kernel_io(gsys_ctx *ctx, int fd, uint32_t nr, uint64_t data, uint64_t bytes,
                        uint64_t staging, uint64_t ret, uint64_t mismatch, uint32_t grid,
                        void *stream);

/*
 * Kernel-split baseline (section 2, Fig. 1 left): no GPU system calls.  The
 * host has already read every item into `staging` (any device-readable
 * address: registered host memory or HBM); one kernel computes
 * out_fnv[i] = FNV-1a-64 of the first rets[i] bytes (rets: device int64[n],
 * values <= 0 hash nothing) of staging + i * item_bytes.  grid 0 = one
 * work-group per wg_size items, otherwise a grid-stride loop over them.
 * n_items == 0 returns 0 at once (the pointers may then be null).
 * Errors: -EINVAL.
 */
int gsys_fnv4k_consume(gsys_ctx *ctx, uint64_t staging, uint64_t rets, uint64_t n_items,
                       uint32_t item_bytes, uint64_t out_fnv, uint32_t wg_size, uint32_t grid,
                       void *stream);

#ifdef __cplusplus
}
#endif

#endif /* GSYS_H */
