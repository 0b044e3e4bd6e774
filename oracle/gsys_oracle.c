/*
 * Oracle for the GPU system-call workloads.  TEST INFRASTRUCTURE ONLY.
 *
 * Only the test suite, the smoke check and the CPU-baseline leg of the
 * benchmark load this library.  The GPU path never calls it, and it shares no
 * code, header, table or helper with the GPU path.
 *
 * What it computes.  The paper's mechanism forwards a system call made by a
 * GPU work-item, work-group or kernel to the CPU, which executes exactly the
 * call that was requested and hands back its return value, keeping the
 * semantics of an ordinary function call (section 3, Fig. 2; section 5).
 * The result of a GPU
 * program that uses such calls is therefore defined as the result of the CPU
 * issuing the same calls itself.  This file is that definition written out:
 * it calls pread/pwrite/recvfrom/sendto/mmap/madvise/munmap directly, in the
 * plainest order, and computes the consumers' outputs byte by byte:
 *
 *   - FNV-1a 64-bit checksum of each item read (the checksum is not in the
 *     paper; it is the published FNV-1a definition: offset basis
 *     0xcbf29ce484222325, prime 0x100000001b3, xor then multiply, per byte);
 *   - word counts in the style of the wordcount case study (section 7.1):
 *     a token is a maximal run of bytes other than space (0x20) and newline
 *     (0x0a); counts[f][q] is the number of tokens of file f equal to query q
 *     (files read with pread, or opened by name and read with read());
 *   - key-value GET replies in the style of the UDP server case study
 *     (section 7.3), with a sorted key index and bsearch;
 *   - memory release with madvise(MADV_DONTNEED) in the style of section 7.2;
 *   - the block permutation written out with pwrite of section 6 (Fig. 6);
 *   - a file written with write() and read back with read() (stateful
 *     calls whose results follow the file offset).
 *
 * Pins (tests/test_oracle_pins.py): published FNV-1a test vectors; slicing of
 * the file bytes for every (offset, length) pair on tiny files including EOF;
 * Python bytes.split() counting; dictionary lookups; zero pages after
 * MADV_DONTNEED on private anonymous memory (Linux madvise(2)); for the
 * permutation, numpy's flat bit-index gather, byte swapping, rotations with a
 * closed form and the order of the permutation.
 *
 * Threads: where a function takes `threads`, items (or files) are split into
 * contiguous ranges, one per POSIX thread, as the paper's CPU wordcount
 * assigns files to cores.
 */
#define _GNU_SOURCE
#include <errno.h>
#include <fcntl.h>
#include <pthread.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#include <sys/mman.h>
#include <sys/socket.h>
#include <netinet/in.h>
#include <unistd.h>

/* ------------------------------------------------------------------ FNV-1a */

uint64_t oracle_fnv1a64(const uint8_t *p, uint64_t n)
{
    uint64_t h = 0xcbf29ce484222325ULL;
    for (uint64_t i = 0; i < n; i++) {
        h ^= (uint64_t)p[i];
        h *= 0x100000001b3ULL;
    }
    return h;
}

/* ------------------------------------------------------ pread + checksum */
/*
 * For item i: r = pread(fd, buf, len, off[i]); ret[i] = r (or -errno);
 * fnv[i] = FNV-1a-64 of the r bytes read (of nothing if r <= 0).
 * This is the per-item call of the pread microbenchmark (section 6, Fig. 5),
 * issued by the CPU itself.
 */
struct pf_job {
    int fd;
    const uint64_t *off;
    uint64_t lo, hi;
    uint32_t len;
    uint64_t *fnv;
    int64_t *ret;
    int err;
};

static void *pf_worker(void *arg)
{
    struct pf_job *j = (struct pf_job *)arg;
    uint8_t *buf = (uint8_t *)malloc(j->len ? j->len : 1);
    if (!buf) { j->err = -ENOMEM; return NULL; }
    for (uint64_t i = j->lo; i < j->hi; i++) {
        ssize_t r = pread(j->fd, buf, j->len, (off_t)j->off[i]);
        if (r < 0) {
            j->ret[i] = -(int64_t)errno;
            j->fnv[i] = oracle_fnv1a64(buf, 0);
        } else {
            j->ret[i] = (int64_t)r;
            j->fnv[i] = oracle_fnv1a64(buf, (uint64_t)r);
        }
    }
    free(buf);
    return NULL;
}

int oracle_pread_fnv(int fd, const uint64_t *off, uint64_t n, uint32_t len,
                     uint64_t *fnv, int64_t *ret, int threads)
{
    if (threads < 1) threads = 1;
    if ((uint64_t)threads > n) threads = n ? (int)n : 1;
    struct pf_job *jobs = (struct pf_job *)calloc((size_t)threads, sizeof *jobs);
    pthread_t *tid = (pthread_t *)calloc((size_t)threads, sizeof *tid);
    if (!jobs || !tid) { free(jobs); free(tid); return -ENOMEM; }
    for (int t = 0; t < threads; t++) {
        jobs[t] = (struct pf_job){fd, off, n * (uint64_t)t / (uint64_t)threads,
                                  n * (uint64_t)(t + 1) / (uint64_t)threads,
                                  len, fnv, ret, 0};
        if (t > 0) pthread_create(&tid[t], NULL, pf_worker, &jobs[t]);
    }
    pf_worker(&jobs[0]);
    int err = jobs[0].err;
    for (int t = 1; t < threads; t++) {
        pthread_join(tid[t], NULL);
        if (jobs[t].err) err = jobs[t].err;
    }
    free(jobs); free(tid);
    return err;
}

/* ------------------------------------------------------------ word counts */
/*
 * counts[f*nq + q] = number of tokens of file f equal to query q.  Each file
 * is read whole with pread (looping on short reads) and scanned once.
 * qbytes holds query q at qbytes + q*qstride, length qlen[q].
 */
struct wc_job {
    const int *fds;
    const uint64_t *sizes;
    uint32_t lo, hi, nq, qstride;
    const uint8_t *qbytes;
    const uint32_t *qlen;
    uint32_t *counts;
    int err;
};

static int is_delim(uint8_t c) { return c == 0x20 || c == 0x0a; }

/* cnt[q] = number of tokens of buf[0..n) equal to query q */
static void count_tokens(const uint8_t *buf, uint64_t n, const uint8_t *qbytes,
                         const uint32_t *qlen, uint32_t nq, uint32_t qstride, uint32_t *cnt)
{
    for (uint32_t q = 0; q < nq; q++) cnt[q] = 0;
    uint64_t p = 0;
    while (p < n) {
        if (is_delim(buf[p])) { p++; continue; }
        uint64_t s = p;
        while (p < n && !is_delim(buf[p])) p++;
        uint64_t tl = p - s;
        for (uint32_t q = 0; q < nq; q++) {
            if (qlen[q] == tl && memcmp(buf + s, qbytes + (uint64_t)q * qstride, tl) == 0)
                cnt[q]++;
        }
    }
}

static void *wc_worker(void *arg)
{
    struct wc_job *j = (struct wc_job *)arg;
    for (uint32_t f = j->lo; f < j->hi; f++) {
        uint64_t size = j->sizes[f];
        uint8_t *buf = (uint8_t *)malloc(size ? size : 1);
        if (!buf) { j->err = -ENOMEM; return NULL; }
        uint64_t got = 0;
        while (got < size) {
            ssize_t r = pread(j->fds[f], buf + got, size - got, (off_t)got);
            if (r < 0) { j->err = -errno; free(buf); return NULL; }
            if (r == 0) break;
            got += (uint64_t)r;
        }
        count_tokens(buf, got, j->qbytes, j->qlen, j->nq, j->qstride,
                     j->counts + (uint64_t)f * j->nq);
        free(buf);
    }
    return NULL;
}

int oracle_wordcount(const int *fds, const uint64_t *sizes, uint32_t nfiles,
                     const uint8_t *qbytes, const uint32_t *qlen, uint32_t nq,
                     uint32_t qstride, uint32_t *counts, int threads)
{
    if (threads < 1) threads = 1;
    if ((uint32_t)threads > nfiles) threads = nfiles ? (int)nfiles : 1;
    struct wc_job *jobs = (struct wc_job *)calloc((size_t)threads, sizeof *jobs);
    pthread_t *tid = (pthread_t *)calloc((size_t)threads, sizeof *tid);
    if (!jobs || !tid) { free(jobs); free(tid); return -ENOMEM; }
    for (int t = 0; t < threads; t++) {
        jobs[t] = (struct wc_job){fds, sizes,
                                  (uint32_t)((uint64_t)nfiles * t / threads),
                                  (uint32_t)((uint64_t)nfiles * (t + 1) / threads),
                                  nq, qstride, qbytes, qlen, counts, 0};
        if (t > 0) pthread_create(&tid[t], NULL, wc_worker, &jobs[t]);
    }
    wc_worker(&jobs[0]);
    int err = jobs[0].err;
    for (int t = 1; t < threads; t++) {
        pthread_join(tid[t], NULL);
        if (jobs[t].err) err = jobs[t].err;
    }
    free(jobs); free(tid);
    return err;
}

/*
 * The wordcount as the case study of section 7.1 issues it: every file is
 * opened by name (openat beneath dirfd), read front to back with read() in
 * pieces of `chunk` bytes until it returns 0, closed, and its tokens are
 * counted as above.  Paths are NUL-terminated strings `stride` bytes apart.
 * rets[f] = bytes read, or -errno of the failing open or read (counts 0).
 */
struct wo_job {
    int dirfd;
    const char *paths;
    uint32_t stride, chunk, lo, hi, nq, qstride;
    const uint8_t *qbytes;
    const uint32_t *qlen;
    uint32_t *counts;
    int64_t *rets;
};

static void *wo_worker(void *arg)
{
    struct wo_job *j = (struct wo_job *)arg;
    for (uint32_t f = j->lo; f < j->hi; f++) {
        uint32_t *cnt = j->counts + (uint64_t)f * j->nq;
        for (uint32_t q = 0; q < j->nq; q++) cnt[q] = 0;
        int fd = openat(j->dirfd, j->paths + (uint64_t)f * j->stride, O_RDONLY | O_CLOEXEC);
        if (fd < 0) { j->rets[f] = -errno; continue; }
        uint64_t cap = j->chunk, got = 0;
        uint8_t *buf = (uint8_t *)malloc(cap);
        int64_t err = 0;
        for (;;) {
            if (got + j->chunk > cap) {
                cap = 2 * cap + j->chunk;
                uint8_t *nb = (uint8_t *)realloc(buf, cap);
                if (!nb) { err = -ENOMEM; break; }
                buf = nb;
            }
            ssize_t r = read(fd, buf + got, j->chunk);
            if (r < 0) { err = -errno; break; }
            if (r == 0) break;
            got += (uint64_t)r;
        }
        close(fd);
        if (err) { j->rets[f] = err; free(buf); continue; }
        count_tokens(buf, got, j->qbytes, j->qlen, j->nq, j->qstride, cnt);
        j->rets[f] = (int64_t)got;
        free(buf);
    }
    return NULL;
}

int oracle_wordcount_open(int dirfd, const char *paths, uint32_t nfiles, uint32_t stride,
                          uint32_t chunk, const uint8_t *qbytes, const uint32_t *qlen,
                          uint32_t nq, uint32_t qstride, uint32_t *counts, int64_t *rets,
                          int threads)
{
    if (!chunk) return -EINVAL;
    if (threads < 1) threads = 1;
    if ((uint32_t)threads > nfiles) threads = nfiles ? (int)nfiles : 1;
    pthread_t tid[256];
    struct wo_job jobs[256];
    if (threads > 256) threads = 256;
    for (int t = 0; t < threads; t++) {
        jobs[t] = (struct wo_job){dirfd, paths, stride, chunk,
                                  (uint32_t)((uint64_t)nfiles * t / threads),
                                  (uint32_t)((uint64_t)nfiles * (t + 1) / threads),
                                  nq, qstride, qbytes, qlen, counts, rets};
        if (pthread_create(&tid[t], NULL, wo_worker, &jobs[t]) != 0) return -EAGAIN;
    }
    for (int t = 0; t < threads; t++) pthread_join(tid[t], NULL);
    return 0;
}

/* ---------------------------------------------- stateful write / read back */
/*
 * File round trip with calls whose effect depends on the file offset
 * (read() and write() advance it; section 4.1 and section 8.1 discuss such
 * order-dependent calls): file f is opened beneath dirfd by name, created and
 * truncated, written in `piece`-byte pieces with write(), closed, opened
 * read-only, read back in the same pieces with read() plus one read of 16
 * bytes at the end of the file, and closed.  rets[f * (2K + 5) + i] records
 * every call's result in that order (K = pieces per file); a failed openat
 * ends the file's sequence.  back receives the bytes read (nfiles x
 * file_bytes).  Calls run one at a time per file, files on `threads`
 * threads.
 */
struct rt_job {
    int dirfd;
    const char *paths;
    uint32_t stride, piece, f0, f1;
    const uint8_t *data;
    uint64_t file_bytes;
    int64_t *rets;
    uint8_t *back;
};

static int64_t sysret(int64_t r) { return r < 0 ? -(int64_t)errno : r; }

static void *rt_worker(void *arg)
{
    struct rt_job *j = (struct rt_job *)arg;
    const uint64_t k = (j->file_bytes + j->piece - 1) / j->piece;
    for (uint32_t f = j->f0; f < j->f1; f++) {
        int64_t *r = j->rets + (uint64_t)f * (2 * k + 5);
        const char *path = j->paths + (uint64_t)f * j->stride;
        const uint8_t *src = j->data + (uint64_t)f * j->file_bytes;
        uint8_t *dst = j->back + (uint64_t)f * j->file_bytes;
        uint64_t i = 0;
        int fd = openat(j->dirfd, path, O_WRONLY | O_CREAT | O_TRUNC | O_CLOEXEC, 0600);
        r[i++] = sysret(fd);
        if (fd < 0) continue;
        for (uint64_t p = 0; p < k; p++) {
            uint64_t off = p * j->piece, n = j->file_bytes - off;
            if (n > j->piece) n = j->piece;
            r[i++] = sysret(write(fd, src + off, n));
        }
        r[i++] = sysret(close(fd));
        fd = openat(j->dirfd, path, O_RDONLY | O_CLOEXEC);
        r[i++] = sysret(fd);
        if (fd < 0) continue;
        for (uint64_t p = 0; p < k; p++) {
            uint64_t off = p * j->piece, n = j->file_bytes - off;
            if (n > j->piece) n = j->piece;
            r[i++] = sysret(read(fd, dst + off, n));
        }
        uint8_t tail[16];
        r[i++] = sysret(read(fd, tail, sizeof tail));
        r[i++] = sysret(close(fd));
    }
    return NULL;
}

int oracle_file_roundtrip(int dirfd, const char *paths, uint32_t nfiles, uint32_t stride,
                          const uint8_t *data, uint64_t file_bytes, uint32_t piece,
                          int64_t *rets, uint8_t *back, int threads)
{
    if (!piece) return -EINVAL;
    if (threads < 1) threads = 1;
    if ((uint32_t)threads > nfiles) threads = nfiles ? (int)nfiles : 1;
    if (threads > 256) threads = 256;
    pthread_t tid[256];
    struct rt_job jobs[256];
    for (int t = 0; t < threads; t++) {
        jobs[t] = (struct rt_job){dirfd, paths, stride, piece,
                                  (uint32_t)((uint64_t)nfiles * t / threads),
                                  (uint32_t)((uint64_t)nfiles * (t + 1) / threads),
                                  data, file_bytes, rets, back};
        if (pthread_create(&tid[t], NULL, rt_worker, &jobs[t]) != 0) return -EAGAIN;
    }
    for (int t = 0; t < threads; t++) pthread_join(tid[t], NULL);
    return 0;
}

/* ----------------------------------------------------------- key-value GET */
/*
 * Request datagram (32 B): u64 id; u8 op (1 = GET); u8 pad[7]; u8 key[16].
 * Reply datagram (16 + len B): u64 id; u8 status (0 hit, 1 miss, 2 bad op);
 * u8 pad; u16 len; u32 pad; value[len].
 * The table is a sorted index of the keys, searched with bsearch.
 */
struct kv_index {
    const uint8_t *keys;     /* n x 16 */
    uint32_t *order;         /* indexes sorted by key bytes */
    uint64_t n;
};

static const uint8_t *g_sort_keys;
static int kv_cmp_idx(const void *a, const void *b)
{
    uint32_t x = *(const uint32_t *)a, y = *(const uint32_t *)b;
    return memcmp(g_sort_keys + 16ULL * x, g_sort_keys + 16ULL * y, 16);
}

struct kv_find { const uint8_t *keys; const uint8_t *want; };
static int kv_cmp_key(const void *k, const void *e)
{
    const struct kv_find *f = (const struct kv_find *)k;
    return memcmp(f->want, f->keys + 16ULL * (*(const uint32_t *)e), 16);
}

void *oracle_kv_build(const uint8_t *keys, uint64_t n)
{
    struct kv_index *ix = (struct kv_index *)calloc(1, sizeof *ix);
    if (!ix) return NULL;
    ix->keys = keys;
    ix->n = n;
    ix->order = (uint32_t *)malloc((n ? n : 1) * sizeof(uint32_t));
    if (!ix->order) { free(ix); return NULL; }
    for (uint64_t i = 0; i < n; i++) ix->order[i] = (uint32_t)i;
    g_sort_keys = keys;       /* qsort has no context argument */
    qsort(ix->order, n, sizeof(uint32_t), kv_cmp_idx);
    return ix;
}

void oracle_kv_free(void *h)
{
    struct kv_index *ix = (struct kv_index *)h;
    if (ix) { free(ix->order); free(ix); }
}

int64_t oracle_kv_find(void *h, const uint8_t *key)
{
    struct kv_index *ix = (struct kv_index *)h;
    struct kv_find f = {ix->keys, key};
    const uint32_t *e = (const uint32_t *)bsearch(&f, ix->order, ix->n,
                                                  sizeof(uint32_t), kv_cmp_key);
    return e ? (int64_t)*e : -1;
}

/* Build the reply for one request datagram; returns the reply length. */
uint32_t oracle_kv_reply(void *h, const uint64_t *val_off, const uint32_t *val_len,
                         const uint8_t *heap, const uint8_t *req, uint32_t req_len,
                         uint8_t *reply)
{
    uint64_t id = 0;
    memset(reply, 0, 16);
    if (req_len >= 8) memcpy(&id, req, 8);
    memcpy(reply, &id, 8);
    if (req_len != 32 || req[8] != 1) { reply[8] = 2; return 16; }
    int64_t i = oracle_kv_find(h, req + 16);
    if (i < 0) { reply[8] = 1; return 16; }
    uint16_t len = (uint16_t)val_len[i];
    reply[8] = 0;
    memcpy(reply + 10, &len, 2);
    memcpy(reply + 16, heap + val_off[i], len);
    return 16u + len;
}

/* A CPU UDP server: serve `n_req` datagrams from `sock` (bound by the caller),
 * replying to each sender.  Returns the number served or -errno. */
int64_t oracle_kv_serve(void *h, int sock, const uint64_t *val_off,
                        const uint32_t *val_len, const uint8_t *heap,
                        uint64_t n_req)
{
    uint8_t req[64];
    uint8_t reply[16 + 65536];
    uint64_t served = 0;
    while (served < n_req) {
        struct sockaddr_in from;
        socklen_t fl = sizeof from;
        ssize_t r = recvfrom(sock, req, sizeof req, 0, (struct sockaddr *)&from, &fl);
        if (r < 0) {
            if (errno == EINTR) continue;
            if (errno == EAGAIN || errno == EWOULDBLOCK) return (int64_t)served;
            return -(int64_t)errno;
        }
        uint32_t n = oracle_kv_reply(h, val_off, val_len, heap, req, (uint32_t)r, reply);
        ssize_t s = sendto(sock, reply, n, 0, (struct sockaddr *)&from, fl);
        if (s < 0 && errno != EAGAIN) return -(int64_t)errno;
        served++;
    }
    return (int64_t)served;
}

/* --------------------------------------------------------- memory release */
/*
 * mmap `bytes` of private anonymous memory; write a 64-byte stamp (the bytes
 * stamp[0..63] with the page index xor-ed into byte 0) at the start of every
 * 4 KiB page; read the stamps back into `before` (64 B per page); madvise
 * MADV_DONTNEED; read the same 64 bytes again into `after`; munmap.
 * Returns 0 or -errno of the first failing call.
 */
int oracle_release(uint64_t bytes, const uint8_t *stamp, uint8_t *before,
                   uint8_t *after)
{
    uint64_t pages = bytes / 4096;
    uint8_t *m = (uint8_t *)mmap(NULL, bytes, PROT_READ | PROT_WRITE,
                                 MAP_PRIVATE | MAP_ANONYMOUS, -1, 0);
    if (m == MAP_FAILED) return -errno;
    for (uint64_t p = 0; p < pages; p++) {
        memcpy(m + p * 4096, stamp, 64);
        m[p * 4096] ^= (uint8_t)p;
    }
    for (uint64_t p = 0; p < pages; p++) memcpy(before + p * 64, m + p * 4096, 64);
    if (madvise(m, bytes, MADV_DONTNEED) != 0) { int e = errno; munmap(m, bytes); return -e; }
    for (uint64_t p = 0; p < pages; p++) memcpy(after + p * 64, m + p * 4096, 64);
    if (munmap(m, bytes) != 0) return -errno;
    return 0;
}

/*
 * One memory-release job of the serving mix (section 7.2 uses madvise from
 * the GPU to hand memory back): mmap 2 MiB of private anonymous memory; fill
 * it with pread from the stamp file at stamp_off; pwrite the first 64 bytes
 * of page `page` to out_fd at out_off; madvise(MADV_DONTNEED); pwrite the
 * first 64 bytes of page 0 to out_off + 64; munmap.  The output file then
 * holds the stamp bytes followed by 64 zero bytes (madvise(2): private
 * anonymous pages read back as zeros).  rets[0..5] receive the six return
 * values.  Returns 0 or the first -errno.
 */
int oracle_release_job(int stamp_fd, uint64_t stamp_off, uint32_t page, int out_fd,
                       uint64_t out_off, int64_t *rets)
{
    const uint64_t bytes = 2u << 20;
    uint8_t *m = (uint8_t *)mmap(NULL, bytes, PROT_READ | PROT_WRITE,
                                 MAP_PRIVATE | MAP_ANONYMOUS, -1, 0);
    if (m == MAP_FAILED) { rets[0] = -errno; return (int)rets[0]; }
    rets[0] = 0;
    ssize_t r = pread(stamp_fd, m, bytes, (off_t)stamp_off);
    rets[1] = r < 0 ? -errno : r;
    r = pwrite(out_fd, m + (uint64_t)page * 4096, 64, (off_t)out_off);
    rets[2] = r < 0 ? -errno : r;
    rets[3] = madvise(m, bytes, MADV_DONTNEED) == 0 ? 0 : -errno;
    r = pwrite(out_fd, m, 64, (off_t)(out_off + 64));
    rets[4] = r < 0 ? -errno : r;
    rets[5] = munmap(m, bytes) == 0 ? 0 : -errno;
    for (int i = 0; i < 6; i++)
        if (rets[i] < 0) return (int)rets[i];
    return 0;
}

/* --------------------------------------- block permutation, then pwrite */
/*
 * The ordering / blocking microbenchmark of section 6 (Fig. 6): an array of
 * random values is cut into 8 KiB blocks, each block is permuted `iters`
 * times, and the permuted block is written to a file with pwrite.  The paper
 * likens the permutation to DES's permutation steps and fixes nothing more;
 * here one round maps the block x (1024 little-endian 64-bit words) to y with
 *
 *     bit j of y[i]  =  bit tau[j] of x[sigma[i]]     (i < 1024, j < 64),
 *
 * a shuffle of the words followed by a shuffle of the bits inside each word.
 * sigma and tau are inputs.  Block b is then written with
 * pwrite(fd, block, 8192, file_off + 8192 * b); ret[b] gets its result or
 * -errno.  Blocks are split into contiguous ranges, one per thread.
 */
#define PERM_WORDS 1024

struct pm_job {
    int fd;
    const uint64_t *in;
    const uint16_t *sigma;
    const uint8_t *tau;
    uint32_t iters;
    uint64_t file_off;
    uint64_t lo, hi;
    int64_t *ret;
};

static uint64_t bit_shuffle(uint64_t w, const uint8_t *tau)
{
    uint64_t y = 0;
    for (int j = 0; j < 64; j++)
        y |= ((w >> tau[j]) & 1u) << j;
    return y;
}

static void *pm_worker(void *arg)
{
    struct pm_job *j = (struct pm_job *)arg;
    uint64_t x[PERM_WORDS], y[PERM_WORDS];
    for (uint64_t b = j->lo; b < j->hi; b++) {
        memcpy(x, j->in + b * PERM_WORDS, sizeof x);
        for (uint32_t it = 0; it < j->iters; it++) {
            for (int i = 0; i < PERM_WORDS; i++)
                y[i] = bit_shuffle(x[j->sigma[i]], j->tau);
            memcpy(x, y, sizeof x);
        }
        ssize_t r = pwrite(j->fd, x, sizeof x, (off_t)(j->file_off + b * sizeof x));
        j->ret[b] = r < 0 ? -errno : r;
    }
    return NULL;
}

int oracle_permute(int fd, const uint64_t *in, uint64_t n_blocks, const uint16_t *sigma,
                   const uint8_t *tau, uint32_t iters, uint64_t file_off, int64_t *ret,
                   int threads)
{
    for (int i = 0; i < PERM_WORDS; i++)
        if (sigma[i] >= PERM_WORDS) return -EINVAL;
    for (int j = 0; j < 64; j++)
        if (tau[j] >= 64) return -EINVAL;
    if (threads < 1) threads = 1;
    if ((uint64_t)threads > n_blocks) threads = n_blocks ? (int)n_blocks : 1;
    pthread_t th[256];
    struct pm_job jobs[256];
    if (threads > 256) threads = 256;
    for (int t = 0; t < threads; t++) {
        jobs[t] = (struct pm_job){fd, in, sigma, tau, iters, file_off,
                                  n_blocks * t / threads, n_blocks * (t + 1) / threads, ret};
        if (pthread_create(&th[t], NULL, pm_worker, &jobs[t]) != 0) return -EAGAIN;
    }
    for (int t = 0; t < threads; t++) pthread_join(th[t], NULL);
    return 0;
}
