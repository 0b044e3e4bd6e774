// Word search over files read with GPU-issued pread calls: the wordcount case
// study of section 7.1 (search 64 strings in many files; work-group
// granularity reads).  counts[f][q] = number of tokens of file f equal to
// query q, where a token is a maximal run of bytes other than space and
// newline.
//
// Files are cut into chunks of at most chunk_max bytes.  A chunk is read with
// one pread that also fetches the byte before it (to tell whether the chunk
// starts inside a token) and OVERLAP bytes after it (to finish the last
// token); a token belongs to the chunk in which it starts.  The persistent
// form takes chunks from a device work counter and prefetches the next one.
//
// Each chunk is scanned from LDS in 32 KiB sub-blocks, streamed from host
// staging with fully coalesced 16-byte loads (the next sub-block's loads are
// in flight while the current one is scanned).  Every lane owns a 64-byte
// stretch: it builds a 64-bit delimiter mask with byte-parallel compares,
// walks the token starts in its stretch with count-trailing-zeros, and for a
// token of at most 16 bytes assembles its bytes from aligned LDS words with
// alignbyte.  The (zero-padded) 16 bytes and the length are looked up in an
// LDS hash table of the queries and compared exactly; matches are counted in
// per-wavefront LDS counters and added to counts[file] once per chunk.
#include "gsys_device.hpp"
#include "gsys.h"
#include "kernels.hpp"

#include <fcntl.h>

#include <algorithm>

namespace gsys_ws {

using namespace gsys;

// 512-wide work-groups: each one keeps a 32 KiB sub-block of host staging in
// flight while it scans the previous one.  Fewer, wider groups (64 of them
// with 128 chunk buffers) scan the 2,000-file corpus at 51 GB/s against 47 GB/s
// for 128 groups of 256 with the same bytes in flight.
constexpr uint32_t kWG = 512;
constexpr uint32_t kSeg = 64;                 // bytes scanned per lane per sub-block
constexpr uint32_t kSB = kWG * kSeg;          // 32 KiB sub-block
constexpr uint32_t kOverlap = 16;             // max query length and read-ahead
constexpr uint32_t kHead = 16;                // staging bytes before chunk byte 0
constexpr uint32_t kCopy = kSB + 48;          // LDS bytes per sub-block (look-behind + halo)
constexpr uint32_t kCopyVec = kCopy / 16;     // 16-byte loads per sub-block
constexpr uint32_t kPerLane = (kCopyVec + kWG - 1) / kWG;
constexpr uint32_t kMaxQ = 64;
constexpr uint32_t kTab = 128;                // query hash table slots

struct WsArgs {
  gsys_dev_ctx c;
  const gsys_chunk* chunks;
  const uint8_t* queries;   // nq x 16 bytes
  const uint32_t* qlens;
  uint32_t* counts;         // nfiles x nq
  unsigned int* work;       // device work counter (zeroed per launch)
  uint64_t staging;         // chunk buffers of `cbuf` bytes
  uint32_t cbuf;
  uint32_t n_chunks;
  uint32_t nq;
  uint32_t passes;          // persistent forms: scans of every chunk in one launch
};

struct Shared {
  uint8_t buf[kCopy];
  uint4 qw[kTab];           // query bytes per slot, zero-padded to 16
  uint32_t tkey[kTab];      // hash key per slot; 0 = empty
  int32_t tq[kTab];         // query index | length << 16 per slot
  uint32_t cnt[kWG / 64][kMaxQ];
  uint32_t next;
};

// Key of a token or query: its (zero-padded) 16 bytes and length mixed into
// 32 bits; never 0.  Equal strings have equal keys; a key match is confirmed
// by comparing all 16 bytes and the length.
__device__ __forceinline__ uint32_t token_key(uint4 w, uint32_t len) {
  uint32_t h = len * 0x9e3779b1u;
  h = (h ^ w.x) * 0x85ebca6bu;
  h = (h ^ (h >> 15) ^ w.y) * 0xc2b2ae35u;
  h = (h ^ (h >> 13) ^ w.z) * 0x27d4eb2fu;
  h = (h ^ (h >> 16) ^ w.w) * 0x165667b1u;
  h ^= h >> 15;
  return h | 1u;
}

__device__ __forceinline__ uint32_t mask_bytes(uint32_t x, int32_t keep) {
  // keep the low `keep` bytes of x (keep <= 0: none, >= 4: all)
  return keep >= 4 ? x : (keep <= 0 ? 0u : (x & ((1u << (8 * keep)) - 1u)));
}

__device__ void build_table(const WsArgs& A, Shared& S) {
  for (uint32_t i = threadIdx.x; i < kTab; i += blockDim.x) {
    S.tkey[i] = 0;
    S.tq[i] = -1;
  }
  for (uint32_t i = threadIdx.x; i < (kWG / 64) * kMaxQ; i += blockDim.x) (&S.cnt[0][0])[i] = 0;
  __syncthreads();
  if (threadIdx.x == 0) {
    for (uint32_t q = 0; q < A.nq; ++q) {
      const uint32_t len = A.qlens[q];
      const uint32_t* qp = reinterpret_cast<const uint32_t*>(A.queries + q * 16);
      uint4 w = make_uint4(mask_bytes(qp[0], (int32_t)len), mask_bytes(qp[1], (int32_t)len - 4),
                           mask_bytes(qp[2], (int32_t)len - 8), mask_bytes(qp[3], (int32_t)len - 12));
      const uint32_t k = token_key(w, len);
      uint32_t s = k & (kTab - 1);
      while (S.tkey[s]) s = (s + 1) & (kTab - 1);
      S.tkey[s] = k;
      S.tq[s] = (int32_t)(q | (len << 16));
      S.qw[s] = w;
    }
  }
  __syncthreads();
}

// 4-bit mask of the bytes of x equal to space or newline (bit j = byte j).
__device__ __forceinline__ uint32_t delim4(uint32_t x) {
  auto zero_bytes = [](uint32_t v) {  // 0x80 in every byte of v that is zero
    return ~(((v & 0x7f7f7f7fu) + 0x7f7f7f7fu) | v) & 0x80808080u;
  };
  const uint32_t z = zero_bytes(x ^ 0x20202020u) | zero_bytes(x ^ 0x0a0a0a0au);
  return ((z >> 7) & 1u) | ((z >> 14) & 2u) | ((z >> 21) & 4u) | ((z >> 28) & 8u);
}

// Staging buffer `slot` holds one chunk: byte k of the chunk at kHead + k and
// the byte before the chunk at kHead - 1.  Issue its pread (work-group
// granularity, relaxed: a consumer call, non-blocking).
__device__ Ticket issue_chunk(const WsArgs& A, uint32_t ci, uint64_t slot) {
  const gsys_chunk ch = A.chunks[ci];
  const uint32_t lb = ch.off > 0 ? 1u : 0u;
  const uint64_t dst = A.staging + slot * A.cbuf + kHead - lb;
  Args6 a{{(uint64_t)(int64_t)ch.fd, dst, (uint64_t)ch.len + kOverlap + lb, ch.off - lb, 0, 0}};
  Ticket tk{0, 0, 0};
  call_wg<O::Relaxed, B::NonBlocking>(A.c, GSYS_NR_PREAD64, 0, a, &tk);
  return tk;
}

// Load this lane's share of the sub-block at staging byte sb0 (bytes
// [sb0, sb0 + kCopy) from stg) into registers.  Only 16-byte vectors that lie
// inside the buffer (`lim` bytes from stg) and start before `data` (the end of
// the bytes the call returned) cross the host link; the rest read as spaces,
// which the scan treats as delimiters, as it does every position past the
// valid extent.
__device__ __forceinline__ void load_sub(const uint8_t* stg, uint32_t lim, uint32_t data,
                                         uint32_t sb0, uint4 (&v)[kPerLane]) {
#pragma unroll
  for (uint32_t k = 0; k < kPerLane; ++k) {
    const uint32_t i = threadIdx.x + k * kWG;
    v[k] = make_uint4(0x20202020u, 0x20202020u, 0x20202020u, 0x20202020u);
    if (i < kCopyVec && sb0 + i * 16 + 16 <= lim && sb0 + i * 16 < data)
      v[k] = to_uint4(ldg16((uint64_t)(stg + sb0 + i * 16)));
  }
}

// Count the tokens that start at range positions [0, own) into
// counts[file].  Range position p is staging byte stg[kHead + p]; `ext`
// bytes from position 0 on are valid (later ones count as delimiters);
// stg[kHead - 1] is the byte before position 0 when lb_ok (else position 0
// starts a token if it is not a delimiter).  `lim` bytes from stg on lie in
// the buffer.
__device__ void scan_range(const WsArgs& A, Shared& S, uint32_t file, const uint8_t* stg,
                           uint32_t lim, uint32_t own_total, int64_t ext, bool lb_ok) {
  const uint32_t wave = threadIdx.x >> 6;
  // staging bytes that hold data: the look-behind byte and positions < ext
  const uint32_t data = (uint32_t)min<int64_t>((int64_t)lim, (int64_t)kHead + max<int64_t>(ext, 0));
  uint4 v[kPerLane];
  if (own_total) load_sub(stg, lim, data, 0, v);
  for (uint32_t sb0 = 0; sb0 < own_total; sb0 += kSB) {
    // LDS buf[i] = staging[sb0 + i], i.e. chunk position sb0 + i - kHead
#pragma unroll
    for (uint32_t k = 0; k < kPerLane; ++k) {
      const uint32_t i = threadIdx.x + k * kWG;
      if (i < kCopyVec) *reinterpret_cast<uint4*>(S.buf + i * 16) = v[k];
    }
    __syncthreads();
    if (sb0 + kSB < own_total) load_sub(stg, lim, data, sb0 + kSB, v);  // in flight during the scan
    const int64_t sb_ext = ext - (int64_t)sb0;                    // valid positions: p < sb_ext
    const uint32_t own = min(kSB, own_total - sb0);               // tokens may start at p < own
    const uint32_t p0 = threadIdx.x * kSeg;
    if (p0 < own) {
      // delimiter masks: bit i of dlo = position p0 + i, bit i of dhi =
      // position p0 + 64 + i (read-ahead); bytes past the valid extent count
      // as delimiters, and so does position 80 (a sentinel)
      const uint32_t* bw = reinterpret_cast<const uint32_t*>(S.buf + kHead + p0);
      uint64_t dlo = 0;
      uint32_t dhi = 0;
#pragma unroll
      for (uint32_t d = 0; d < 16; ++d) dlo |= (uint64_t)delim4(bw[d]) << (4 * d);
#pragma unroll
      for (uint32_t d = 0; d < 4; ++d) dhi |= delim4(bw[16 + d]) << (4 * d);
      const int64_t vlen = sb_ext - (int64_t)p0;  // valid bytes from p0 on
      if (vlen < 64) dlo |= vlen <= 0 ? ~0ull : (~0ull << vlen);
      if (vlen < 80) dhi |= vlen <= 64 ? 0xffffu : (0xffffu << (vlen - 64));
      dhi |= 1u << 16;
      uint32_t prev_delim;  // position p0 - 1
      if (sb0 == 0 && p0 == 0) prev_delim = lb_ok ? (delim4(S.buf[kHead - 1]) & 1u) : 1u;
      else if ((int64_t)p0 - 1 >= sb_ext) prev_delim = 1u;
      else prev_delim = delim4(S.buf[kHead + p0 - 1]) & 1u;
      const uint32_t own_n = min(kSeg, own - p0);
      const uint64_t own_mask = own_n >= 64 ? ~0ull : ((1ull << own_n) - 1ull);
      uint64_t starts = ~dlo & ((dlo << 1) | prev_delim) & own_mask;
      while (starts) {
        const uint32_t s = (uint32_t)__builtin_ctzll(starts);
        starts &= starts - 1;
        // first delimiter at or after s
        const uint64_t after = s < 64 ? (dlo >> s) : 0ull;
        uint32_t len;
        if (after) len = (uint32_t)__builtin_ctzll(after);
        else len = (64 - s) + (uint32_t)__builtin_ctz(dhi);
        if (len > kOverlap) continue;
        // the token's bytes, from aligned LDS words
        const uint32_t bpos = kHead + p0 + s;
        const uint32_t* aw = reinterpret_cast<const uint32_t*>(S.buf + (bpos & ~3u));
        const uint32_t sh = bpos & 3u;
        const uint32_t a0 = aw[0], a1 = aw[1], a2 = aw[2], a3 = aw[3], a4 = aw[4];
        uint4 w = make_uint4(__builtin_amdgcn_alignbyte(a1, a0, sh),
                             __builtin_amdgcn_alignbyte(a2, a1, sh),
                             __builtin_amdgcn_alignbyte(a3, a2, sh),
                             __builtin_amdgcn_alignbyte(a4, a3, sh));
        w.x = mask_bytes(w.x, (int32_t)len);
        w.y = mask_bytes(w.y, (int32_t)len - 4);
        w.z = mask_bytes(w.z, (int32_t)len - 8);
        w.w = mask_bytes(w.w, (int32_t)len - 12);
        const uint32_t k = token_key(w, len);
        uint32_t t = k & (kTab - 1);
        for (uint32_t n = 0; n < kTab; ++n) {
          const uint32_t tk = S.tkey[t];
          if (!tk) break;
          if (tk == k) {
            const uint4 q = S.qw[t];
            const int32_t tq = S.tq[t];
            if (q.x == w.x && q.y == w.y && q.z == w.z && q.w == w.w &&
                (uint32_t)(tq >> 16) == len) {
              atomicAdd(&S.cnt[wave][tq & 0xffff], 1u);
              break;
            }
          }
          t = (t + 1) & (kTab - 1);
        }
      }
    }
    __syncthreads();
  }
  // flush this chunk's counts
  for (uint32_t q = threadIdx.x; q < A.nq; q += blockDim.x) {
    uint32_t v = 0;
#pragma unroll
    for (uint32_t w = 0; w < kWG / 64; ++w) {
      v += S.cnt[w][q];
      S.cnt[w][q] = 0;
    }
    if (v) atomicAdd(&A.counts[(uint64_t)file * A.nq + q], v);
  }
  __syncthreads();
}

__device__ void scan_chunk(const WsArgs& A, Shared& S, uint32_t ci, uint64_t slot, int64_t ret) {
  const gsys_chunk ch = A.chunks[ci];
  const uint32_t lb = ch.off > 0 ? 1u : 0u;
  // bytes available at chunk positions >= 0 (chunk + read-ahead, EOF-bounded)
  const int64_t ext = ret > (int64_t)lb ? ret - (int64_t)lb : 0;
  const bool lb_ok = lb && ret >= 1;
  const uint8_t* stg = reinterpret_cast<const uint8_t*>(A.staging) + slot * A.cbuf;
  scan_range(A, S, ch.file, stg, A.cbuf, ch.len, ext, lb_ok);
}

// The next work item for the whole work-group.  The leading barrier closes
// whatever thread-0-only code ran before it (a weak blocking call's wait, a
// result store): without it such code joins the atomic below into one
// thread-0 region across the loop's back edge, and the compiled loop then
// lets the other work-items of thread 0's wavefront pass the barrier below
// before thread 0 has taken the item, read a stale S.next, and never leave
// the loop.
__device__ __forceinline__ uint32_t grab(const WsArgs& A, Shared& S) {
  __syncthreads();
  if (threadIdx.x == 0) S.next = atomicAdd(A.work, 1u);
  __syncthreads();
  const uint32_t v = S.next;
  __syncthreads();
  return v;
}

// Persistent form: work items come from a device work counter; the pread of
// the next one is issued before the current one is scanned.  Work item w is
// chunk w mod n_chunks of pass w / n_chunks: with several passes the
// work-groups go from one pass to the next without draining, and each pass
// adds its counts.
__global__ __launch_bounds__(kWG) void wordscan_persistent(WsArgs A) {
  __shared__ Shared S;
  build_table(A, S);
  const uint32_t total = A.n_chunks * A.passes;
  uint32_t cur = grab(A, S);
  if (cur >= total) return;
  uint32_t bi = 0;
  Ticket tk = issue_chunk(A, cur % A.n_chunks, (uint64_t)blockIdx.x * 2 + bi);
  for (;;) {
    const uint32_t nxt = grab(A, S);
    Ticket tkn{0, 0, 0};
    if (nxt < total)
      tkn = issue_chunk(A, nxt % A.n_chunks, (uint64_t)blockIdx.x * 2 + (bi ^ 1u));
    const int64_t r = wait_wg(A.c, tk);
    scan_chunk(A, S, cur % A.n_chunks, (uint64_t)blockIdx.x * 2 + bi, r);
    if (nxt >= total) break;
    cur = nxt;
    tk = tkn;
    bi ^= 1u;
  }
}

// Plain form: one work-group per chunk, blocking relaxed work-group call
// (the paper's wordcount setting: work-group granularity, blocking, weak).
__global__ __launch_bounds__(kWG) void wordscan_plain(WsArgs A) {
  __shared__ Shared S;
  build_table(A, S);
  const uint32_t ci = blockIdx.x;
  if (ci >= A.n_chunks) return;
  const gsys_chunk ch = A.chunks[ci];
  const uint32_t lb = ch.off > 0 ? 1u : 0u;
  const uint64_t dst = A.staging + (uint64_t)ci * A.cbuf + kHead - lb;
  Args6 a{{(uint64_t)(int64_t)ch.fd, dst, (uint64_t)ch.len + kOverlap + lb, ch.off - lb, 0, 0}};
  const int64_t r = call_wg<O::Relaxed, B::Blocking>(A.c, GSYS_NR_PREAD64, 0, a);
  scan_chunk(A, S, ci, ci, r);
}

// ---------------------------------------------------------------------------
// The wordcount as the case study issues it (section 7.1): each work-group
// takes a file, opens it by name, reads it front to back with read() (the
// file offset advances on the host), scans the pieces and closes the file.
// Reads are sequential, so there is no read-ahead: a piece owns the tokens
// that start before its last kOverlap bytes, and those bytes, with the byte
// before them, are carried in front of the next piece (the next read is
// already in flight into the other buffer while this piece is scanned).  A
// read shorter than asked, or of 0 bytes, ends the file (a regular file).
//
// Piece buffer layout: [0, kOpenHead) carry, data from kOpenHead on.  The
// carry's 16 bytes sit at [kOpenHead - 16, kOpenHead), the byte before them
// at kOpenHead - 17, each piece's data on a fresh 64-byte line.

constexpr uint32_t kOpenHead = 64;
constexpr uint32_t kCarry = kOverlap;  // deferred bytes

struct WoArgs {
  WsArgs w;             // queries, counts, staging (2 buffers of w.cbuf per group)
  uint64_t paths;       // registered host buffer: nfiles x GSYS_PATH_MAX bytes
  int64_t* file_ret;    // device: bytes read per file, or -errno
  uint64_t progress;    // host-visible: 2 x u64 per work-group, or 0
  uint32_t nfiles;
  uint32_t chunk;       // bytes per read()
  int32_t dirfd;
};

// Where a work-group is (thread 0 only): word 0 = (file + 1) << 32 | phase,
// word 1 = piece << 32 | low 32 bits of the last call's ticket.  Written
// with system-scope stores, so the host can read it while the kernel runs.
enum : uint32_t { kPhOpen = 1, kPhRead = 2, kPhScan = 3, kPhClose = 4, kPhDone = 5 };
__device__ __forceinline__ void progress(const WoArgs& A, uint32_t f, uint32_t phase,
                                         uint32_t piece, uint64_t ticket) {
  if (!A.progress || threadIdx.x != 0) return;
  uint64_t* p = reinterpret_cast<uint64_t*>(A.progress) + 2ull * blockIdx.x;
  st_sys(p + 1, ((uint64_t)piece << 32) | (uint32_t)ticket);
  st_sys(p, ((uint64_t)(f + 1) << 32) | phase);
}

__device__ void open_and_scan(const WoArgs& A, Shared& S, uint32_t f) {
  const gsys_dev_ctx& c = A.w.c;
  const uint64_t base = A.w.staging + (uint64_t)blockIdx.x * 2 * A.w.cbuf;
  progress(A, f, kPhOpen, 0, 0);
  // openat: a consumer call, blocking: every work-item needs the descriptor
  const int64_t fd = call_wg<O::Relaxed, B::Blocking>(
      c, GSYS_NR_OPENAT, 0,
      Args6{{(uint64_t)(int64_t)A.dirfd, A.paths + (uint64_t)f * GSYS_PATH_MAX,
             (uint64_t)O_RDONLY, 0, 0, 0}});
  if (fd < 0) {
    if (threadIdx.x == 0) A.file_ret[f] = fd;
    return;
  }
  auto issue = [&](uint32_t b) {
    Ticket tk{0, 0, 0};
    call_wg<O::Relaxed, B::NonBlocking>(
        c, GSYS_NR_READ, 0,
        Args6{{(uint64_t)fd, base + b * A.w.cbuf + kOpenHead, A.chunk, 0, 0, 0}}, &tk);
    return tk;
  };
  int64_t total = 0, err = 0;
  uint32_t b = 0, piece = 0;
  bool first = true;
  Ticket tk = issue(0);
  for (;;) {
    progress(A, f, kPhRead, piece, tk.t);
    const int64_t r = wait_wg(c, tk);
    if (r < 0) {
      err = r;
      break;
    }
    const bool end = (uint64_t)r < A.chunk;
    const uint64_t buf = base + b * A.w.cbuf;
    if (!end) {
      // carry this piece's last kCarry + 1 bytes in front of the next one,
      // then start reading it
      const uint64_t nb = base + (b ^ 1u) * A.w.cbuf;
      if (threadIdx.x <= kCarry)
        gp<uint8_t>(nb + kOpenHead - kCarry - 1)[threadIdx.x] =
            gp<const uint8_t>(buf + kOpenHead + (uint64_t)r - kCarry - 1)[threadIdx.x];
      tk = issue(b ^ 1u);
    }
    // the range: the carry (none for the first piece), then the data
    const uint32_t carry = first ? 0u : kCarry;
    const int64_t ext = (int64_t)carry + r;
    const uint32_t own = end ? (uint32_t)ext : (uint32_t)(ext - kCarry);
    const uint32_t p0 = kOpenHead - carry;  // buffer byte of range position 0
    progress(A, f, kPhScan, piece, tk.t);
    scan_range(A.w, S, f, reinterpret_cast<const uint8_t*>(buf + p0 - kHead),
               A.w.cbuf - (p0 - kHead), own, ext, !first);
    total += r;
    if (end) break;
    b ^= 1u;
    first = false;
    ++piece;
  }
  // close: a producer call (every work-item is done with the descriptor);
  // the designated caller records the file's result
  progress(A, f, kPhClose, piece, 0);
  const int64_t rc = call_wg<O::Relaxed, B::Blocking>(c, GSYS_NR_CLOSE, 0,
                                                      Args6{{(uint64_t)fd, 0, 0, 0, 0, 0}});
  if (threadIdx.x == 0) A.file_ret[f] = err ? err : (rc < 0 ? rc : total);
}

__global__ __launch_bounds__(kWG) void wordopen_persistent(WoArgs A) {
  __shared__ Shared S;
  build_table(A.w, S);
  uint32_t last = ~0u;
  for (;;) {
    // grab() opens with a barrier: the thread-0-only result store that ends
    // open_and_scan never shares a region with the next grab's atomic
    const uint32_t f = grab(A.w, S);
    if (f >= A.nfiles) break;
    open_and_scan(A, S, f);
    last = f;
  }
  progress(A, last, kPhDone, 0, 0);
}

__global__ void zero_u32(uint32_t* p, uint64_t n) {
  for (uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n;
       i += (uint64_t)gridDim.x * blockDim.x)
    p[i] = 0;
}

}  // namespace gsys_ws

using namespace gsys_ws;

int gsys_wordscan(gsys_ctx* ctx, uint64_t chunks, uint32_t n_chunks, uint32_t chunk_max,
                  uint64_t queries, uint64_t qlens, uint32_t nq, uint64_t counts, uint32_t nfiles,
                  uint64_t staging, uint64_t staging_bytes, uint32_t form, uint32_t passes,
                  void* stream) {
  // no chunks (every file empty, or no files) only zeroes the counts
  if (!ctx || (!chunks && n_chunks) || !queries || !qlens || !counts) return -EINVAL;
  if (passes == 0 || (form == GSYS_PLAIN && passes != 1) ||
      (uint64_t)n_chunks * passes > 0xffffffffull)
    return -EINVAL;
  if (nq == 0 || nq > kMaxQ || chunk_max == 0 || chunk_max > (64u << 20)) return -EINVAL;
  const uint32_t cbuf = (chunk_max + 64 + 15) & ~15u;
  if (gsys_internal::check_host_range(ctx, staging, staging_bytes)) return -EFAULT;
  const uint64_t per_wg = 2ull * cbuf;
  hipStream_t s = (hipStream_t)stream;
  WsArgs A;
  if (int e = gsys_device_ctx(ctx, &A.c)) return e;
  A.chunks = (const gsys_chunk*)chunks;
  A.queries = (const uint8_t*)queries;
  A.qlens = (const uint32_t*)qlens;
  A.counts = (uint32_t*)counts;
  A.work = (unsigned int*)gsys_internal::kstate(ctx) + 8;
  A.staging = staging;
  A.cbuf = cbuf;
  A.n_chunks = n_chunks;
  A.nq = nq;
  A.passes = passes;
  if (form != GSYS_PLAIN && form != GSYS_PERSISTENT && form != GSYS_GRAPH) return -EINVAL;
  // zero the counts and the work counter, then scan
  uint64_t ncount = (uint64_t)nfiles * nq;
  uint64_t nwork = 2;
  uint32_t* counts32 = (uint32_t*)counts;
  uint32_t* work32 = (uint32_t*)A.work;
  void* zc_args[] = {&counts32, &ncount};
  void* zw_args[] = {&work32, &nwork};
  void* args[] = {&A};
  const dim3 zc_grid((uint32_t)std::max<uint64_t>(1, std::min<uint64_t>((ncount + 255) / 256, 4096)));
  gsys_internal::KLaunch k[3] = {{(const void*)zero_u32, zc_grid, dim3(256), 0, zc_args},
                                 {(const void*)zero_u32, dim3(1), dim3(64), 0, zw_args},
                                 {nullptr, dim3(1), dim3(kWG), 0, args}};
  if (form == GSYS_PLAIN) {
    if (n_chunks && staging_bytes < (uint64_t)cbuf * n_chunks) return -EINVAL;
    k[2].kernel = (const void*)wordscan_plain;
    k[2].grid = dim3(n_chunks);
  } else {
    if (n_chunks && staging_bytes < per_wg) return -EINVAL;
    uint32_t grid = gsys_internal::resident_grid(ctx, (const void*)wordscan_persistent, kWG, 0);
    if (!grid) return -ENODEV;
    grid = (uint32_t)std::min<uint64_t>(
        {(uint64_t)grid, staging_bytes / per_wg, (uint64_t)n_chunks * passes});
    const uint32_t req = gsys_internal::persistent_grid_override(ctx);
    if (req && req < grid) grid = req;
    k[2].kernel = (const void*)wordscan_persistent;
    k[2].grid = dim3(grid);
  }
  if (form == GSYS_GRAPH && n_chunks) {
    // one graph per shape: both fills and the scan, replayed with this
    // call's arguments
    const uint64_t key = gsys_internal::hash_words(
        {0x3C5ull, zc_grid.x, k[2].grid.x});
    return gsys_internal::launch_graph(ctx, key, k, 3, s);
  }
  for (uint32_t i = 0; i < 3; ++i) {
    if (i == 2 && !n_chunks) break;
    if (int e = gsys_internal::launch(ctx, k[i].kernel, k[i].grid.x, k[i].block.x, 0, k[i].args, s))
      return e;
  }
  return 0;
}

uint64_t gsys_wordcount_open_buffer_bytes(uint32_t chunk) {
  return ((uint64_t)kOpenHead + chunk + kCopy + 15) & ~15ull;
}

int gsys_wordcount_open(gsys_ctx* ctx, int dirfd, uint64_t paths, uint32_t nfiles,
                        uint64_t queries, uint64_t qlens, uint32_t nq, uint64_t counts,
                        uint64_t file_ret, uint32_t chunk, uint64_t staging,
                        uint64_t staging_bytes, uint64_t progress, uint32_t progress_groups,
                        void* stream) {
  if (!ctx) return -EINVAL;
  if (nq == 0 || nq > kMaxQ) return -EINVAL;
  if (chunk < 64 || chunk % 64 || chunk > (64u << 20)) return -EINVAL;
  if (!nfiles) return 0;  // the outputs are empty and may be null
  if (!queries || !qlens || !counts || !file_ret) return -EINVAL;
  if (gsys_internal::check_host_range(ctx, paths, (uint64_t)nfiles * GSYS_PATH_MAX)) return -EFAULT;
  // carry head + data + the scanner's window past the last valid byte
  const uint32_t cbuf = (uint32_t)gsys_wordcount_open_buffer_bytes(chunk);
  const uint64_t per_wg = 2ull * cbuf;
  if (staging_bytes < per_wg) return -EINVAL;
  if (gsys_internal::check_host_range(ctx, staging, staging_bytes)) return -EFAULT;
  if (progress && (!progress_groups ||
                   gsys_internal::check_host_range(ctx, progress, 16ull * progress_groups)))
    return progress_groups ? -EFAULT : -EINVAL;
  hipStream_t s = (hipStream_t)stream;
  WoArgs A;
  if (int e = gsys_device_ctx(ctx, &A.w.c)) return e;
  A.w.chunks = nullptr;
  A.w.queries = (const uint8_t*)queries;
  A.w.qlens = (const uint32_t*)qlens;
  A.w.counts = (uint32_t*)counts;
  A.w.work = (unsigned int*)gsys_internal::kstate(ctx) + 8;
  A.w.staging = staging;
  A.w.cbuf = cbuf;
  A.w.n_chunks = 0;
  A.w.passes = 1;
  A.w.nq = nq;
  A.paths = paths;
  A.file_ret = (int64_t*)file_ret;
  A.nfiles = nfiles;
  A.chunk = chunk;
  A.dirfd = dirfd;
  const uint64_t ncount = (uint64_t)nfiles * nq;
  if (gsys_internal::no_device(ctx)) return -ENODEV;
  hipLaunchKernelGGL(zero_u32, dim3((uint32_t)std::min<uint64_t>((ncount + 255) / 256, 4096)),
                     dim3(256), 0, s, (uint32_t*)counts, ncount);
  hipLaunchKernelGGL(zero_u32, dim3(1), dim3(64), 0, s, (uint32_t*)A.w.work, (uint64_t)2);
  if (hipGetLastError() != hipSuccess) return -ENODEV;
  uint32_t grid = gsys_internal::resident_grid(ctx, (const void*)wordopen_persistent, kWG, 0);
  if (!grid) return -ENODEV;
  grid = (uint32_t)std::min<uint64_t>({(uint64_t)grid, staging_bytes / per_wg, (uint64_t)nfiles});
  const uint32_t req = gsys_internal::persistent_grid_override(ctx);
  if (req && req < grid) grid = req;
  if (progress && progress_groups < grid) grid = progress_groups;  // one record per work-group
  A.progress = progress;
  void* args[] = {&A};
  return gsys_internal::launch(ctx, (const void*)wordopen_persistent, grid, kWG, 0, args, s);
}
