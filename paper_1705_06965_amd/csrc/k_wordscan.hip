// Word search over files read with GPU-issued pread calls: the wordcount case
// study of section 7.1 (search 64 strings in many files; work-group
// granularity reads).  counts[f][q] = number of tokens of file f equal to
// query q, where a token is a maximal run of bytes other than space and
// newline.
//
// Files are cut into chunks of at most chunk_max bytes.  A chunk is read with
// one pread that also fetches the byte before it (to tell whether the chunk
// starts inside a token) and OVERLAP bytes after it (to finish the last
// token); a token belongs to the chunk in which it starts.  Chunks are taken
// from a device work counter.  Each chunk is scanned from LDS: the work-group
// streams 16 KiB sub-blocks of host staging into LDS with fully coalesced
// 16-byte loads, every lane scans a 64-byte stretch (finishing the token it
// opened past the stretch), and a completed token of at most OVERLAP bytes
// is looked up in an LDS hash table of the queries by FNV-1a-64 and confirmed
// byte by byte; matches are counted with LDS atomics and flushed per chunk.
#include "gsys_device.hpp"
#include "gsys.h"
#include "kernels.hpp"

#include <algorithm>

namespace gsys_ws {

using namespace gsys;

constexpr uint32_t kWG = 256;
constexpr uint32_t kSeg = 64;                 // bytes scanned per lane per sub-block
constexpr uint32_t kSB = kWG * kSeg;          // 16 KiB sub-block
constexpr uint32_t kOverlap = 16;             // max query length and read-ahead
constexpr uint32_t kHead = 16;                // staging bytes before chunk byte 0
constexpr uint32_t kCopy = kSB + 48;          // LDS bytes per sub-block (look-behind + halo)
constexpr uint32_t kMaxQ = 64;
constexpr uint32_t kTab = 128;                // query hash table slots

__device__ __forceinline__ bool is_delim(uint32_t b) { return b == 0x20u || b == 0x0au; }

__device__ __forceinline__ uint64_t fnv_byte(uint64_t h, uint32_t byte) {
  h ^= byte;
  return (h << 40) + h * 0x1b3ull;
}

struct WsArgs {
  gsys_dev_ctx c;
  const gsys_chunk* chunks;
  const uint8_t* queries;   // nq x 16 bytes
  const uint32_t* qlens;
  uint32_t* counts;         // nfiles x nq
  unsigned int* work;       // device work counter (zeroed per launch)
  uint64_t staging;         // 2 buffers per work-group of `cbuf` bytes
  uint32_t cbuf;
  uint32_t n_chunks;
  uint32_t nq;
};

struct Shared {
  uint8_t buf[kCopy];
  uint64_t thash[kTab];
  int32_t tq[kTab];
  uint8_t qb[kMaxQ * 16];
  uint32_t ql[kMaxQ];
  uint32_t cnt[kMaxQ];
  uint32_t next;
};

__device__ void build_table(const WsArgs& A, Shared& S) {
  for (uint32_t i = threadIdx.x; i < kMaxQ * 16 / 4; i += blockDim.x)
    reinterpret_cast<uint32_t*>(S.qb)[i] =
        i * 4 < A.nq * 16 ? reinterpret_cast<const uint32_t*>(A.queries)[i] : 0u;
  for (uint32_t i = threadIdx.x; i < kMaxQ; i += blockDim.x) {
    S.ql[i] = i < A.nq ? A.qlens[i] : 0u;
    S.cnt[i] = 0;
  }
  for (uint32_t i = threadIdx.x; i < kTab; i += blockDim.x) S.tq[i] = -1;
  __syncthreads();
  if (threadIdx.x == 0) {
    for (uint32_t q = 0; q < A.nq; ++q) {
      uint64_t h = 0xcbf29ce484222325ull;
      for (uint32_t k = 0; k < S.ql[q]; ++k) h = fnv_byte(h, S.qb[q * 16 + k]);
      uint32_t s = (uint32_t)(h ^ (h >> 29)) & (kTab - 1);
      while (S.tq[s] >= 0) s = (s + 1) & (kTab - 1);
      S.tq[s] = (int32_t)q;
      S.thash[s] = h;
    }
  }
  __syncthreads();
}

// token [start, start + len) of the LDS buffer (buffer index, not position)
__device__ __forceinline__ void probe(Shared& S, uint64_t h, uint32_t len, uint32_t start) {
  uint32_t s = (uint32_t)(h ^ (h >> 29)) & (kTab - 1);
  for (uint32_t n = 0; n < kTab; ++n) {
    const int32_t q = S.tq[s];
    if (q < 0) return;
    if (S.thash[s] == h && S.ql[q] == len) {
      bool eq = true;
      for (uint32_t k = 0; k < len; ++k) eq &= S.buf[start + k] == S.qb[q * 16 + k];
      if (eq) {
        atomicAdd(&S.cnt[q], 1u);
        return;
      }
    }
    s = (s + 1) & (kTab - 1);
  }
}

// Issue the pread of chunk `ci` into staging buffer `slot` (work-group
// granularity, relaxed: a consumer call, non-blocking).  The buffer holds
// byte k of the chunk at kHead + k and the byte before the chunk at
// kHead - 1.
__device__ Ticket issue_chunk(const WsArgs& A, uint32_t ci, uint64_t slot) {
  const gsys_chunk ch = A.chunks[ci];
  const uint32_t lb = ch.off > 0 ? 1u : 0u;
  const uint64_t dst = A.staging + slot * A.cbuf + kHead - lb;
  Args6 a{{(uint64_t)(int64_t)ch.fd, dst, (uint64_t)ch.len + kOverlap + lb, ch.off - lb, 0, 0}};
  Ticket tk{0, 0, 0};
  call_wg<O::Relaxed, B::NonBlocking>(A.c, GSYS_NR_PREAD64, 0, a, &tk);
  return tk;
}

__device__ void scan_chunk(const WsArgs& A, Shared& S, uint32_t ci, uint64_t slot, int64_t ret) {
  const gsys_chunk ch = A.chunks[ci];
  const uint32_t lb = ch.off > 0 ? 1u : 0u;
  // bytes available at chunk positions >= 0 (chunk + read-ahead, EOF-bounded)
  const int64_t ext = ret > (int64_t)lb ? ret - (int64_t)lb : 0;
  const bool lb_ok = lb && ret >= 1;
  const uint8_t* stg = reinterpret_cast<const uint8_t*>(A.staging) + slot * A.cbuf;
  for (uint32_t sb0 = 0; sb0 < ch.len; sb0 += kSB) {
    // LDS buf[i] = staging[sb0 + i], i.e. chunk position sb0 + i - kHead
    for (uint32_t i = threadIdx.x; i < kCopy / 16; i += blockDim.x) {
      uint4 v = make_uint4(0x20202020u, 0x20202020u, 0x20202020u, 0x20202020u);
      if (sb0 + i * 16 + 16 <= A.cbuf) v = *reinterpret_cast<const uint4*>(stg + sb0 + i * 16);
      *reinterpret_cast<uint4*>(S.buf + i * 16) = v;
    }
    __syncthreads();
    const int64_t sb_ext = ext - (int64_t)sb0;                   // valid positions: p < sb_ext
    const uint32_t own = min(kSB, ch.len - sb0);                 // tokens may start at p < own
    const uint32_t p0 = threadIdx.x * kSeg;
    if (p0 < own) {
      const uint32_t own_end = min(p0 + kSeg, own);
      auto byte_at = [&](int64_t p) -> uint32_t {
        if (p < 0) return (sb0 == 0 && !lb_ok) ? 0x20u : S.buf[kHead + p];
        return p < sb_ext ? S.buf[kHead + p] : 0x20u;
      };
      bool skip = !is_delim(byte_at((int64_t)p0 - 1));  // a token that started before p0
      uint32_t len = 0, start = 0;
      uint64_t h = 0;
      for (uint32_t p = p0; p < own_end + kOverlap; ++p) {
        if (p >= own_end && len == 0 && !skip) break;
        const uint32_t b = byte_at(p);
        if (is_delim(b)) {
          if (len && !skip && len <= kOverlap) probe(S, h, len, kHead + start);
          skip = false;
          len = 0;
          if (p >= own_end) break;
        } else if (skip) {
          // still inside the previous stretch's token
        } else {
          if (len == 0) {
            if (p >= own_end) break;
            h = 0xcbf29ce484222325ull;
            start = p;
          }
          h = fnv_byte(h, b);
          ++len;
        }
      }
    }
    __syncthreads();
  }
  // flush this chunk's counts
  for (uint32_t q = threadIdx.x; q < A.nq; q += blockDim.x) {
    const uint32_t v = S.cnt[q];
    if (v) atomicAdd(&A.counts[(uint64_t)ch.file * A.nq + q], v);
    S.cnt[q] = 0;
  }
  __syncthreads();
}

__device__ __forceinline__ uint32_t grab(const WsArgs& A, Shared& S) {
  if (threadIdx.x == 0) S.next = atomicAdd(A.work, 1u);
  __syncthreads();
  const uint32_t v = S.next;
  __syncthreads();
  return v;
}

// Persistent form: chunks come from a device work counter; the pread of the
// next chunk is issued before the current one is scanned.
__global__ __launch_bounds__(kWG) void wordscan_persistent(WsArgs A) {
  __shared__ Shared S;
  build_table(A, S);
  uint32_t cur = grab(A, S);
  if (cur >= A.n_chunks) return;
  uint32_t bi = 0;
  Ticket tk = issue_chunk(A, cur, (uint64_t)blockIdx.x * 2 + bi);
  for (;;) {
    const uint32_t nxt = grab(A, S);
    Ticket tkn{0, 0, 0};
    if (nxt < A.n_chunks) tkn = issue_chunk(A, nxt, (uint64_t)blockIdx.x * 2 + (bi ^ 1u));
    const int64_t r = wait_wg(A.c, tk);
    scan_chunk(A, S, cur, (uint64_t)blockIdx.x * 2 + bi, r);
    if (nxt >= A.n_chunks) break;
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

__global__ void zero_u32(uint32_t* p, uint64_t n) {
  for (uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n;
       i += (uint64_t)gridDim.x * blockDim.x)
    p[i] = 0;
}

}  // namespace gsys_ws

using namespace gsys_ws;

int gsys_wordscan(gsys_ctx* ctx, uint64_t chunks, uint32_t n_chunks, uint32_t chunk_max,
                  uint64_t queries, uint64_t qlens, uint32_t nq, uint64_t counts, uint32_t nfiles,
                  uint64_t staging, uint64_t staging_bytes, uint32_t form, void* stream) {
  if (!ctx || !chunks || !queries || !qlens || !counts) return -EINVAL;
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
  const uint64_t ncount = (uint64_t)nfiles * nq;
  if (ncount) {
    hipLaunchKernelGGL(zero_u32, dim3((uint32_t)std::min<uint64_t>((ncount + 255) / 256, 4096)),
                       dim3(256), 0, s, (uint32_t*)counts, ncount);
  }
  hipLaunchKernelGGL(zero_u32, dim3(1), dim3(64), 0, s, (uint32_t*)A.work, (uint64_t)2);
  if (hipGetLastError() != hipSuccess) return -ENODEV;
  if (!n_chunks) return 0;
  void* args[] = {&A};
  if (form == GSYS_PLAIN) {
    if (staging_bytes < (uint64_t)cbuf * n_chunks) return -EINVAL;
    return gsys_internal::launch(ctx, (const void*)wordscan_plain, n_chunks, kWG, 0, args, s);
  }
  if (form != GSYS_PERSISTENT && form != GSYS_GRAPH) return -EINVAL;
  if (staging_bytes < per_wg) return -EINVAL;
  uint32_t grid = gsys_internal::resident_grid(ctx, (const void*)wordscan_persistent, kWG, 0);
  if (!grid) return -ENODEV;
  grid = (uint32_t)std::min<uint64_t>({(uint64_t)grid, staging_bytes / per_wg, (uint64_t)n_chunks});
  const uint32_t req = gsys_internal::persistent_grid_override(ctx);
  if (req && req < grid) grid = req;
  return gsys_internal::launch(ctx, (const void*)wordscan_persistent, grid, kWG, 0, args, s);
}
