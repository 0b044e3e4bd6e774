// Block permutation written out with pwrite: the ordering / blocking
// microbenchmark of section 6 (Fig. 6).  An array of random words is cut
// into 8 KiB blocks; a work-group of 1024 work-items permutes one block
// `iters` times in LDS and then writes it to a file with one pwrite at
// work-group granularity.  The four cells strong / relaxed x blocking /
// non-blocking differ only in what the work-group does around that call:
//
//   strong-block     barrier, call, wait, barrier: every wavefront stays
//   strong-nonblock  barrier, call, barrier: nobody waits for the host
//   weak-block       barrier, call; only the caller's wavefront waits, the
//                    other fifteen leave
//   weak-nonblock    barrier, call, leave
//
// A pwrite is a producer call, so even relaxed ordering keeps the barrier
// before the call: every work-item's part of the block must be stored before
// the host reads it.  Work-groups that leave early free their wave slots for
// the next blocks while the host is still writing, which is the overlap the
// benchmark measures.
//
// One round maps block x to y with bit j of y[i] = bit tau[j] of x[sigma[i]]
// (a word shuffle and a bit shuffle inside each word, as DES's permutation
// steps shuffle bits).  Work-item i owns word i.  The bit shuffle is done a
// byte at a time: tab[k][v] holds, for byte k of a word having value v, the
// output bits that those eight input bits land on, so a word costs eight LDS
// lookups and seven ORs per round.  The tables are built per work-group from
// tau (2048 entries, two per work-item).  sigma and tau travel in the kernel
// arguments.
#include "gsys_device.hpp"
#include "gsys.h"
#include "kernels.hpp"

namespace gsys_pm {

using namespace gsys;

constexpr uint32_t kWords = 1024;
constexpr uint32_t kBlock = kWords * 8;

struct PmArgs {
  gsys_dev_ctx c;
  const uint64_t* in;   // device, n_blocks * 1024 words
  uint64_t stage;       // registered host buffer, kBlock bytes per block
  int64_t* out_ret;     // device, one per block
  uint64_t n_blocks;
  uint64_t file_off;
  uint32_t iters;
  int32_t fd;
  uint16_t sigma[kWords];
  uint8_t tau[64];
};

template <O o, B b>
__global__ __launch_bounds__(1024) void permute(PmArgs A) {
  __shared__ uint64_t buf[2][kWords];
  __shared__ uint64_t tab[8][256];
  __shared__ uint8_t dst_bit[64];
  const uint32_t t = threadIdx.x;
  const uint64_t blk = blockIdx.x;
  if (t < 64) dst_bit[A.tau[t]] = (uint8_t)t;  // input bit tau[t] -> output bit t
  buf[0][t] = A.in[blk * kWords + t];
  const uint32_t src = A.sigma[t];
  __syncthreads();
  for (uint32_t e = t; e < 8 * 256; e += kWords) {
    const uint32_t k = e >> 8, v = e & 255u;
    uint64_t m = 0;
#pragma unroll
    for (uint32_t q = 0; q < 8; ++q) m |= (uint64_t)((v >> q) & 1u) << dst_bit[8 * k + q];
    tab[k][v] = m;
  }
  __syncthreads();
  uint32_t cur = 0;
  for (uint32_t it = 0; it < A.iters; ++it) {
    const uint64_t w = buf[cur][src];
    uint64_t y = 0;
#pragma unroll
    for (uint32_t k = 0; k < 8; ++k) y |= tab[k][(uint32_t)(w >> (8 * k)) & 255u];
    // buf[cur ^ 1] was last read before the previous round's barrier
    buf[cur ^ 1][t] = y;
    __syncthreads();
    cur ^= 1;
  }
  const uint64_t at = A.stage + blk * kBlock;
  gp<uint64_t>(at)[t] = buf[cur][t];
  Ticket tk{0, 0, 0};
  const int64_t r = call_wg<o, b>(
      A.c, GSYS_NR_PWRITE64, 0,
      Args6{{(uint64_t)(int64_t)A.fd, at, kBlock, A.file_off + blk * kBlock, 0, 0}}, &tk);
  if (t == 0) {
    if constexpr (b == B::Blocking)
      A.out_ret[blk] = r;
    else
      A.out_ret[blk] = (r < 0 && r != GSYS_NOT_WAITED) ? r : GSYS_NOT_WAITED;
  }
}

}  // namespace gsys_pm

using namespace gsys_pm;

int gsys_permute(gsys_ctx* ctx, int fd, uint64_t in, const uint16_t* sigma, const uint8_t* tau,
                 uint64_t n_blocks, uint32_t iters, uint64_t staging, uint64_t file_off,
                 uint64_t out_ret, uint32_t cell, void* stream) {
  if (!ctx || !sigma || !tau) return -EINVAL;
  if (n_blocks == 0) return 0;
  if (!in || !out_ret || n_blocks > 0x7fffffffull) return -EINVAL;
  if (file_off > (1ull << 62) || n_blocks * kBlock > (1ull << 62) - file_off) return -EINVAL;
  bool seen_w[kWords] = {};
  for (uint32_t i = 0; i < kWords; ++i) {
    if (sigma[i] >= kWords || seen_w[sigma[i]]) return -EINVAL;
    seen_w[sigma[i]] = true;
  }
  bool seen_b[64] = {};
  for (uint32_t j = 0; j < 64; ++j) {
    if (tau[j] >= 64 || seen_b[tau[j]]) return -EINVAL;
    seen_b[tau[j]] = true;
  }
  if (GSYS_CELL_GRAN(cell) != GSYS_GRAN_WG) return -EINVAL;
  if (gsys_internal::check_host_range(ctx, staging, n_blocks * kBlock)) return -EFAULT;
  PmArgs A;
  if (int e = gsys_device_ctx(ctx, &A.c)) return e;
  A.in = (const uint64_t*)in;
  A.stage = staging;
  A.out_ret = (int64_t*)out_ret;
  A.n_blocks = n_blocks;
  A.file_off = file_off;
  A.iters = iters;
  A.fd = fd;
  for (uint32_t i = 0; i < kWords; ++i) A.sigma[i] = sigma[i];
  for (uint32_t j = 0; j < 64; ++j) A.tau[j] = tau[j];
  const bool strong = (cell & GSYS_CELL_STRONG) != 0;
  const bool blocking = (cell & GSYS_CELL_BLOCKING) != 0;
  const void* k;
  if (strong)
    k = blocking ? (const void*)permute<O::Strong, B::Blocking>
                 : (const void*)permute<O::Strong, B::NonBlocking>;
  else
    k = blocking ? (const void*)permute<O::Relaxed, B::Blocking>
                 : (const void*)permute<O::Relaxed, B::NonBlocking>;
  void* args[] = {&A};
  return gsys_internal::launch(ctx, k, (uint32_t)n_blocks, kWords, 0, args, (hipStream_t)stream);
}
