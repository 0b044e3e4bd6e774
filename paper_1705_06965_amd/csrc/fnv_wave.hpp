// FNV-1a-64 of many items at once on gfx950: one lane per item (the hash is
// a serial byte chain), items staged through LDS with coalesced loads.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "gsys_device.hpp"

namespace gsys_k {

using namespace gsys;

// h * 0x100000001b3 mod 2^64 written as (h << 40) + h * 0x1b3.
__device__ __forceinline__ uint64_t fnv_byte(uint64_t h, uint32_t byte) {
  h ^= byte;
  return (h << 40) + h * 0x1b3ull;
}

__device__ __forceinline__ uint64_t fnv_word(uint64_t h, uint32_t w, int nbytes) {
#pragma unroll
  for (int j = 0; j < 4; ++j)
    if (j < nbytes) h = fnv_byte(h, (w >> (8 * j)) & 0xffu);
  return h;
}

__device__ __forceinline__ uint64_t fnv_word4(uint64_t h, uint32_t w) {
  h = fnv_byte(h, w & 0xffu);
  h = fnv_byte(h, (w >> 8) & 0xffu);
  h = fnv_byte(h, (w >> 16) & 0xffu);
  return fnv_byte(h, w >> 24);
}

__device__ __forceinline__ uint64_t shfl64(uint64_t v, int src) {
  uint32_t lo = (uint32_t)__shfl((int)(uint32_t)v, src, 64);
  uint32_t hi = (uint32_t)__shfl((int)(uint32_t)(v >> 32), src, 64);
  return ((uint64_t)hi << 32) | lo;
}

// Per step every row (item) of the wave contributes CH contiguous bytes:
// CH/16 lanes x 16 B per row, 1024/CH rows per load instruction, CH/16
// instructions for the 64 rows.  The next step's loads are issued before the
// current step is hashed, so the host-link round trip overlaps the FNV chain.
// Rows of a wavefront are consecutive items, so row r starts at
// row0 + r * item_bytes; each row's byte count sits in LDS next to the tile.
// The loads are global and the tile accesses LDS (not flat) instructions, so
// the LDS reads of the hashing loop never wait for the loads in flight.
template <uint32_t CH>
struct Tile {
  static constexpr uint32_t kLanesPerRow = CH / 16;
  static constexpr uint32_t kRowsPerLoad = 64 / kLanesPerRow;
  static constexpr uint32_t kLoads = 64 / kRowsPerLoad;
  static constexpr uint32_t kRowStride = CH + 16;  // pad: conflict-free 16-byte LDS reads
  static constexpr uint32_t kBytes = 64 * kRowStride + 64 * 4;  // + each row's byte count
};

// 256-byte rows for work-groups of up to 256 work-items; 128-byte rows for
// larger work-groups (fewer registers per lane are available there).  Rows of
// 256 bytes read host staging at the link's rate (57 GB/s measured on MI355X
// against 42 GB/s for 128-byte rows): each row's request covers two
// 128-byte lines.
template <uint32_t WGMAX>
constexpr uint32_t chunk_for() { return WGMAX <= 256 ? 256u : 128u; }

// All 64 lanes of the wave call this.  Lane l hashes `nbytes` bytes of item
// row0 + l * item_bytes.  `tile` is this wave's LDS tile (Tile<CH>::kBytes).
template <uint32_t CH>
__device__ __forceinline__ uint64_t wave_fnv_t(uint64_t row0, uint32_t nbytes,
                                               uint32_t item_bytes, uint8_t* tile_generic) {
  using T = Tile<CH>;
  lptr_t<uint8_t> tile = lp(tile_generic);
  const uint32_t lane = lane_id();
  const uint32_t col = lane % T::kLanesPerRow;
  const uint32_t rsub = lane / T::kLanesPerRow;
  uint32_t maxlen = nbytes;
  for (int o = 32; o > 0; o >>= 1) maxlen = max(maxlen, (uint32_t)__shfl_xor((int)maxlen, o, 64));
  if (maxlen > item_bytes) maxlen = item_bytes;
  lptr_t<uint32_t> rlen = reinterpret_cast<lptr_t<uint32_t>>(tile + 64 * T::kRowStride);
  rlen[lane] = nbytes;
  __builtin_amdgcn_wave_barrier();
  uint64_t h = 0xcbf29ce484222325ull;
  u32x4 v[T::kLoads];
  auto load = [&](uint32_t off) {
#pragma unroll
    for (uint32_t k = 0; k < T::kLoads; ++k) {
      const uint32_t r = k * T::kRowsPerLoad + rsub;
      v[k] = u32x4{0, 0, 0, 0};
      // a row is read only where it holds bytes, inside its own item slot
      if (off < rlen[r] && off + col * 16 < item_bytes)
        v[k] = ldg16(row0 + (uint64_t)r * item_bytes + off + col * 16);
    }
  };
  if (maxlen) load(0);
  for (uint32_t off = 0; off < maxlen; off += CH) {
#pragma unroll
    for (uint32_t k = 0; k < T::kLoads; ++k) {
      const uint32_t r = k * T::kRowsPerLoad + rsub;
      *reinterpret_cast<lptr_t<u32x4>>(tile + r * T::kRowStride + col * 16) = v[k];
    }
    __builtin_amdgcn_wave_barrier();
    if (off + CH < maxlen) load(off + CH);  // prefetch the next step
    lptr_t<const uint8_t> row = tile + lane * T::kRowStride;
    if (off + CH <= nbytes) {
#pragma unroll 2
      for (uint32_t q = 0; q < CH / 16; ++q) {
        const u32x4 w = *reinterpret_cast<lptr_t<const u32x4>>(row + q * 16);
        h = fnv_word4(h, w.x);
        h = fnv_word4(h, w.y);
        h = fnv_word4(h, w.z);
        h = fnv_word4(h, w.w);
      }
    } else if (off < nbytes) {
      const uint32_t left = nbytes - off;
      for (uint32_t q = 0; q < CH / 4 && q * 4 < left; ++q) {
        const uint32_t w = *reinterpret_cast<lptr_t<const uint32_t>>(row + q * 4);
        const int nb = (int)min(4u, left - q * 4);
        h = fnv_word(h, w, nb);
      }
    }
    __builtin_amdgcn_wave_barrier();
  }
  return h;
}

}  // namespace gsys_k
