// tb_tiles.h -- per-tile cell counting shared by the reorder pass and the block
// builder: a particle i that starts cells at depths A_i .. D_i (A_i > D_i: none)
// adds one cell to each of those depths; per-thread counts are packed two
// 16-bit depths to a word and scanned across the workgroup.
#pragma once

#include "tb_internal.h"

namespace tb {

constexpr int kWaves = kCellThreads / 64;

#if defined(__HIP_DEVICE_COMPILE__) || defined(__HIPCC__)

// Per-thread packed per-depth counts of the cells started by this thread's
// particles (particle i starts the cells at depths A_i .. D_i).
__device__ inline void thread_level_counts(const uint8_t A[kCellIpt], const uint8_t D[kCellIpt],
                                           uint32_t c[kLevelWords]) {
#pragma unroll
  for (int wi = 0; wi < kLevelWords; ++wi) c[wi] = 0;
#pragma unroll
  for (int j = 0; j < kCellIpt; ++j) {
    const int a = A[j], d = D[j];
#pragma unroll
    for (int wi = 0; wi < kLevelWords; ++wi) {
      const int lo = 2 * wi, hi = 2 * wi + 1;
      c[wi] += (uint32_t)(a <= lo && lo <= d) | ((uint32_t)(a <= hi && hi <= d && hi < kLevels) << 16);
    }
  }
}

// Block-wide exclusive scan of the packed counters; also returns the totals.
__device__ inline void block_level_scan(uint32_t *wtot, uint32_t c[kLevelWords],
                                        uint32_t tot[kLevelWords]) {
  const int wv = threadIdx.x / 64;
  uint32_t inc[kLevelWords];
#pragma unroll
  for (int wi = 0; wi < kLevelWords; ++wi) inc[wi] = wave_inclusive_scan(c[wi]);
  if (lane_id() == 63) {
#pragma unroll
    for (int wi = 0; wi < kLevelWords; ++wi) wtot[wv * kLevelWords + wi] = inc[wi];
  }
  __syncthreads();
#pragma unroll
  for (int wi = 0; wi < kLevelWords; ++wi) {
    uint32_t off = 0, t = 0;
#pragma unroll
    for (int q = 0; q < kWaves; ++q) {
      const uint32_t v = wtot[q * kLevelWords + wi];
      off += (q < wv) ? v : 0u;
      t += v;
    }
    c[wi] = off + inc[wi] - c[wi];
    tot[wi] = t;
  }
  __syncthreads();  // wtot may be reused at once
}

__device__ __forceinline__ uint32_t unpack(const uint32_t w[kLevelWords], int d) {
  return (w[d >> 1] >> ((d & 1) * 16)) & 0xffffu;
}

// Tile t of set b covers [t0, t1) inside the set's range [S, E).
struct TileRange {
  int b;
  int64_t S, E, t0, t1;
};

__device__ __forceinline__ TileRange tile_range(int64_t t, const int64_t *__restrict__ tile_start,
                                                const int32_t *__restrict__ tile_set,
                                                const int64_t *__restrict__ set_off) {
  TileRange r;
  r.b = tile_set[t];
  r.S = set_off[r.b];
  r.E = set_off[r.b + 1];
  r.t0 = r.S + (t - tile_start[r.b]) * (int64_t)kCellTile;
  r.t1 = min(r.t0 + (int64_t)kCellTile, r.E);
  return r;
}

#endif

}  // namespace tb
