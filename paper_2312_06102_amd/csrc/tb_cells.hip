// tb_cells.hip -- leaves straight from the sorted keys (Sec. 2.3.1, Algorithm 1,
// Appendix A) and the level-ordered placement of every cell.
//
// Algorithm 1 walks the sorted keys once: the first particle k of a leaf gets
// the leaf depth D_k = max(minDepth(k-1, k), minDepth(k, k+n_leaf)) and the
// leaf absorbs the following particles that share its depth-D_k prefix.  Here
// the same leaves come out of a data-parallel form of that formula:
//
//   a_i = minDepth(i-1, i)            (0 for i = 0)
//   w_j = minDepth(j, j+n_leaf)       (for j + n_leaf < N, else 0)
//   D_i = min(21, max{ w_j : i - n_leaf <= j <= i })
//
// D_i is the depth of the leaf that holds particle i (a depth-d cell around i
// holds more than n_leaf particles exactly when some window [j, j+n_leaf]
// inside it contains i), and particle i is the first particle of the leaf
// exactly when a_i <= D_i -- where Algorithm 1 would start a new leaf.  For
// such a particle D_i equals the printed D_k.  The same particle is also the
// first particle of its ancestors at depths a_i .. D_i-1, which is how the
// bottom-up pass below knows, before any parent exists, how many cells each
// depth will hold and where each cell goes in the (depth, key) order.
//
// k_reorder    : particles in key order (the reorder step) and their keys; from
//                the keys of its tile plus an n_leaf halo, a_i and D_i of every
//                particle and the tile's per-depth cell counts;
// k_cell_scan  : per-depth prefix over the tiles of each set;
// k_set_scan_* : first cell of every set and depth;
// k_cell_emit  : writes key, depth, first particle and first-child slot of
//                every cell, and count plus moments of every leaf.
// (With TB_SUBTREES the cells are written block by block instead:
// tb_blocks.hip.)
#include "tb_internal.h"
#include "tb_moments.h"
#include "tb_tiles.h"

namespace tb {

constexpr int kMaxSpan = (kCellTile + TB_MAX_NLEAF + kCellThreads - 1) / kCellThreads;

__host__ __device__ constexpr size_t round16(size_t x) { return (x + 15) & ~size_t(15); }

// Shared layout of the reorder pass (dynamic LDS, sized for the actual n_leaf).
struct WindowLds {
  uint64_t *keys;  // [T + 2 NL + 1]  keys of [t0 - NL - 1, t1 + NL)
  uint8_t *m;      // [T + NL]        w_j, then the sparse max table, j in [t0 - NL, t1)
  uint8_t *a;      // [T + NL]        a_i, i in [t0, t1 + NL)
  uint32_t *wtot;  // [kWaves][kLevelWords]
};

__host__ __device__ inline size_t window_lds_bytes(int nl) {
  return round16((size_t)(kCellTile + 2 * nl + 1) * 8) + 2 * round16(kCellTile + nl) +
         (size_t)kWaves * kLevelWords * 4;
}

__device__ inline WindowLds carve_window(unsigned char *base, int nl) {
  WindowLds s;
  s.keys = reinterpret_cast<uint64_t *>(base);
  base += round16((size_t)(kCellTile + 2 * nl + 1) * 8);
  s.m = base;
  base += round16(kCellTile + nl);
  s.a = base;
  base += round16(kCellTile + nl);
  s.wtot = reinterpret_cast<uint32_t *>(base);
  return s;
}

// Shared layout of the emit pass.
struct EmitLds {
  uint8_t *a;          // [T + NL]        a_i, i in [t0, t1 + NL)
  uint8_t *d;          // [T]             D_i, i in [t0, t1)
  uint32_t *wtot;      // [kWaves][kLevelWords]
  uint32_t *lvl;       // [kLevels]       per-depth base of this tile
  uint16_t *off;       // [kLevels][kCellThreads] next cell slot per depth per thread
  float4 *rec;         // [T + NL]        sorted (x, y, z, m) of [t0, t1 + NL); stored once
                       //                 the cells are placed, over the dead `off` and `leaf`
  uint32_t *leaf;      // [T]             leaf starting in the tile: local first particle |
                       //                 depth << 11 | slot within its depth << 16; beside
                       //                 `off`, and read into registers before `rec` is stored
  uint8_t *heads;      // [T / 8]         bit li: particle t0 + li starts a leaf
  uint32_t *nleaf;     // [1]
};

__host__ __device__ inline size_t emit_off_bytes() {
  return round16((size_t)kLevels * kCellThreads * 2);
}

__host__ __device__ inline size_t emit_union_bytes(int nl) {
  const size_t cells = emit_off_bytes() + (size_t)kCellTile * 4;  // off, then leaf
  const size_t rec = (size_t)(kCellTile + nl) * 16;
  return round16(cells > rec ? cells : rec);
}

__host__ __device__ inline size_t emit_lds_bytes(int nl) {
  return round16(kCellTile + nl) + round16(kCellTile) + round16((size_t)kWaves * kLevelWords * 4) +
         round16(kLevels * 4) + emit_union_bytes(nl) + kCellTile / 8 + 16;
}

__device__ inline EmitLds carve_emit(unsigned char *base, int nl) {
  EmitLds s;
  s.a = base;
  base += round16(kCellTile + nl);
  s.d = base;
  base += round16(kCellTile);
  s.wtot = reinterpret_cast<uint32_t *>(base);
  base += round16((size_t)kWaves * kLevelWords * 4);
  s.lvl = reinterpret_cast<uint32_t *>(base);
  base += round16(kLevels * 4);
  // the per-depth cursors and the leaf list are dead once the cells are placed
  // (each thread keeps its leaf entries in registers); the particle records
  // take their place for the moment phase
  s.off = reinterpret_cast<uint16_t *>(base);
  s.leaf = reinterpret_cast<uint32_t *>(base + emit_off_bytes());
  s.rec = reinterpret_cast<float4 *>(base);
  base += emit_union_bytes(nl);
  s.heads = base;
  base += kCellTile / 8;
  s.nleaf = reinterpret_cast<uint32_t *>(base);
  return s;
}

// From the key window in LDS (positions [t0 - nl - 1, t1 + nl), zero outside
// the set [S, E)): a_i and the windowed maximum, and (in A[], D[]) a_i and the
// leaf depth of this thread's IPT consecutive particles.  The set's first
// particle starts a root (a = 0) and windows never reach across the set's ends.
__device__ inline void depths_from_window(const WindowLds &s, int64_t S, int64_t E, int nl,
                                          int64_t t0, int64_t t1, uint8_t A[kCellIpt],
                                          uint8_t D[kCellIpt]) {
  const int T = (int)(t1 - t0);
  // a_i for i in [t0, t1 + nl)
  for (int i = threadIdx.x; i < T + nl; i += kCellThreads) {
    const int64_t g = t0 + i;
    uint8_t v = 0;
    if (g > S && g < E) v = (uint8_t)min_depth(s.keys[i + nl], s.keys[i + nl + 1]);
    s.a[i] = v;
  }
  // w_j for j in [t0 - nl, t1)
  for (int i = threadIdx.x; i < T + nl; i += kCellThreads) {
    const int64_t j = t0 - nl + i;
    uint8_t v = 0;
    if (j >= S && j + nl < E) v = (uint8_t)min_depth(s.keys[i + 1], s.keys[i + 1 + nl]);
    s.m[i] = v;
  }
  __syncthreads();
  // sparse table: after the loop m[x] = max(w[x .. x + 2^k - 1]) with 2^k <= nl + 1
  const int span = T + nl;
  int pk = 1;
  while (2 * pk <= nl + 1) {
    uint8_t tmp[kMaxSpan];
#pragma unroll
    for (int r = 0; r < kMaxSpan; ++r) {
      const int x = threadIdx.x + r * kCellThreads;
      uint8_t v = 0;
      if (x < span) {
        v = s.m[x];
        if (x + pk < span) v = max(v, s.m[x + pk]);
      }
      tmp[r] = v;
    }
    __syncthreads();
#pragma unroll
    for (int r = 0; r < kMaxSpan; ++r) {
      const int x = threadIdx.x + r * kCellThreads;
      if (x < span) s.m[x] = tmp[r];
    }
    __syncthreads();
    pk *= 2;
  }
  // window [i - nl, i] = [i - nl, i - nl + pk - 1] u [i - pk + 1, i]
#pragma unroll
  for (int j = 0; j < kCellIpt; ++j) {
    const int li = threadIdx.x * kCellIpt + j;  // particle t0 + li
    uint8_t d = 0, av = 23;
    if (li < T) {
      const int mx = max(s.m[li], s.m[li + nl + 1 - pk]);
      d = (uint8_t)min(mx, kMaxDepth);
      av = s.a[li];
    }
    A[j] = av;
    D[j] = d;
  }
}

// ---------------------------------------------------------------------------
// reorder pass (Sec. 2.3, step iii) with the leaf depths
// ---------------------------------------------------------------------------
// sorted[s] = packed[perm[s]]: the particles in key order, one 16-byte record
// each, and their keys recomputed from the gathered positions (the same FP64
// arithmetic as the key pass, so the keys are identical).  One workgroup per
// cell tile, so the whole tile shares one set and one root box.  The workgroup
// also gathers the n_leaf + 1 particles on either side of its tile (inside the
// set), which gives it the key window of the leaf-depth formula: it stores
// a_i | D_i << 8 for every particle of the tile and the tile's cell count per
// depth.  Every thread issues all of a batch's index loads, then all of its
// gathers, so the random reads overlap.  Also fills the optional pos_sorted /
// mass_sorted / key_sorted outputs and checks the masses.
__global__ __launch_bounds__(kCellThreads) void k_reorder(
    const int32_t *__restrict__ perm, const float4 *__restrict__ packed, int64_t n, int nl,
    const int64_t *__restrict__ tile_start, const int32_t *__restrict__ tile_set,
    const int64_t *__restrict__ set_off, int32_t nsets, const double *__restrict__ box,
    int64_t cell_tiles, float4 *__restrict__ sorted, uint64_t *__restrict__ keys,
    uint64_t *__restrict__ key_out, float *__restrict__ pos_sorted,
    float *__restrict__ mass_sorted, uint16_t *__restrict__ ad, uint32_t *__restrict__ tile_cnt,
    int hilbert, const uint32_t *__restrict__ oversize, int32_t *__restrict__ status_word) {
  extern __shared__ __align__(16) unsigned char lds[];
  const WindowLds s = carve_window(lds, nl);
  // a batch set over the caller's index bound: every particle gets the root key
  const bool flat = oversize && *oversize != 0u;
  const int64_t tile = xcd_tile(blockIdx.x, gridDim.x);
  if (tile >= tile_start[nsets]) return;
  const TileRange tr = tile_range(tile, tile_start, tile_set, set_off);
  const int64_t t0 = tr.t0, t1 = tr.t1;
  const double lo0 = box[4 * tr.b + 0], lo1 = box[4 * tr.b + 1], lo2 = box[4 * tr.b + 2];
  const double scale = 2097152.0 / box[4 * tr.b + 3];
  const int T = (int)(t1 - t0);
  const int64_t ws = t0 - nl - 1;  // window start (may be negative)
  const int wn = T + 2 * nl + 1;
  bool internal = false, bad = false;
  // 9 items per thread cover the tile and its halo in one round trip for
  // n_leaf <= 127
  constexpr int kBatch = kCellIpt + 1;
  for (int i0 = 0; i0 < wn; i0 += kBatch * kCellThreads) {
    int32_t p[kBatch];
#pragma unroll
    for (int r = 0; r < kBatch; ++r) {
      const int i = i0 + r * kCellThreads + threadIdx.x;
      const int64_t g = ws + i;
      const bool in = i < wn && g >= tr.S && g < tr.E;
      p[r] = perm[in ? g : t0];
    }
    float4 rec[kBatch];
#pragma unroll
    for (int r = 0; r < kBatch; ++r) {
      const int i = i0 + r * kCellThreads + threadIdx.x;
      const int64_t g = ws + i;
      const bool in = i < wn && g >= tr.S && g < tr.E;
      const bool ok = p[r] >= 0 && p[r] < n;
      internal |= in && !ok;
      rec[r] = packed[ok ? p[r] : 0];
    }
#pragma unroll
    for (int r = 0; r < kBatch; ++r) {
      const int i = i0 + r * kCellThreads + threadIdx.x;
      const int64_t g = ws + i;
      const bool in = i < wn && g >= tr.S && g < tr.E;
      const uint64_t key =
          !in ? 0ull
          : flat
              ? 1ull << 63
              : particle_key(rec[r].x, rec[r].y, rec[r].z, lo0, lo1, lo2, scale, hilbert != 0);
      if (i < wn) s.keys[i] = key;
      if (g >= t0 && g < t1 && i < wn) {
        sorted[g] = rec[r];
        keys[g] = key;
        if (key_out) key_out[g] = key;
        bad |= !(rec[r].w > 0.0f && isfinite(rec[r].w));
        if (pos_sorted) {
          pos_sorted[3 * g + 0] = rec[r].x;
          pos_sorted[3 * g + 1] = rec[r].y;
          pos_sorted[3 * g + 2] = rec[r].z;
        }
        if (mass_sorted) mass_sorted[g] = rec[r].w;
      }
    }
  }
  if (__ballot(bad) != 0 && lane_id() == 0) atomicOr(status_word, TB_STATUS_MASS);
  if (__ballot(internal) != 0 && lane_id() == 0) atomicOr(status_word, TB_STATUS_INTERNAL);
  __syncthreads();

  uint8_t A[kCellIpt], D[kCellIpt];
  depths_from_window(s, tr.S, tr.E, nl, t0, t1, A, D);
#pragma unroll
  for (int j = 0; j < kCellIpt; ++j) {
    const int li = threadIdx.x * kCellIpt + j;
    if (li < T) ad[t0 + li] = (uint16_t)(A[j] | (D[j] << 8));
  }
  uint32_t c[kLevelWords], tot[kLevelWords];
  thread_level_counts(A, D, c);
  block_level_scan(s.wtot, c, tot);
  const int d = threadIdx.x;
  if (d < kLevels) {
    uint32_t cnt = 0;
#pragma unroll
    for (int wi = 0; wi < kLevelWords; ++wi)
      if (wi == (d >> 1)) cnt = (tot[wi] >> ((d & 1) * 16)) & 0xffffu;
    tile_cnt[d * cell_tiles + tile] = cnt;
  }
}

// Exclusive prefix of the per-tile counts over the earlier tiles of the same
// set, one workgroup per (depth, set); the set's total per depth goes to
// set_tot[b][d].  A single set uses 1024-thread workgroups (8192 tiles, i.e.
// 2^24 particles, per round), batches 256-thread ones (their sets are small).
constexpr int kScanItems = 8;

template <int THREADS>
__global__ __launch_bounds__(THREADS) void k_cell_scan(
    const uint32_t *__restrict__ tile_cnt, int64_t cell_tiles,
    const int64_t *__restrict__ tile_start, int32_t nsets, uint32_t *__restrict__ excl,
    uint32_t *__restrict__ set_tot) {
  __shared__ uint32_t s_w[THREADS / 64];
  const int d = blockIdx.x;
  const uint32_t *row = tile_cnt + d * cell_tiles;
  uint32_t *out = excl + d * cell_tiles;
  const int wv = threadIdx.x / 64;
  for (int b = blockIdx.y; b < nsets; b += gridDim.y) {
    const int64_t ts = tile_start[b], te = tile_start[b + 1];
    uint32_t carry = 0;
    for (int64_t c0 = ts; c0 < te; c0 += (int64_t)THREADS * kScanItems) {
      const int64_t q = c0 + (int64_t)threadIdx.x * kScanItems;
      uint32_t v[kScanItems], sum = 0;
#pragma unroll
      for (int r = 0; r < kScanItems; ++r) v[r] = (q + r < te) ? row[q + r] : 0u;
#pragma unroll
      for (int r = 0; r < kScanItems; ++r) sum += v[r];
      const uint32_t inc = wave_inclusive_scan(sum);
      if (lane_id() == 63) s_w[wv] = inc;
      __syncthreads();
      uint32_t off = 0, tot = 0;
#pragma unroll
      for (int k = 0; k < THREADS / 64; ++k) {
        const uint32_t t = s_w[k];
        off += (k < wv) ? t : 0u;
        tot += t;
      }
      __syncthreads();
      uint32_t run = carry + off + inc - sum;
#pragma unroll
      for (int r = 0; r < kScanItems; ++r) {
        if (q + r < te) out[q + r] = run;
        run += v[r];
      }
      carry += tot;
    }
    if (threadIdx.x == 0) set_tot[b * kLevels + d] = carry;
  }
}

// Rows of the set scan: 0 = cells per set; r = 1..21 = parent-pass chunks at
// depth r - 1 (children at depth r).
__device__ inline void set_rows(const uint32_t *__restrict__ set_tot, int32_t nsets, int b,
                                uint32_t t[kLevels], uint32_t v[kLevels]) {
#pragma unroll
  for (int d = 0; d < kLevels; ++d) t[d] = (b < nsets) ? set_tot[b * kLevels + d] : 0u;
  v[0] = 0;
#pragma unroll
  for (int d = 0; d < kLevels; ++d) v[0] += t[d];
#pragma unroll
  for (int r = 1; r < kLevels; ++r) v[r] = (t[r] + kParentChunk - 1) / kParentChunk;
}

// Sets [b0, b0 + THREADS), one per thread, every row at once, given in s_carry
// the sums of every row over the sets before b0: writes the first cell of every
// set and of every depth of every set (level_offset [B][23], cell_offsets), the
// parent-pass chunk tables and the boxes used, and leaves in s_w the block's
// per-wave row sums.
template <int THREADS>
__device__ inline void set_scan_block(
    int b0, const uint32_t *__restrict__ set_tot, int32_t nsets, int64_t *__restrict__ set_cells,
    int64_t *__restrict__ lvl_off, int64_t *__restrict__ level_offset,
    int64_t *__restrict__ cell_offsets, int64_t *__restrict__ par_start,
    const double *__restrict__ box, double *__restrict__ box_out,
    uint32_t (*s_w)[THREADS / 64], const int64_t *s_carry) {
  const int wv = threadIdx.x / 64;
  const int b = b0 + threadIdx.x;
  uint32_t t[kLevels], v[kLevels], inc[kLevels];
  set_rows(set_tot, nsets, b, t, v);
#pragma unroll
  for (int r = 0; r < kLevels; ++r) inc[r] = wave_inclusive_scan(v[r]);
  if (lane_id() == 63) {
#pragma unroll
    for (int r = 0; r < kLevels; ++r) s_w[r][wv] = inc[r];
  }
  __syncthreads();
  int64_t off[kLevels];
#pragma unroll
  for (int r = 0; r < kLevels; ++r) {
    int64_t o = s_carry[r];
    for (int q = 0; q < wv; ++q) o += s_w[r][q];
    off[r] = o + (int64_t)(inc[r] - v[r]);
  }
  if (b < nsets) {
    set_cells[b] = off[0];
    if (cell_offsets) cell_offsets[b] = off[0];
    int64_t run = off[0];
#pragma unroll
    for (int d = 0; d < kLevels; ++d) {
      lvl_off[b * (kLevels + 1) + d] = run;
      level_offset[b * (kLevels + 1) + d] = run;
      run += t[d];
    }
    lvl_off[b * (kLevels + 1) + kLevels] = run;
    level_offset[b * (kLevels + 1) + kLevels] = run;
    if (box_out)
      for (int k = 0; k < 4; ++k) box_out[4 * b + k] = box[4 * b + k];
#pragma unroll
    for (int r = 1; r < kLevels; ++r) par_start[(r - 1) * (nsets + 1) + b] = off[r];
  }
}

// The totals over all sets: set_cells[B], cell_offsets[B], n_cells and the last
// entry of every parent-pass chunk table (thread r < kLevels writes row r).
__device__ inline void set_scan_totals(int r, int64_t total, int32_t nsets,
                                       int64_t *__restrict__ set_cells,
                                       int64_t *__restrict__ cell_offsets,
                                       int64_t *__restrict__ n_cells,
                                       int64_t *__restrict__ par_start) {
  if (r == 0) {
    set_cells[nsets] = total;
    if (cell_offsets) cell_offsets[nsets] = total;
    *n_cells = total;
  } else {
    par_start[(r - 1) * (nsets + 1) + nsets] = total;
  }
}

// Up to 64 sets: one wave does the whole scan.
__global__ __launch_bounds__(64) void k_set_scan_wave(
    const uint32_t *__restrict__ set_tot, int32_t nsets, int64_t *__restrict__ set_cells,
    int64_t *__restrict__ lvl_off, int64_t *__restrict__ level_offset,
    int64_t *__restrict__ cell_offsets, int64_t *__restrict__ n_cells,
    int64_t *__restrict__ par_start, const double *__restrict__ box,
    double *__restrict__ box_out) {
  __shared__ uint32_t s_w[kLevels][1];
  __shared__ int64_t s_carry[kLevels];
  if (threadIdx.x < kLevels) s_carry[threadIdx.x] = 0;
  __syncthreads();
  set_scan_block<64>(0, set_tot, nsets, set_cells, lvl_off, level_offset, cell_offsets,
                     par_start, box, box_out, s_w, s_carry);
  __syncthreads();
  if (threadIdx.x < kLevels)
    set_scan_totals(threadIdx.x, (int64_t)s_w[threadIdx.x][0], nsets, set_cells, cell_offsets,
                    n_cells, par_start);
}

// More sets: kSetScanThreads sets per workgroup over G workgroups, in two
// launches.  k_set_sums writes the row sums of each workgroup's sets,
// wg_sum[g][r]; k_set_scan_wg adds the sums of the earlier workgroups to its own
// block scan.
constexpr int kSetScanThreads = 256;

__global__ __launch_bounds__(kSetScanThreads) void k_set_sums(
    const uint32_t *__restrict__ set_tot, int32_t nsets, int64_t *__restrict__ wg_sum) {
  constexpr int W = kSetScanThreads / 64;
  __shared__ uint32_t s_w[kLevels][W];
  uint32_t t[kLevels], v[kLevels];
  set_rows(set_tot, nsets, blockIdx.x * kSetScanThreads + threadIdx.x, t, v);
#pragma unroll
  for (int r = 0; r < kLevels; ++r) {
    const uint32_t inc = wave_inclusive_scan(v[r]);
    if (lane_id() == 63) s_w[r][threadIdx.x / 64] = inc;
  }
  __syncthreads();
  if (threadIdx.x < kLevels) {
    int64_t tot = 0;
    for (int q = 0; q < W; ++q) tot += s_w[threadIdx.x][q];
    wg_sum[blockIdx.x * kLevels + threadIdx.x] = tot;
  }
}

__global__ __launch_bounds__(kSetScanThreads) void k_set_scan_wg(
    const uint32_t *__restrict__ set_tot, int32_t nsets, const int64_t *__restrict__ wg_sum,
    int64_t *__restrict__ set_cells, int64_t *__restrict__ lvl_off,
    int64_t *__restrict__ level_offset, int64_t *__restrict__ cell_offsets,
    int64_t *__restrict__ n_cells, int64_t *__restrict__ par_start,
    const double *__restrict__ box, double *__restrict__ box_out) {
  constexpr int W = kSetScanThreads / 64;
  __shared__ uint32_t s_w[kLevels][W];
  __shared__ int64_t s_carry[kLevels];
  if (threadIdx.x < kLevels) {
    int64_t c = 0;
    for (int g = 0; g < (int)blockIdx.x; ++g) c += wg_sum[g * kLevels + threadIdx.x];
    s_carry[threadIdx.x] = c;
  }
  __syncthreads();
  set_scan_block<kSetScanThreads>(blockIdx.x * kSetScanThreads, set_tot, nsets, set_cells,
                                  lvl_off, level_offset, cell_offsets, par_start, box, box_out,
                                  s_w, s_carry);
  __syncthreads();
  if (blockIdx.x + 1 == gridDim.x && threadIdx.x < kLevels) {
    int64_t tot = s_carry[threadIdx.x];
    for (int q = 0; q < W; ++q) tot += s_w[threadIdx.x][q];
    set_scan_totals(threadIdx.x, tot, nsets, set_cells, cell_offsets, n_cells, par_start);
  }
}

// ---------------------------------------------------------------------------
// leaf moments
// ---------------------------------------------------------------------------

// End (exclusive) of the leaf that starts at particle i with depth dl, from
// the a_i of the particles after it (a: [t0, t1 + nl) relative to t0).
__device__ inline int64_t leaf_end(const uint8_t *a, const uint64_t *__restrict__ keys, int64_t n,
                                   int nl, int64_t t0, int64_t i, int dl) {
  // n is the end of the particle's set
  const int64_t lim = min(n, i + nl + 1);
  for (int64_t j = i + 1; j < lim; ++j)
    if (a[j - t0] <= dl) return j;
  if (lim == n) return n;
  // only a depth-21 leaf of identical keys can be longer than n_leaf
  const uint64_t k = keys[i];
  int64_t lo = i + nl + 1, hi = n;  // first index in [lo, hi) whose key differs
  while (lo < hi) {
    const int64_t mid = lo + (hi - lo) / 2;
    if (keys[mid] == k)
      lo = mid + 1;
    else
      hi = mid;
  }
  return lo;
}

// The same leaf end from the tile's head mask: a leaf ends where the next leaf
// starts (a particle inside the leaf shares the leaf's prefix with its
// predecessor, so it starts no cell; the first particle past the leaf differs
// from its predecessor at depth <= the leaf depth and starts its own leaf).
// Only a leaf reaching past the tile falls back to the halo scan.
__device__ inline int64_t leaf_end_fast(const EmitLds &s, const uint64_t *__restrict__ keys,
                                        int64_t n, int nl, int64_t t0, int T, int li, int dl) {
  const uint64_t *hw = reinterpret_cast<const uint64_t *>(s.heads);
  const int nw = (T + 63) >> 6;
  int w = li >> 6;
  const int b = li & 63;
  uint64_t bits = b == 63 ? 0ull : (hw[w] >> (b + 1)) << (b + 1);
  while (bits == 0 && ++w < nw) bits = hw[w];
  if (bits != 0) {
    const int p = (w << 6) + __ffsll((long long)bits) - 1;
    if (p < T) return t0 + p;
  }
  return leaf_end(s.a, keys, n, nl, t0, t0 + li, dl);
}

// ---------------------------------------------------------------------------
// emit pass
// ---------------------------------------------------------------------------
// One workgroup per cell tile: a_i and D_i (from the reorder pass) give every
// cell whose first particle lies in the tile; the per-depth prefix places it.
template <bool MIXED>
__global__ __launch_bounds__(kCellThreads) void k_cell_emit(
    const uint64_t *__restrict__ keys, const uint16_t *__restrict__ ad, int nl,
    const uint32_t *__restrict__ excl, int64_t cell_tiles, const int64_t *__restrict__ tile_start,
    const int32_t *__restrict__ tile_set, const int64_t *__restrict__ set_off, int32_t nsets,
    const int64_t *__restrict__ lvl_off, const double *__restrict__ box,
    const float4 *__restrict__ sorted, uint64_t *__restrict__ cell_key,
    uint8_t *__restrict__ cell_level, int32_t *__restrict__ cell_first,
    int32_t *__restrict__ cell_count, int32_t *__restrict__ child_ptr, void *__restrict__ com_v,
    void *__restrict__ quad_v, float *__restrict__ m_lo, int32_t *__restrict__ head_parent,
    int64_t c_max, int hilbert, int32_t *__restrict__ status_word) {
  extern __shared__ __align__(16) unsigned char lds[];
  const EmitLds s = carve_emit(lds, nl);
  const int64_t tile = xcd_tile(blockIdx.x, gridDim.x);
  if (tile >= tile_start[nsets]) return;
  const TileRange tr = tile_range(tile, tile_start, tile_set, set_off);
  const int64_t t0 = tr.t0, t1 = tr.t1, n = tr.E;  // n: end of this tile's set
  const int T = (int)(t1 - t0);

  // per-depth base of this tile: the set's first cell of the depth plus the
  // cells of the set's earlier tiles
  if (threadIdx.x < kLevels) {
    const int d = threadIdx.x;
    s.lvl[d] = (uint32_t)(lvl_off[tr.b * (kLevels + 1) + d] + excl[d * cell_tiles + tile]);
  }
  if (threadIdx.x == 0) *s.nleaf = 0;
  // this thread's particles t0 + 8t .. t0 + 8t + 7: their keys (issued first,
  // so that they travel with the batched loads below)
  uint64_t kk[kCellIpt];
#pragma unroll
  for (int j = 0; j < kCellIpt; ++j) {
    const int li = threadIdx.x * kCellIpt + j;
    kk[j] = keys[t0 + (li < T ? li : T - 1)];
  }
  // the (a, D) of the tile's particles and the n_leaf halo into LDS, in one
  // batch of loads
  const int span = (int)(min(t1 + (int64_t)nl, n) - t0);
  constexpr int kRecBatch = kCellIpt + 1;  // covers span for n_leaf <= 256
  for (int x0 = 0; x0 < span; x0 += kRecBatch * kCellThreads) {
    uint16_t v[kRecBatch];
#pragma unroll
    for (int u = 0; u < kRecBatch; ++u) {
      const int x = x0 + u * kCellThreads + threadIdx.x;
      v[u] = ad[t0 + (x < span ? x : span - 1)];
    }
#pragma unroll
    for (int u = 0; u < kRecBatch; ++u) {
      const int x = x0 + u * kCellThreads + threadIdx.x;
      if (x < span) {
        s.a[x] = (uint8_t)(v[u] & 0xff);
        if (x < T) s.d[x] = (uint8_t)(v[u] >> 8);
      }
    }
  }
  __syncthreads();
  uint8_t A[kCellIpt], D[kCellIpt];
#pragma unroll
  for (int j = 0; j < kCellIpt; ++j) {
    const int li = threadIdx.x * kCellIpt + j;
    A[j] = li < T ? s.a[li] : 23;  // 23: starts no cell
    D[j] = li < T ? s.d[li] : 0;
  }
  {
    // the head mask holds one byte per thread: bit j of byte t is particle 8t + j
    static_assert(kCellIpt == 8 && kCellThreads * kCellIpt == kCellTile,
                  "the head mask layout needs 8 particles per thread");
    uint32_t hb = 0;
#pragma unroll
    for (int j = 0; j < kCellIpt; ++j) hb |= (A[j] <= D[j] ? 1u : 0u) << j;
    s.heads[threadIdx.x] = (uint8_t)hb;  // items 8t .. 8t+7 (none past the tile end)
  }
  uint32_t c[kLevelWords], tot[kLevelWords];
  thread_level_counts(A, D, c);
  block_level_scan(s.wtot, c, tot);  // its barrier also publishes s.heads
#pragma unroll
  for (int d = 0; d < kLevels; ++d) s.off[d * kCellThreads + threadIdx.x] = (uint16_t)unpack(c, d);
  // this thread's leaves go to a contiguous run of the leaf list
  uint32_t my_leaves = 0;
#pragma unroll
  for (int j = 0; j < kCellIpt; ++j) my_leaves += (A[j] <= D[j]) ? 1u : 0u;
  const uint32_t inc = wave_inclusive_scan(my_leaves);
  uint32_t wave_base = 0;
  if (lane_id() == 63) wave_base = atomicAdd(s.nleaf, inc);
  wave_base = __shfl(wave_base, 63, 64);
  uint32_t leaf_slot = wave_base + inc - my_leaves;

  // cell structure; leaves are queued for the moment phase
  bool internal = false;
#pragma unroll
  for (int j = 0; j < kCellIpt; ++j) {
    const int a = A[j], dl = D[j];
    if (a > dl) continue;
    const int li = threadIdx.x * kCellIpt + j;
    const int64_t i = t0 + li;
    const uint64_t key = kk[j];
    for (int d = a; d <= dl; ++d) {
      const uint32_t rel = s.off[d * kCellThreads + threadIdx.x];
      s.off[d * kCellThreads + threadIdx.x] = (uint16_t)(rel + 1);
      const uint32_t ci = s.lvl[d] + rel;
      if ((int64_t)ci >= c_max) {  // cannot happen with consistent counts
        internal = true;
        continue;
      }
      cell_key[ci] = key >> (63 - 3 * d);
      cell_level[ci] = (uint8_t)d;
      cell_first[ci] = (int32_t)i;
      if (d < dl) {
        // first child: this particle's cell one depth down (emitted next)
        const uint32_t fc = s.lvl[d + 1] + s.off[(d + 1) * kCellThreads + threadIdx.x];
        reinterpret_cast<int2 *>(child_ptr)[ci] = make_int2((int32_t)fc, 0);
        if ((int64_t)fc < c_max) head_parent[fc] = (int32_t)ci;
      } else {
        reinterpret_cast<int2 *>(child_ptr)[ci] = make_int2(-1, 0);
        s.leaf[leaf_slot] = (uint32_t)li | ((uint32_t)dl << 11) | (rel << 16);
        ++leaf_slot;
      }
    }
  }
  __syncthreads();
  // the leaf list shares its space with the records: each thread keeps its
  // entries (at most kCellIpt: a tile starts at most one leaf a particle)
  const uint32_t nlv = *s.nleaf;
  uint32_t my_leaf[kCellIpt];
#pragma unroll
  for (int k = 0; k < kCellIpt; ++k) {
    const uint32_t x = threadIdx.x + (uint32_t)k * kCellThreads;
    my_leaf[k] = x < nlv ? s.leaf[x] : 0u;
  }
  __syncthreads();

  // the cursors and the leaf list are dead: the particle records (tile and
  // halo) take their place, in batched loads
  for (int x0 = 0; x0 < span; x0 += kRecBatch * kCellThreads) {
    float4 r[kRecBatch];
#pragma unroll
    for (int u = 0; u < kRecBatch; ++u) {
      const int x = x0 + u * kCellThreads + threadIdx.x;
      r[u] = sorted[t0 + (x < span ? x : span - 1)];
    }
#pragma unroll
    for (int u = 0; u < kRecBatch; ++u) {
      const int x = x0 + u * kCellThreads + threadIdx.x;
      if (x < span) s.rec[x] = r[u];
    }
  }
  __syncthreads();

  // leaf moments: one lane per leaf, particles read from LDS
  const double lo[3] = {box[4 * tr.b + 0], box[4 * tr.b + 1], box[4 * tr.b + 2]};
  const double side = box[4 * tr.b + 3];
#pragma unroll 1
  for (int k = 0; k < kCellIpt; ++k) {
    if (threadIdx.x + (uint32_t)k * kCellThreads >= nlv) break;
    // this thread's next entry; the rest move down (constant register indices)
    const uint32_t le = my_leaf[0];
#pragma unroll
    for (int j = 0; j + 1 < kCellIpt; ++j) my_leaf[j] = my_leaf[j + 1];
    const int li = le & 0x7ff;
    const int dl = (le >> 11) & 31;
    if (dl > kMaxDepth || li >= T) {  // cannot happen: entries come from the loop above
      internal = true;
      continue;
    }
    const uint32_t ci = s.lvl[dl] + (le >> 16);
    if ((int64_t)ci >= c_max) {
      internal = true;
      continue;
    }
    const int64_t i = t0 + li;
    const uint64_t key = keys[i];
    const int64_t e = leaf_end_fast(s, keys, n, nl, t0, T, li, dl);
    cell_count[ci] = (int32_t)(e - i);
    const int sh = kMaxDepth - dl;
    uint32_t ijk[3];
    if (hilbert) {
      cell_coords(key >> (3 * sh), dl, true, ijk);
    } else {
      ijk[0] = compact3(key >> 2) >> sh;
      ijk[1] = compact3(key >> 1) >> sh;
      ijk[2] = compact3(key) >> sh;
    }
    const int64_t e_lds = min(e, t0 + (int64_t)span);
    if constexpr (!MIXED) {
      double *com = static_cast<double *>(com_v);
      double *quad = static_cast<double *>(quad_v);
      const double h = ldexp(side, -dl);
      const double off[3] = {((double)ijk[0] + 0.5) * h, ((double)ijk[1] + 0.5) * h,
                             ((double)ijk[2] + 0.5) * h};
      LeafSums acc = {0.0, {0.0, 0.0, 0.0}, {0.0, 0.0, 0.0, 0.0, 0.0, 0.0}};
      for (int64_t q = i; q < e_lds; ++q) leaf_add(acc, s.rec[q - t0], lo, off);
      // only a saturated depth-21 leaf reaches past the staged halo
      for (int64_t q = e_lds; q < e; ++q) leaf_add(acc, sorted[q], lo, off);
      double cm[4], qd[6];
      leaf_finish(acc, cm, qd);
      double2 *cd = reinterpret_cast<double2 *>(com + 4 * (int64_t)ci);
      cd[0] = make_double2(cm[0], cm[1]);
      cd[1] = make_double2(cm[2], cm[3]);
      double2 *qq = reinterpret_cast<double2 *>(quad + 6 * (int64_t)ci);
      qq[0] = make_double2(qd[0], qd[1]);
      qq[1] = make_double2(qd[2], qd[3]);
      qq[2] = make_double2(qd[4], qd[5]);
    } else {
      float *com = static_cast<float *>(com_v);
      float *quad = static_cast<float *>(quad_v);
      const double scale = 2097152.0 / side;
      const uint32_t base[3] = {ijk[0] << sh, ijk[1] << sh, ijk[2] << sh};
      const float half = ldexpf(1.0f, sh - 1);
      LeafSumsF acc;
#pragma unroll
      for (int k = 0; k < 10; ++k) acc.s[k] = acc.c[k] = 0.0f;
      for (int64_t q = i; q < e_lds; ++q) leaf_add_f(acc, s.rec[q - t0], lo, scale, base, half, dl);
      for (int64_t q = e_lds; q < e; ++q) leaf_add_f(acc, sorted[q], lo, scale, base, half, dl);
      float cm[4], qd[6], mlo;
      leaf_finish_f(acc, cm, mlo, qd);
      // stored in absolute units: scaling by the side (a power of two) is exact
      const float l = ldexpf((float)side, -dl);
      reinterpret_cast<float4 *>(com)[ci] = make_float4(cm[0] * l, cm[1] * l, cm[2] * l, cm[3]);
      const float l2 = l * l;
      float2 *qq = reinterpret_cast<float2 *>(quad + 6 * (int64_t)ci);
      qq[0] = make_float2(qd[0] * l2, qd[1] * l2);
      qq[1] = make_float2(qd[2] * l2, qd[3] * l2);
      qq[2] = make_float2(qd[4] * l2, qd[5] * l2);
      m_lo[ci] = mlo;
    }
  }
  if (__ballot(internal) != 0 && lane_id() == 0) atomicOr(status_word, TB_STATUS_INTERNAL);
}

hipError_t launch_cell_scan(const Plan &p, const Work &w, const tb_tree &out,
                            int64_t *cell_offsets, hipStream_t s) {
  const int gy = p.nsets < 65535 ? p.nsets : 65535;
  if (p.nsets == 1)
    k_cell_scan<1024><<<dim3(kLevels, 1), 1024, 0, s>>>(w.cell_cnt, p.cell_tiles, w.tile_start,
                                                       p.nsets, w.cell_excl, w.set_tot);
  else
    k_cell_scan<256><<<dim3(kLevels, gy), 256, 0, s>>>(w.cell_cnt, p.cell_tiles, w.tile_start,
                                                      p.nsets, w.cell_excl, w.set_tot);
  if (p.nsets <= 64) {
    k_set_scan_wave<<<1, 64, 0, s>>>(w.set_tot, p.nsets, w.set_cells, w.lvl_off, out.level_offset,
                                     cell_offsets, out.n_cells, w.par_start, w.box, out.box_out);
  } else {
    const int g = (p.nsets + kSetScanThreads - 1) / kSetScanThreads;
    k_set_sums<<<g, kSetScanThreads, 0, s>>>(w.set_tot, p.nsets, w.set_wg);
    k_set_scan_wg<<<g, kSetScanThreads, 0, s>>>(w.set_tot, p.nsets, w.set_wg, w.set_cells,
                                                w.lvl_off, out.level_offset, cell_offsets,
                                                out.n_cells, w.par_start, w.box, out.box_out);
  }
  return hipGetLastError();
}

hipError_t launch_reorder(const Plan &p, const Work &w, const tb_tree &out, hipStream_t s) {
  k_reorder<<<(unsigned)p.cell_tiles, kCellThreads, window_lds_bytes(p.n_leaf), s>>>(
      out.perm, w.packed, p.n, p.n_leaf, w.tile_start, w.tile_set, w.set_off, p.nsets, w.box,
      p.cell_tiles, w.sorted, sorted_keys(p, w), out.key_sorted, out.pos_sorted, out.mass_sorted,
      w.ad, w.cell_cnt, (p.flags & TB_HILBERT) ? 1 : 0,
      p.set_index_bits ? w.counters + kOversizeCounter : nullptr, out.status);
  return hipGetLastError();
}

// Largest dynamic LDS a workgroup may use on the current device (cached per
// device), after opting the cell kernels in to it.
size_t cell_lds_limit() {
  static int cached_dev = -1;
  static size_t cached = 0;
  int dev = 0;
  if (hipGetDevice(&dev) != hipSuccess) return 0;
  if (dev != cached_dev) {
    int v = 0;
    if (hipDeviceGetAttribute(&v, hipDeviceAttributeMaxSharedMemoryPerBlock, dev) != hipSuccess) return 0;
    const int want = (int)cell_emit_lds(TB_MAX_NLEAF);
    const int opt = v < want ? v : want;
    (void)hipFuncSetAttribute(reinterpret_cast<const void *>(k_cell_emit<false>),
                              hipFuncAttributeMaxDynamicSharedMemorySize, opt);
    (void)hipFuncSetAttribute(reinterpret_cast<const void *>(k_cell_emit<true>),
                              hipFuncAttributeMaxDynamicSharedMemorySize, opt);
    (void)hipFuncSetAttribute(reinterpret_cast<const void *>(k_reorder),
                              hipFuncAttributeMaxDynamicSharedMemorySize, opt);
    cached = (size_t)v;
    cached_dev = dev;
  }
  return cached;
}

hipError_t launch_cell_emit(const Plan &p, const Work &w, const tb_tree &out, hipStream_t s) {
  const size_t lds = emit_lds_bytes(p.n_leaf);
  auto k = (p.flags & 0xffu) == TB_MIXED ? k_cell_emit<true> : k_cell_emit<false>;
  k<<<(unsigned)p.cell_tiles, kCellThreads, lds, s>>>(
      sorted_keys(p, w), w.ad, p.n_leaf, w.cell_excl, p.cell_tiles, w.tile_start, w.tile_set,
      w.set_off, p.nsets, w.lvl_off, w.box, w.sorted, out.cell_key, out.cell_level,
      out.cell_first, out.cell_count, out.child_ptr, out.com, out.quad, w.m_lo, w.head_parent,
      p.c_max, (p.flags & TB_HILBERT) ? 1 : 0, out.status);
  return hipGetLastError();
}

// Dynamic LDS of the reorder pass for this n_leaf.
size_t cell_reorder_lds(int nl) { return window_lds_bytes(nl); }

// The larger of the two cell kernels' LDS needs for this n_leaf.
size_t cell_emit_lds(int nl) {
  const size_t a = emit_lds_bytes(nl), b = window_lds_bytes(nl);
  return a > b ? a : b;
}

}  // namespace tb
