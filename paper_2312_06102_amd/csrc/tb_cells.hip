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
// k_set_scan   : first cell of every set and depth.
// The cells themselves are written block by block (tb_blocks.hip).
#include "tb_internal.h"
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
    int32_t *__restrict__ status_word) {
  extern __shared__ __align__(16) unsigned char lds[];
  const WindowLds s = carve_window(lds, nl);
  const int64_t tile = blockIdx.x;
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
          in ? morton_key(rec[r].x, rec[r].y, rec[r].z, lo0, lo1, lo2, scale) : 0ull;
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

// One workgroup over all sets, THREADS sets per round: the first cell of every
// set and of every depth of every set, the outputs level_offset [B][23],
// cell_offsets [B+1] and n_cells, and the boxes used.
template <int THREADS>
__global__ __launch_bounds__(THREADS) void k_set_scan(
    const uint32_t *__restrict__ set_tot, int32_t nsets, int64_t *__restrict__ set_cells,
    int64_t *__restrict__ lvl_off, int64_t *__restrict__ level_offset,
    int64_t *__restrict__ cell_offsets, int64_t *__restrict__ n_cells,
    const double *__restrict__ box, double *__restrict__ box_out) {
  constexpr int kSetScanWaves = THREADS / 64;
  __shared__ uint32_t s_w[kSetScanWaves];
  __shared__ int64_t s_carry;
  const int wv = threadIdx.x / 64;
  if (threadIdx.x == 0) s_carry = 0;
  __syncthreads();
  for (int r0 = 0; r0 < nsets; r0 += THREADS) {
    const int b = r0 + threadIdx.x;
    uint32_t t[kLevels], v = 0;
#pragma unroll
    for (int d = 0; d < kLevels; ++d) {
      t[d] = (b < nsets) ? set_tot[b * kLevels + d] : 0u;
      v += t[d];
    }
    const uint32_t inc = wave_inclusive_scan(v);
    if (lane_id() == 63) s_w[wv] = inc;
    __syncthreads();
    int64_t off = s_carry, tot = 0;
    for (int q = 0; q < kSetScanWaves; ++q) {
      off += q < wv ? s_w[q] : 0u;
      tot += s_w[q];
    }
    off += (int64_t)(inc - v);
    if (b < nsets) {
      set_cells[b] = off;
      if (cell_offsets) cell_offsets[b] = off;
      int64_t run = off;
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
    }
    __syncthreads();
    if (threadIdx.x == 0) s_carry += tot;
    __syncthreads();
  }
  if (threadIdx.x == 0) {
    set_cells[nsets] = s_carry;
    if (cell_offsets) cell_offsets[nsets] = s_carry;
    *n_cells = s_carry;
  }
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
  if (p.nsets <= 64)
    k_set_scan<64><<<1, 64, 0, s>>>(w.set_tot, p.nsets, w.set_cells, w.lvl_off, out.level_offset,
                                    cell_offsets, out.n_cells, w.box, out.box_out);
  else
    k_set_scan<1024><<<1, 1024, 0, s>>>(w.set_tot, p.nsets, w.set_cells, w.lvl_off,
                                        out.level_offset, cell_offsets, out.n_cells, w.box,
                                        out.box_out);
  return hipGetLastError();
}

hipError_t launch_reorder(const Plan &p, const Work &w, const tb_tree &out, hipStream_t s) {
  k_reorder<<<(unsigned)p.cell_tiles, kCellThreads, window_lds_bytes(p.n_leaf), s>>>(
      out.perm, w.packed, p.n, p.n_leaf, w.tile_start, w.tile_set, w.set_off, p.nsets, w.box,
      p.cell_tiles, w.sorted, sorted_keys(p, w), out.key_sorted, out.pos_sorted, out.mass_sorted,
      w.ad, w.cell_cnt, out.status);
  return hipGetLastError();
}

// Largest dynamic LDS a workgroup may use on the current device (cached per
// device), after opting the reorder kernel in to it.
size_t cell_lds_limit() {
  static int cached_dev = -1;
  static size_t cached = 0;
  int dev = 0;
  if (hipGetDevice(&dev) != hipSuccess) return 0;
  if (dev != cached_dev) {
    int v = 0;
    if (hipDeviceGetAttribute(&v, hipDeviceAttributeMaxSharedMemoryPerBlock, dev) != hipSuccess) return 0;
    const int want = (int)cell_reorder_lds(TB_MAX_NLEAF);
    const int opt = v < want ? v : want;
    (void)hipFuncSetAttribute(reinterpret_cast<const void *>(k_reorder),
                              hipFuncAttributeMaxDynamicSharedMemorySize, opt);
    cached = (size_t)v;
    cached_dev = dev;
  }
  return cached;
}

// Dynamic LDS of the reorder pass for this n_leaf.
size_t cell_reorder_lds(int nl) { return window_lds_bytes(nl); }

}  // namespace tb
