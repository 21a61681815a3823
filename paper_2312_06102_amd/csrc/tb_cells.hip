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
// k_cell_count : per tile, per-depth cell counts; decoupled look-back gives
//                every tile its per-depth prefix.
// k_cell_emit  : writes key, depth, first particle and first-child slot of
//                every cell, and count plus moments of every leaf (the leaf's
//                particles are gathered through perm: the reorder step).
#include "tb_internal.h"

namespace tb {

constexpr int kWaves = kCellThreads / 64;
constexpr int kMaxSpan = (kCellTile + TB_MAX_NLEAF + kCellThreads - 1) / kCellThreads;

// Shared layout (dynamic LDS), sized for the actual n_leaf.
struct CellLds {
  uint64_t *keys;  // [T + 2 NL + 1]  keys of [t0 - NL - 1, t1 + NL)
  uint8_t *m;      // [T + NL]        w_j, then the sparse max table, j in [t0 - NL, t1)
  uint8_t *a;      // [T + NL]        a_i, i in [t0, t1 + NL)
  uint32_t *wtot;  // [kWaves][kLevelWords]
  uint32_t *lvl;   // [kLevels]       per-depth base of this tile
  uint32_t *off;   // [kLevels][kCellThreads] next cell index per depth per thread
};

__host__ __device__ inline size_t cell_lds_bytes(int nl, bool emit) {
  size_t b = (size_t)(kCellTile + 2 * nl + 1) * 8;
  b += 2 * (size_t)((kCellTile + nl + 15) & ~15);
  b += (size_t)kWaves * kLevelWords * 4 + kLevels * 4;
  if (emit) b += (size_t)kLevels * kCellThreads * 4;
  return b;
}

__device__ inline CellLds carve_lds(unsigned char *base, int nl, bool emit) {
  CellLds s;
  s.keys = reinterpret_cast<uint64_t *>(base);
  base += (size_t)(kCellTile + 2 * nl + 1) * 8;
  const size_t span = (size_t)((kCellTile + nl + 15) & ~15);
  s.m = base;
  base += span;
  s.a = base;
  base += span;
  s.wtot = reinterpret_cast<uint32_t *>(base);
  base += kWaves * kLevelWords * 4;
  s.lvl = reinterpret_cast<uint32_t *>(base);
  base += kLevels * 4;
  s.off = emit ? reinterpret_cast<uint32_t *>(base) : nullptr;
  return s;
}

// Loads the key window, computes a_i and the windowed maximum, and returns
// (in D[]) the leaf depth of this thread's IPT consecutive particles.
__device__ inline void tile_depths(const CellLds &s, const uint64_t *__restrict__ keys, int64_t n,
                                   int nl, int64_t t0, int64_t t1, uint8_t A[kCellIpt],
                                   uint8_t D[kCellIpt]) {
  const int T = (int)(t1 - t0);
  const int64_t ws = t0 - nl - 1;  // window start (may be negative)
  const int wn = T + 2 * nl + 1;
  for (int i = threadIdx.x; i < wn; i += kCellThreads) {
    const int64_t g = ws + i;
    s.keys[i] = (g >= 0 && g < n) ? keys[g] : 0ull;
  }
  __syncthreads();
  // a_i for i in [t0, t1 + nl)
  for (int i = threadIdx.x; i < T + nl; i += kCellThreads) {
    const int64_t g = t0 + i;
    uint8_t v = 0;
    if (g > 0 && g < n) v = (uint8_t)min_depth(s.keys[i + nl], s.keys[i + nl + 1]);
    s.a[i] = v;
  }
  // w_j for j in [t0 - nl, t1)
  for (int i = threadIdx.x; i < T + nl; i += kCellThreads) {
    const int64_t j = t0 - nl + i;
    uint8_t v = 0;
    if (j >= 0 && j + nl < n) v = (uint8_t)min_depth(s.keys[i + 1], s.keys[i + 1 + nl]);
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

// Per-thread packed per-depth counts of cells whose first particle is one of
// this thread's particles (particle i starts the cells at depths a_i .. D_i).
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
__device__ inline void block_level_scan(const CellLds &s, uint32_t c[kLevelWords],
                                        uint32_t tot[kLevelWords]) {
  const int wv = threadIdx.x / 64;
  uint32_t inc[kLevelWords];
#pragma unroll
  for (int wi = 0; wi < kLevelWords; ++wi) inc[wi] = wave_inclusive_scan(c[wi]);
  if (lane_id() == 63) {
#pragma unroll
    for (int wi = 0; wi < kLevelWords; ++wi) s.wtot[wv * kLevelWords + wi] = inc[wi];
  }
  __syncthreads();
#pragma unroll
  for (int wi = 0; wi < kLevelWords; ++wi) {
    uint32_t off = 0, t = 0;
#pragma unroll
    for (int q = 0; q < kWaves; ++q) {
      const uint32_t v = s.wtot[q * kLevelWords + wi];
      off += (q < wv) ? v : 0u;
      t += v;
    }
    c[wi] = off + inc[wi] - c[wi];
    tot[wi] = t;
  }
}

__device__ __forceinline__ uint32_t unpack(const uint32_t w[kLevelWords], int d) {
  return (w[d >> 1] >> ((d & 1) * 16)) & 0xffffu;
}

// ---------------------------------------------------------------------------
// count pass
// ---------------------------------------------------------------------------
__global__ __launch_bounds__(kCellThreads) void k_cell_count(
    const uint64_t *__restrict__ keys, int64_t n, int nl, uint64_t *__restrict__ cstatus,
    uint32_t *__restrict__ cincl, uint32_t *__restrict__ tile_counter, int64_t n_tiles,
    int32_t *__restrict__ status_word) {
  extern __shared__ __align__(16) unsigned char lds[];
  const CellLds s = carve_lds(lds, nl, false);
  __shared__ uint32_t s_tile;
  if (threadIdx.x == 0) s_tile = atomicAdd(tile_counter, 1u);
  __syncthreads();
  const int64_t tile = s_tile;
  if (tile >= n_tiles) {  // the counter was not reset: never true after k_init
    if (threadIdx.x == 0) atomicOr(status_word, TB_STATUS_INTERNAL);
    return;
  }
  const int64_t t0 = tile * kCellTile;
  const int64_t t1 = min(t0 + (int64_t)kCellTile, n);
  uint8_t A[kCellIpt], D[kCellIpt];
  tile_depths(s, keys, n, nl, t0, t1, A, D);
  uint32_t c[kLevelWords], tot[kLevelWords];
  thread_level_counts(A, D, c);
  block_level_scan(s, c, tot);
  // thread d publishes this tile's depth-d count and looks back for its prefix
  const int d = threadIdx.x;
  if (d < kLevels) {
    uint32_t cnt = 0;
#pragma unroll
    for (int wi = 0; wi < kLevelWords; ++wi)
      if (wi == (d >> 1)) cnt = (tot[wi] >> ((d & 1) * 16)) & 0xffffu;
    uint64_t *st = cstatus + tile * kLevels + d;
    if (tile == 0) {
      atomic_store_agent(st, kFlagInclusive | cnt);
      cincl[d] = cnt;
    } else {
      atomic_store_agent(st, kFlagAggregate | cnt);
      uint32_t excl = 0;
      int64_t q = tile - 1;
      bool timed_out = false;
      while (true) {
        const uint64_t sw = wait_published(cstatus + q * kLevels + d, timed_out);
        excl += (uint32_t)sw;
        if ((sw & kFlagMask) == kFlagInclusive || q == 0) break;
        --q;
      }
      if (timed_out) atomicOr(status_word, TB_STATUS_INTERNAL);
      atomic_store_agent(st, kFlagInclusive | (uint64_t)(excl + cnt));
      cincl[tile * kLevels + d] = excl + cnt;
    }
  }
}

// ---------------------------------------------------------------------------
// emit pass
// ---------------------------------------------------------------------------

// Inverse of the 3-way bit spread: gathers bits 0, 3, 6, ... into bits 0, 1, 2, ...
__device__ __forceinline__ uint32_t compact3(uint64_t v) {
  v &= 0x1249249249249249ull;
  v = (v ^ (v >> 2)) & 0x10c30c30c30c30c3ull;
  v = (v ^ (v >> 4)) & 0x100f00f00f00f00full;
  v = (v ^ (v >> 8)) & 0x001f0000ff0000ffull;
  v = (v ^ (v >> 16)) & 0x001f00000000ffffull;
  v = (v ^ (v >> 32)) & 0x1fffffull;
  return (uint32_t)v;
}

// End (exclusive) of the leaf that starts at particle i with depth dl.
__device__ inline int64_t leaf_end(const CellLds &s, const uint64_t *__restrict__ keys, int64_t n,
                                   int nl, int64_t t0, int64_t i, int dl) {
  const int64_t lim = min(n, i + nl + 1);
  for (int64_t j = i + 1; j < lim; ++j)
    if (s.a[j - t0] <= dl) return j;
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

struct LeafOut {
  double *com;
  double *quad;
  float *comf;
  float *quadf;
  float *pos_sorted;
  float *mass_sorted;
};

// FP64 leaf moments in the leaf's frame.
__device__ inline bool leaf_moments_fp64(const float *__restrict__ pos,
                                         const float *__restrict__ mass,
                                         const int32_t *__restrict__ perm, int64_t n, int64_t i0, int64_t i1,
                                         const double lo[3], const double off[3], double com[4],
                                         double quad[6], float *__restrict__ pos_sorted,
                                         float *__restrict__ mass_sorted, bool &internal) {
  double s0 = 0, s1[3] = {0, 0, 0}, s2[6] = {0, 0, 0, 0, 0, 0};
  bool bad = false;
  for (int64_t s = i0; s < i1; ++s) {
    const int64_t p = perm[s];
    if (p < 0 || p >= n) {  // perm is a permutation of [0, n)
      internal = true;
      continue;
    }
    const float x = pos[3 * p + 0], y = pos[3 * p + 1], z = pos[3 * p + 2];
    const float mf = mass[p];
    bad |= !(mf > 0.0f && isfinite(mf));
    if (pos_sorted) {
      pos_sorted[3 * s + 0] = x;
      pos_sorted[3 * s + 1] = y;
      pos_sorted[3 * s + 2] = z;
    }
    if (mass_sorted) mass_sorted[s] = mf;
    const double m = (double)mf;
    const double r0 = __dsub_rn(__dsub_rn((double)x, lo[0]), off[0]);
    const double r1 = __dsub_rn(__dsub_rn((double)y, lo[1]), off[1]);
    const double r2 = __dsub_rn(__dsub_rn((double)z, lo[2]), off[2]);
    s0 += m;
    s1[0] += m * r0;
    s1[1] += m * r1;
    s1[2] += m * r2;
    s2[0] += m * r0 * r0;
    s2[1] += m * r0 * r1;
    s2[2] += m * r0 * r2;
    s2[3] += m * r1 * r1;
    s2[4] += m * r1 * r2;
    s2[5] += m * r2 * r2;
  }
  const double M = s0;
  const double c0 = s1[0] / M, c1 = s1[1] / M, c2 = s1[2] / M;
  // second moments about the centre of mass, then the traceless combination
  const double xx = s2[0] - M * c0 * c0, xy = s2[1] - M * c0 * c1, xz = s2[2] - M * c0 * c2;
  const double yy = s2[3] - M * c1 * c1, yz = s2[4] - M * c1 * c2, zz = s2[5] - M * c2 * c2;
  const double tr = xx + yy + zz;
  com[0] = c0;
  com[1] = c1;
  com[2] = c2;
  com[3] = M;
  quad[0] = 3.0 * xx - tr;
  quad[1] = 3.0 * xy;
  quad[2] = 3.0 * xz;
  quad[3] = 3.0 * yy - tr;
  quad[4] = 3.0 * yz;
  quad[5] = 3.0 * zz - tr;
  return bad;
}

__global__ __launch_bounds__(kCellThreads) void k_cell_emit(
    const uint64_t *__restrict__ keys, int64_t n, int nl, const uint32_t *__restrict__ cincl,
    int64_t n_tiles, const double *__restrict__ box, const float *__restrict__ pos,
    const float *__restrict__ mass, const int32_t *__restrict__ perm,
    uint64_t *__restrict__ cell_key, uint8_t *__restrict__ cell_level,
    int32_t *__restrict__ cell_first, int32_t *__restrict__ cell_count,
    int32_t *__restrict__ child_ptr, double *__restrict__ com, double *__restrict__ quad,
    int64_t *__restrict__ level_offset, int64_t *__restrict__ n_cells, int64_t c_max,
    int32_t *__restrict__ status_word, double *__restrict__ box_out,
    float *__restrict__ pos_sorted, float *__restrict__ mass_sorted) {
  extern __shared__ __align__(16) unsigned char lds[];
  const CellLds s = carve_lds(lds, nl, true);
  const int64_t tile = blockIdx.x;
  const int64_t t0 = tile * kCellTile;
  const int64_t t1 = min(t0 + (int64_t)kCellTile, n);

  // per-depth base of this tile: level offset + prefix of earlier tiles
  if (threadIdx.x == 0) {
    uint32_t run = 0;
    for (int d = 0; d < kLevels; ++d) {
      const uint32_t tot = cincl[(n_tiles - 1) * kLevels + d];
      const uint32_t before = tile > 0 ? cincl[(tile - 1) * kLevels + d] : 0u;
      s.lvl[d] = run + before;
      if (tile == 0) level_offset[d] = run;
      run += tot;
    }
    if (tile == 0) {
      level_offset[kLevels] = run;
      *n_cells = run;
      if (box_out) {
        box_out[0] = box[0];
        box_out[1] = box[1];
        box_out[2] = box[2];
        box_out[3] = box[3];
      }
    }
  }
  uint8_t A[kCellIpt], D[kCellIpt];
  tile_depths(s, keys, n, nl, t0, t1, A, D);  // contains barriers after s.lvl is written
  uint32_t c[kLevelWords], tot[kLevelWords];
  thread_level_counts(A, D, c);
  block_level_scan(s, c, tot);
#pragma unroll
  for (int d = 0; d < kLevels; ++d) s.off[d * kCellThreads + threadIdx.x] = s.lvl[d] + unpack(c, d);

  const double lo[3] = {box[0], box[1], box[2]};
  const double side = box[3];
  bool bad = false, internal = false;
  for (int j = 0; j < kCellIpt; ++j) {
    const int a = A[j], dl = D[j];
    if (a > dl) continue;
    const int64_t i = t0 + threadIdx.x * kCellIpt + j;
    const uint64_t key = s.keys[(i - t0) + nl + 1];
    for (int d = a; d <= dl; ++d) {
      const uint32_t ci = s.off[d * kCellThreads + threadIdx.x];
      s.off[d * kCellThreads + threadIdx.x] = ci + 1;
      if ((int64_t)ci >= c_max) {  // cannot happen with consistent counts
        internal = true;
        continue;
      }
      cell_key[ci] = key >> (63 - 3 * d);
      cell_level[ci] = (uint8_t)d;
      cell_first[ci] = (int32_t)i;
      if (d < dl) {
        // first child: this particle's cell one depth down (emitted next)
        const uint32_t fc = s.off[(d + 1) * kCellThreads + threadIdx.x];
        child_ptr[2 * (int64_t)ci] = (int32_t)fc;
        child_ptr[2 * (int64_t)ci + 1] = 0;
      } else {
        child_ptr[2 * (int64_t)ci] = -1;
        child_ptr[2 * (int64_t)ci + 1] = 0;
        const int64_t e = leaf_end(s, keys, n, nl, t0, i, dl);
        cell_count[ci] = (int32_t)(e - i);
        const double h = ldexp(side, -dl);
        const int sh = kMaxDepth - dl;
        const double off[3] = {((double)(compact3(key >> 2) >> sh) + 0.5) * h,
                               ((double)(compact3(key >> 1) >> sh) + 0.5) * h,
                               ((double)(compact3(key) >> sh) + 0.5) * h};
        double cm[4], qd[6];
        bad |= leaf_moments_fp64(pos, mass, perm, n, i, e, lo, off, cm, qd, pos_sorted, mass_sorted,
                                 internal);
#pragma unroll
        for (int q = 0; q < 4; ++q) com[4 * (int64_t)ci + q] = cm[q];
#pragma unroll
        for (int q = 0; q < 6; ++q) quad[6 * (int64_t)ci + q] = qd[q];
      }
    }
  }
  if (__ballot(bad) != 0 && lane_id() == 0) atomicOr(status_word, TB_STATUS_MASS);
  if (__ballot(internal) != 0 && lane_id() == 0) atomicOr(status_word, TB_STATUS_INTERNAL);
}

hipError_t launch_cell_count(const Plan &p, const Work &w, int32_t *out_status, hipStream_t s) {
  const size_t lds = cell_lds_bytes(p.n_leaf, false);
  k_cell_count<<<(unsigned)p.cell_tiles, kCellThreads, lds, s>>>(
      sorted_keys(p, w), p.n, p.n_leaf, w.cell_status, w.cell_incl, w.counters + 32, p.cell_tiles,
      out_status);
  return hipGetLastError();
}

hipError_t launch_cell_emit(const Plan &p, const Work &w, const float *pos, const float *mass,
                            const tb_tree &out, hipStream_t s) {
  const size_t lds = cell_lds_bytes(p.n_leaf, true);
  k_cell_emit<<<(unsigned)p.cell_tiles, kCellThreads, lds, s>>>(
      sorted_keys(p, w), p.n, p.n_leaf, w.cell_incl, p.cell_tiles, w.box, pos, mass, out.perm,
      out.cell_key, out.cell_level, out.cell_first, out.cell_count, out.child_ptr,
      static_cast<double *>(out.com), static_cast<double *>(out.quad), out.level_offset,
      out.n_cells, p.c_max, out.status, out.box_out, out.pos_sorted, out.mass_sorted);
  return hipGetLastError();
}

size_t cell_emit_lds(int nl) { return cell_lds_bytes(nl, true); }

}  // namespace tb
