// tb_blocks.hip -- the cells, built subtree by subtree (Sec. 2.3.3, eq. 2).
//
// The paper divides the sorted keys recursively into blocks until each block
// is a subtree of at most n_serial particles; blocks share no cell, each is
// built on its own, and the cells above the blocks are built last.  The blocks
// are the leaves of the tree that n_leaf = n_serial would give, so the leaf
// formula itself finds them: with w_j = minDepth(j, j + n_serial),
//   Ds_i = min(21, max{ w_j : i - n_serial <= j <= i })
// is the depth of the block holding particle i, and particle i starts a block
// exactly when a_i = minDepth(i-1, i) <= Ds_i (a block of more than n_serial
// particles can only be a depth-21 run of identical keys).
//
// k_blocks      : per tile of 2048 sorted particles, Ds_i by a windowed maximum
//                 (suffix maxima over the previous tile, prefix maxima over this
//                 one) and the block starts: blk[i] = d_root, or kNoBlock.
// k_block_build : one workgroup per tile builds every block that starts in the
//                 tile, a batch of whole blocks (at most 2048 particles) at a
//                 time, entirely inside the workgroup:
//                   - a_i from the batch's keys; the leaf depth of eq. 2,
//                     D_i = max(minDepth(i, i-1), minDepth(i, i+n_leaf), d_root),
//                     with the neighbour terms inside the batch (a term that
//                     reaches another block is at most d_root, so it changes
//                     nothing);
//                   - every cell the batch's particles start (particle i starts
//                     depths A_i .. D_i) placed in the (depth, key) order from
//                     the per-tile prefix of the reorder pass's counts;
//                   - leaf moments from the particles, then the block's
//                     internal cells bottom-up from their children;
//                   - the cells above a block root (started by its first
//                     particle, depths a_i .. d_root - 1) get their structure
//                     here and go to a per-depth list.
// k_upper       : those upper cells, deepest first, from their children.
#include "tb_internal.h"
#include "tb_moments.h"
#include "tb_tiles.h"

namespace tb {

constexpr int kSerial = kCellTile;  // n_serial: the most particles of a block built in LDS
constexpr uint8_t kNoBlock = 0xff;
constexpr int kUpperThreads = 1024;
static_assert(kSerial == kCellThreads * kCellIpt, "one batch is one tile's worth of particles");
static_assert(kCellThreads == 4 * 64, "the depth scan gives each lane four threads");

// ---------------------------------------------------------------------------
// block-wide scans (256 threads)
// ---------------------------------------------------------------------------
__device__ __forceinline__ uint32_t wave_incl_max(uint32_t v) {
  const int l = lane_id();
#pragma unroll
  for (int o = 1; o < 64; o <<= 1) {
    const uint32_t t = __shfl_up(v, o, 64);
    if (l >= o) v = max(v, t);
  }
  return v;
}

__device__ __forceinline__ uint32_t wave_incl_max_rev(uint32_t v) {
  const int l = lane_id();
#pragma unroll
  for (int o = 1; o < 64; o <<= 1) {
    const uint32_t t = __shfl_down(v, o, 64);
    if (l + o < 64) v = max(v, t);
  }
  return v;
}

// max of v over the threads before this one (REV: after this one)
template <bool REV>
__device__ inline uint32_t block_excl_max(uint32_t v, uint32_t *s_w) {
  const int wv = threadIdx.x / 64, l = lane_id();
  const uint32_t inc = REV ? wave_incl_max_rev(v) : wave_incl_max(v);
  if (REV ? l == 0 : l == 63) s_w[wv] = inc;
  __syncthreads();
  uint32_t off = 0;
#pragma unroll
  for (int q = 0; q < kWaves; ++q)
    if (REV ? q > wv : q < wv) off = max(off, s_w[q]);
  const uint32_t nb = REV ? __shfl_down(inc, 1, 64) : __shfl_up(inc, 1, 64);
  const uint32_t ex = (REV ? l == 63 : l == 0) ? 0u : nb;
  __syncthreads();
  return max(off, ex);
}

__device__ inline uint32_t block_excl_sum(uint32_t v, uint32_t *s_w, uint32_t *total) {
  const int wv = threadIdx.x / 64;
  const uint32_t inc = wave_inclusive_scan(v);
  if (lane_id() == 63) s_w[wv] = inc;
  __syncthreads();
  uint32_t off = 0, tot = 0;
#pragma unroll
  for (int q = 0; q < kWaves; ++q) {
    const uint32_t t = s_w[q];
    off += q < wv ? t : 0u;
    tot += t;
  }
  __syncthreads();
  *total = tot;
  return off + inc - v;
}

// s_cnt[d][t] holds the cells that thread t's particles start at depth d; turns
// them into the exclusive prefix over the threads and writes the totals.  Wave
// w scans the depths d = w, w + 4, ...; each lane takes four threads' counts.
__device__ inline void lds_depth_scan(uint16_t (*s_cnt)[kCellThreads], uint32_t *s_tot) {
  const int wv = threadIdx.x / 64, l = lane_id();
  for (int d = wv; d < kLevels; d += kWaves) {
    uint32_t v[4], sum = 0;
#pragma unroll
    for (int k = 0; k < 4; ++k) {
      v[k] = s_cnt[d][4 * l + k];
      sum += v[k];
    }
    const uint32_t inc = wave_inclusive_scan(sum);
    uint32_t run = inc - sum;
#pragma unroll
    for (int k = 0; k < 4; ++k) {
      s_cnt[d][4 * l + k] = (uint16_t)run;
      run += v[k];
    }
    if (l == 63) s_tot[d] = inc;
  }
  __syncthreads();
}

// ---------------------------------------------------------------------------
// block decomposition
// ---------------------------------------------------------------------------
__global__ __launch_bounds__(kCellThreads) void k_blocks(
    const uint64_t *__restrict__ keys, const int64_t *__restrict__ tile_start,
    const int32_t *__restrict__ tile_set, const int64_t *__restrict__ set_off, int32_t nsets,
    uint8_t *__restrict__ blk) {
  __shared__ uint64_t s_k[3 * kSerial];  // keys of [t0 - n_s, t0 + 2 n_s); 0 outside the set
  __shared__ uint8_t s_w[2 * kSerial];   // w_j for j in [t0 - n_s, t0 + n_s)
  __shared__ uint32_t s_red[kWaves];
  const int64_t tile = blockIdx.x;
  if (tile >= tile_start[nsets]) return;
  const TileRange tr = tile_range(tile, tile_start, tile_set, set_off);
  const int64_t base = tr.t0 - kSerial;
  const int T = (int)(tr.t1 - tr.t0);
  constexpr int KB = 3 * kSerial / kCellThreads;
  {
    uint64_t v[KB];
#pragma unroll
    for (int r = 0; r < KB; ++r) {
      const int64_t g = base + r * kCellThreads + threadIdx.x;
      v[r] = (g >= tr.S && g < tr.E) ? keys[g] : 0ull;
    }
#pragma unroll
    for (int r = 0; r < KB; ++r) s_k[r * kCellThreads + threadIdx.x] = v[r];
  }
  __syncthreads();
  for (int x = threadIdx.x; x < 2 * kSerial; x += kCellThreads) {
    const int64_t j = base + x;
    uint8_t v = 0;
    if (j >= tr.S && j + kSerial < tr.E) v = (uint8_t)min_depth(s_k[x], s_k[x + kSerial]);
    s_w[x] = v;
  }
  __syncthreads();
  // particle i = t0 + y has the window j in [i - n_s, i], i.e. w entries y .. y + n_s:
  // the suffix maximum over [y, n_s) and the prefix maximum over [n_s, n_s + y]
  const int y0 = threadIdx.x * kCellIpt;
  uint32_t pre[kCellIpt], suf[kCellIpt];
  uint32_t run = 0;
#pragma unroll
  for (int j = 0; j < kCellIpt; ++j) {
    run = max(run, (uint32_t)s_w[kSerial + y0 + j]);
    pre[j] = run;
  }
  const uint32_t pex = block_excl_max<false>(run, s_red);
  run = 0;
#pragma unroll
  for (int j = kCellIpt - 1; j >= 0; --j) {
    run = max(run, (uint32_t)s_w[y0 + j]);
    suf[j] = run;
  }
  const uint32_t sex = block_excl_max<true>(run, s_red);
#pragma unroll
  for (int j = 0; j < kCellIpt; ++j) {
    const int y = y0 + j;
    if (y >= T) break;
    const int64_t i = tr.t0 + y;
    const uint32_t ds = min((uint32_t)kMaxDepth, max(max(pre[j], pex), max(suf[j], sex)));
    const uint32_t a =
        i == tr.S ? 0u : (uint32_t)min_depth(s_k[kSerial + y - 1], s_k[kSerial + y]);
    blk[i] = a <= ds ? (uint8_t)ds : kNoBlock;
  }
}

// ---------------------------------------------------------------------------
// blocks, built inside one workgroup each
// ---------------------------------------------------------------------------
struct BlockOut {
  uint64_t *cell_key;
  uint8_t *cell_level;
  int32_t *cell_first, *cell_count, *child_ptr;
  void *com, *quad;
  float *m_lo;
  int32_t *upper;       // [kLevels][upper_cap] slots of the cells above the blocks
  uint32_t *upper_cnt;  // [kLevels]
  int64_t upper_cap;
  int64_t c_max;
  bool hilbert;  // Peano-Hilbert keys
};

template <bool MIXED>
__device__ inline void leaf_moments(const BlockOut &o, int64_t ci, const float4 *__restrict__ sorted,
                                    int64_t i, int64_t e, uint64_t key, int dl, const double lo[3],
                                    double side) {
  const int sh = kMaxDepth - dl;
  uint32_t ijk[3];
  cell_coords(key >> (3 * sh), dl, o.hilbert, ijk);
  if constexpr (!MIXED) {
    const double h = ldexp(side, -dl);
    const double off[3] = {((double)ijk[0] + 0.5) * h, ((double)ijk[1] + 0.5) * h,
                           ((double)ijk[2] + 0.5) * h};
    LeafSums acc;
    leaf_zero(acc);
    for (int64_t q = i; q < e; ++q) leaf_add(acc, sorted[q], lo, off);
    double cm[4], qd[6];
    leaf_finish(acc, cm, qd);
    store_moments_fp64(static_cast<double *>(o.com), static_cast<double *>(o.quad), ci, cm, qd);
  } else {
    const double scale = 2097152.0 / side;
    const uint32_t base[3] = {ijk[0] << sh, ijk[1] << sh, ijk[2] << sh};
    const float half = ldexpf(1.0f, sh - 1);
    LeafSumsF acc;
    leaf_zero(acc);
    for (int64_t q = i; q < e; ++q) leaf_add_f(acc, sorted[q], lo, scale, base, half, dl);
    float cm[4], qd[6], mlo;
    leaf_finish_f(acc, cm, mlo, qd);
    store_moments_mixed(static_cast<float *>(o.com), static_cast<float *>(o.quad), o.m_lo, ci, cm,
                        mlo, qd, ldexpf((float)side, -dl));
  }
  o.cell_count[ci] = (int32_t)(e - i);
}

template <bool MIXED>
__device__ inline void parent_moments(const BlockOut &o, int64_t pc, int64_t c0, int nch, int dp,
                                      double side) {
  if constexpr (!MIXED)
    parent_from_children_fp64(pc, c0, nch, dp, side, o.cell_key, o.cell_count, o.child_ptr,
                              static_cast<double *>(o.com), static_cast<double *>(o.quad),
                              o.hilbert);
  else
    parent_from_children_mixed(pc, c0, nch, dp, side, o.cell_key, o.cell_count, o.child_ptr,
                               static_cast<float *>(o.com), static_cast<float *>(o.quad), o.m_lo,
                               o.hilbert);
}

// The structure of cell (d, key) with first particle i; nch and count of
// internal cells come later.  Returns false (and writes nothing) for a slot out
// of range, which consistent counts never give.
__device__ inline bool put_cell(const BlockOut &o, uint32_t slot, int d, uint64_t pkey, int64_t i,
                                int32_t first_child) {
  if ((int64_t)slot >= o.c_max) return false;
  o.cell_key[slot] = pkey >> (63 - 3 * d);
  o.cell_level[slot] = (uint8_t)d;
  o.cell_first[slot] = (int32_t)i;
  reinterpret_cast<int2 *>(o.child_ptr)[slot] = make_int2(first_child, 0);
  return true;
}

__device__ inline bool put_upper(const BlockOut &o, uint32_t slot, int d) {
  const uint32_t k = atomicAdd(&o.upper_cnt[d], 1u);
  if ((int64_t)k >= o.upper_cap) return false;
  o.upper[(int64_t)d * o.upper_cap + k] = (int32_t)slot;
  return true;
}

template <bool MIXED>
__global__ __launch_bounds__(kCellThreads) void k_block_build(
    const uint64_t *__restrict__ keys, const uint16_t *__restrict__ ad,
    const uint8_t *__restrict__ blk, int nl, const uint32_t *__restrict__ excl,
    int64_t cell_tiles, const int64_t *__restrict__ tile_start,
    const int32_t *__restrict__ tile_set, const int64_t *__restrict__ set_off, int32_t nsets,
    const int64_t *__restrict__ lvl_off, const double *__restrict__ box,
    const float4 *__restrict__ sorted, BlockOut o, int32_t *__restrict__ status_word) {
  // blk of [t0, t0 + W) before the batches (W is at most two tiles), the leaf
  // queue (batch offsets of first particles, below kSerial) during them
  __shared__ __align__(16) unsigned char s_u[2 * kSerial];
  uint8_t *s_bw = s_u;
  uint16_t *s_leaf = reinterpret_cast<uint16_t *>(s_u);
  __shared__ uint16_t s_st[kSerial];      // block starts in the tile (offsets from t0)
  __shared__ uint8_t s_sd[kSerial];       // their root depths
  __shared__ uint64_t s_key[kSerial + 1]; // keys of [bs - 1, be)
  __shared__ uint8_t s_dr[kSerial];       // root depth of each batch particle's block
  __shared__ uint8_t s_a[kSerial];        // A_x: the shallowest depth particle x starts
  __shared__ uint8_t s_d[kSerial];        // D_x: its leaf depth (eq. 2)
  __shared__ __align__(8) uint8_t s_mask[kLevels + 1][kCellThreads];  // bit x: A_x <= d
  __shared__ uint16_t s_off[kLevels][kCellThreads];  // cells per depth of the earlier threads
  // w_j (offset nl), then the windowed maxima: in s_off's space, since they are
  // dead once every thread holds its particles' depths, before s_off is written
  uint8_t *s_m = reinterpret_cast<uint8_t *>(&s_off[0][0]);
  static_assert(sizeof(s_off) >= kSerial + TB_MAX_NLEAF, "the window maxima fit in s_off");
  __shared__ uint32_t s_tot[kLevels];      // cells per depth of the batch
  __shared__ uint32_t s_base[2][kLevels];  // first slot per depth: tile t (running), tile t+1
  __shared__ uint32_t s_cnt1[kLevels];     // cells per depth the batch starts in tile t
  __shared__ uint32_t s_red[kWaves];
  __shared__ uint32_t s_nst, s_next, s_nleaf, s_k1, s_be, s_long, s_dmax, s_dmin;

  const int64_t tile = blockIdx.x;
  if (tile >= tile_start[nsets]) return;
  const TileRange tr = tile_range(tile, tile_start, tile_set, set_off);
  const int64_t t0 = tr.t0, S = tr.S, E = tr.E;
  const int T = (int)(tr.t1 - t0);
  const int W = (int)(min(tr.t1 + (int64_t)kSerial, E) - t0);
  const double lo[3] = {box[4 * tr.b + 0], box[4 * tr.b + 1], box[4 * tr.b + 2]};
  const double side = box[4 * tr.b + 3];
  bool bad = false;

  for (int x = threadIdx.x; x < W; x += kCellThreads) s_bw[x] = blk[t0 + x];
  __syncthreads();
  // the block starts of this tile, in order
  {
    uint32_t f = 0;
#pragma unroll
    for (int j = 0; j < kCellIpt; ++j) {
      const int y = threadIdx.x * kCellIpt + j;
      if (y < T && s_bw[y] != kNoBlock) f |= 1u << j;
    }
    uint32_t tot;
    uint32_t pos = block_excl_sum((uint32_t)__popc(f), s_red, &tot);
#pragma unroll
    for (int j = 0; j < kCellIpt; ++j) {
      if ((f >> j) & 1u) {
        const int y = threadIdx.x * kCellIpt + j;
        s_st[pos] = (uint16_t)y;
        s_sd[pos] = s_bw[y];
        ++pos;
      }
    }
    if (threadIdx.x == 0) {
      s_nst = tot;
      s_next = (uint32_t)W;
    }
  }
  __syncthreads();
  // the first block start after the tile, inside the window
  for (int y = T + threadIdx.x; y < W; y += kCellThreads)
    if (s_bw[y] != kNoBlock) atomicMin(&s_next, (uint32_t)y);
  __syncthreads();
  const int nst = (int)s_nst;
  if (nst == 0) return;  // every particle here belongs to a block of an earlier tile
  // end (offset from t0) of block k; kBeyond when it lies past the window
  const uint32_t kBeyond = 0xffffffffu;
  const bool window_is_set_end = t0 + W == E;
  auto block_end = [&](int k) -> uint32_t {
    if (k + 1 < nst) return s_st[k + 1];
    if (s_next < (uint32_t)W) return s_next;
    return window_is_set_end ? (uint32_t)W : kBeyond;
  };

  // slot bases: cells of earlier tiles of the set, plus those started by this
  // tile's particles before its first block (they belong to an earlier block)
  {
    uint8_t A[kCellIpt], D[kCellIpt];
    const int ybeg = s_st[0];
#pragma unroll
    for (int j = 0; j < kCellIpt; ++j) {
      const int y = threadIdx.x * kCellIpt + j;
      uint16_t v = 0xffff;  // a = 255 > D: no cell
      if (y < ybeg) v = ad[t0 + y];
      A[j] = (uint8_t)(v & 0xff);
      D[j] = (uint8_t)(v >> 8);
    }
    if (threadIdx.x < kLevels) s_cnt1[threadIdx.x] = 0;
    __syncthreads();
    uint32_t c[kLevelWords];
    thread_level_counts(A, D, c);
#pragma unroll
    for (int d = 0; d < kLevels; ++d) {
      const uint32_t v = unpack(c, d);
      if (v) atomicAdd(&s_cnt1[d], v);
    }
    __syncthreads();
    if (threadIdx.x < kLevels) {
      const int d = threadIdx.x;
      const int64_t lb = lvl_off[tr.b * (kLevels + 1) + d];
      s_base[0][d] = (uint32_t)(lb + excl[d * cell_tiles + tile] + s_cnt1[d]);
      const bool next_in_set = tile + 1 < tile_start[tr.b + 1];
      s_base[1][d] = next_in_set ? (uint32_t)(lb + excl[d * cell_tiles + tile + 1]) : 0u;
    }
  }
  __syncthreads();

  for (int k0 = 0; k0 < nst;) {
    if (threadIdx.x == 0) {
      const uint32_t bs = s_st[k0];
      const uint32_t e0 = block_end(k0);
      uint32_t k1 = (uint32_t)k0 + 1, be = e0, lng = 0;
      if (e0 == kBeyond || e0 - bs > (uint32_t)kSerial) {
        lng = 1;  // one block of more than n_serial identical keys
      } else {
        // the most whole blocks that fit one batch (ends increase with k)
        uint32_t lo_k = k1, hi_k = (uint32_t)nst;
        while (lo_k < hi_k) {
          const uint32_t mid = (lo_k + hi_k + 1) >> 1;
          const uint32_t e = block_end((int)mid - 1);
          if (e != kBeyond && e - bs <= (uint32_t)kSerial)
            lo_k = mid;
          else
            hi_k = mid - 1;
        }
        k1 = lo_k;
        be = block_end((int)k1 - 1);
      }
      s_k1 = k1;
      s_be = be;
      s_long = lng;
    }
    __syncthreads();
    const int k1 = (int)s_k1;
    const int bs = s_st[k0];
    if (s_long) {
      // ---- a depth-21 block of identical keys, larger than a batch ----
      const int64_t g0 = t0 + bs;
      if (threadIdx.x == 0) {
        int64_t ge;
        if (s_be != kBeyond) {
          ge = t0 + s_be;
        } else {  // first key after the run: binary search over the sorted keys
          const uint64_t k = keys[g0];
          int64_t lo_i = t0 + W, hi_i = E;
          while (lo_i < hi_i) {
            const int64_t mid = lo_i + (hi_i - lo_i) / 2;
            if (keys[mid] == k)
              lo_i = mid + 1;
            else
              hi_i = mid;
          }
          ge = lo_i;
        }
        const uint64_t key = keys[g0];
        const int a = g0 == S ? 0 : min_depth(keys[g0 - 1], key);
        if (s_sd[k0] != kMaxDepth || a > kMaxDepth) {
          bad = true;
        } else {
          for (int d = a; d <= kMaxDepth; ++d) {
            const uint32_t slot = s_base[0][d];
            const int32_t fc = d < kMaxDepth ? (int32_t)s_base[0][d + 1] : -1;
            if (!put_cell(o, slot, d, key, g0, fc)) {
              bad = true;
              continue;
            }
            if (d < kMaxDepth && !put_upper(o, slot, d)) bad = true;
          }
          if ((int64_t)s_base[0][kMaxDepth] < o.c_max)
            leaf_moments<MIXED>(o, s_base[0][kMaxDepth], sorted, g0, ge, key, kMaxDepth, lo, side);
          for (int d = a; d <= kMaxDepth; ++d) s_base[0][d] += 1;
        }
      }
      k0 = k1;
      __syncthreads();
      continue;
    }

    // ---- a batch of whole blocks [bs, be), at most n_serial particles ----
    const int n = (int)s_be - bs;
    for (int x = threadIdx.x; x <= n; x += kCellThreads) {
      const int64_t g = t0 + bs - 1 + x;
      s_key[x] = (g >= S && g < E) ? keys[g] : 0ull;
    }
    for (int x = threadIdx.x; x < n; x += kCellThreads) {
      // the block of particle bs + x: the last start at or before it
      int lo_k = k0, hi_k = k1 - 1;
      while (lo_k < hi_k) {
        const int mid = (lo_k + hi_k + 1) >> 1;
        if (s_st[mid] <= bs + x)
          lo_k = mid;
        else
          hi_k = mid - 1;
      }
      s_dr[x] = s_sd[lo_k];
    }
    __syncthreads();
    // w_j = minDepth(j, j + n_leaf) inside the batch, stored at j + nl; zero before it
    for (int x = threadIdx.x; x < n + nl; x += kCellThreads) {
      const int j = x - nl;
      uint8_t v = 0;
      if (j >= 0 && j + nl < n) v = (uint8_t)min_depth(s_key[j + 1], s_key[j + 1 + nl]);
      s_m[x] = v;
    }
    __syncthreads();
    // sparse table: afterwards s_m[x] = max of the 2^k entries from x, 2^k <= nl + 1
    int pk = 1;
    const int span = n + nl;
    while (2 * pk <= nl + 1) {
      constexpr int R = (kSerial + TB_MAX_NLEAF + kCellThreads - 1) / kCellThreads;
      uint8_t tmp[R];
#pragma unroll
      for (int r = 0; r < R; ++r) {
        const int x = threadIdx.x + r * kCellThreads;
        uint8_t v = 0;
        if (x < span) {
          v = s_m[x];
          if (x + pk < span) v = max(v, s_m[x + pk]);
        }
        tmp[r] = v;
      }
      __syncthreads();
#pragma unroll
      for (int r = 0; r < R; ++r) {
        const int x = threadIdx.x + r * kCellThreads;
        if (x < span) s_m[x] = tmp[r];
      }
      __syncthreads();
      pk *= 2;
    }
    // this thread's particles x = 8t .. 8t+7: A (cells start) and D (eq. 2)
    uint32_t dmax = 0, dmin = kLevels;
    {
      uint8_t A[kCellIpt], D[kCellIpt];
#pragma unroll
      for (int j = 0; j < kCellIpt; ++j) {
        const int x = threadIdx.x * kCellIpt + j;
        uint8_t a = 23, dd = 0;
        if (x < n) {
          // window [x - nl, x] of the w stored at offset nl: [x, x + nl]
          const int mx = max(s_m[x], s_m[x + nl + 1 - pk]);
          const int dr = s_dr[x];
          dd = (uint8_t)min(max(mx, dr), kMaxDepth);
          a = (t0 + bs + x == S) ? 0 : (uint8_t)min_depth(s_key[x], s_key[x + 1]);
          if (dd > 0 && max((int)a, dr) < dd) dmax = max(dmax, (uint32_t)dd - 1);
          dmin = min(dmin, (uint32_t)dr);
        }
        A[j] = a;
        D[j] = dd;
      }
      __syncthreads();  // s_m is dead: s_off, which holds it, is written next
      // depth masks: bit x of s_mask[d] set when particle x starts a cell at depth <= d
#pragma unroll
      for (int d = 0; d <= kLevels; ++d) {
        uint32_t bits = 0;
#pragma unroll
        for (int j = 0; j < kCellIpt; ++j) bits |= (A[j] <= d ? 1u : 0u) << j;
        s_mask[d][threadIdx.x] = (uint8_t)bits;
      }
      // cells per depth of this thread's particles, then the prefix over threads
      uint32_t c[kLevelWords];
      thread_level_counts(A, D, c);
#pragma unroll
      for (int d = 0; d < kLevels; ++d) s_off[d][threadIdx.x] = (uint16_t)unpack(c, d);
#pragma unroll
      for (int j = 0; j < kCellIpt; ++j) {
        s_a[threadIdx.x * kCellIpt + j] = A[j];
        s_d[threadIdx.x * kCellIpt + j] = D[j];
      }
    }
    __syncthreads();
    lds_depth_scan(s_off, s_tot);
    // cells the batch starts in tile t: the prefix at the tile's end
    if (threadIdx.x < kLevels) {
      const int d = threadIdx.x, xt = T - bs;
      uint32_t v = s_tot[d];
      if (xt < n) {
        const int t = xt / kCellIpt;
        v = s_off[d][t];
        for (int q = t * kCellIpt; q < xt; ++q)
          if (s_a[q] <= d && d <= s_d[q]) ++v;
      }
      s_cnt1[d] = v;
    }
    if (threadIdx.x == 0) {
      s_nleaf = 0;
      s_dmax = 0;
      s_dmin = kLevels;
    }
    __syncthreads();
    atomicMax(&s_dmax, dmax);
    atomicMin(&s_dmin, dmin);

    // global slot of the cell with rank r (among the batch's cells at depth d)
    // started by batch particle x
    auto to_slot = [&](int x, int d, uint32_t r) -> uint32_t {
      return bs + x < T ? s_base[0][d] + r : s_base[1][d] + r - s_cnt1[d];
    };

    // structure of every cell, each thread through its particles in order and
    // each particle's depths upwards, so that the running per-depth cursors give
    // the rank of the cell and of its first child; leaves queued
    for (int j = 0; j < kCellIpt; ++j) {
      const int x = (int)threadIdx.x * kCellIpt + j;
      if (x >= n) break;
      const int a = s_a[x], dl = s_d[x];
      if (a > dl) continue;
      const int64_t i = t0 + bs + x;
      const uint64_t key = s_key[x + 1];
      const int dr = s_dr[x];
      for (int d = a; d <= dl; ++d) {
        const uint32_t r = s_off[d][threadIdx.x];
        s_off[d][threadIdx.x] = (uint16_t)(r + 1);
        const uint32_t slot = to_slot(x, d, r);
        const int32_t fc = d < dl ? (int32_t)to_slot(x, d + 1, s_off[d + 1][threadIdx.x]) : -1;
        if (!put_cell(o, slot, d, key, i, fc)) {
          bad = true;
          continue;
        }
        if (d < dr && !put_upper(o, slot, d)) bad = true;
        if (d == dl) s_leaf[atomicAdd(&s_nleaf, 1u)] = (uint16_t)x;
      }
    }
    __syncthreads();

    // slot of the depth-d cell that particle x starts, from the final cursors of
    // its thread: minus the cells its thread's later particles start at depth d
    auto slot_at = [&](int x, int d) -> uint32_t {
      const int t = x / kCellIpt;
      uint32_t r = s_off[d][t];
      for (int q = x; q < (t + 1) * kCellIpt && q < n; ++q)
        if (s_a[q] <= d && d <= s_d[q]) --r;
      return to_slot(x, d, r);
    };
    // a depth-d cell that particle x starts ends at the next particle of the
    // batch that starts a cell at depth <= d (the batch ends with a block)
    const uint64_t *mw = reinterpret_cast<const uint64_t *>(&s_mask[0][0]);
    constexpr int kMaskWords = kCellThreads * kCellIpt / 64;
    auto next_start = [&](int x, int d) -> int {
      if (x + 1 >= n) return n;
      const uint64_t *m = mw + d * kMaskWords;
      int w = (x + 1) >> 6;
      const int b = (x + 1) & 63;
      uint64_t bits = (m[w] >> b) << b;
      const int nw = (n + 63) >> 6;
      while (bits == 0 && ++w < nw) bits = m[w];
      if (bits == 0) return n;
      const int p = (w << 6) + __ffsll((long long)bits) - 1;
      return p < n ? p : n;
    };
    // particles in [x, e) that start a cell at depth <= d
    auto starts_in = [&](int x, int e, int d) -> int {
      const uint64_t *m = mw + d * kMaskWords;
      int cnt = 0;
      for (int w = x >> 6; w <= (e - 1) >> 6; ++w) {
        uint64_t bits = m[w];
        const int lo_b = w == (x >> 6) ? (x & 63) : 0;
        const int hi_b = w == ((e - 1) >> 6) ? ((e - 1) & 63) : 63;
        bits >>= lo_b;
        if (hi_b - lo_b < 63) bits &= (1ull << (hi_b - lo_b + 1)) - 1ull;
        cnt += __popcll(bits);
      }
      return cnt;
    };

    // leaf moments, one lane per leaf
    const uint32_t nlv = s_nleaf;
    for (uint32_t q = threadIdx.x; q < nlv; q += kCellThreads) {
      const int x = (int)s_leaf[q];
      const int dl = s_d[x];
      const int e = next_start(x, dl);
      const uint32_t ci = slot_at(x, dl);
      if ((int64_t)ci >= o.c_max) {
        bad = true;
        continue;
      }
      leaf_moments<MIXED>(o, ci, sorted, t0 + bs + x, t0 + bs + e, s_key[x + 1], dl, lo, side);
    }
    __syncthreads();

    // the blocks' internal cells, deepest first, from their children (written by
    // this workgroup: visible after the barrier)
    const int dtop = (int)s_dmax, dbot = (int)s_dmin;
    for (int d = dtop; d >= dbot; --d) {
      for (int j = 0; j < kCellIpt; ++j) {
        const int x = (int)threadIdx.x * kCellIpt + j;
        if (x >= n) break;
        if (max((int)s_a[x], (int)s_dr[x]) > d || d >= s_d[x]) continue;
        const int e = next_start(x, d);
        const int nch = starts_in(x, e, d + 1);
        const uint32_t p = slot_at(x, d), c0 = slot_at(x, d + 1);
        if ((int64_t)p >= o.c_max || (int64_t)c0 + nch > o.c_max || nch < 1 || nch > 8) {
          bad = true;
          continue;
        }
        parent_moments<MIXED>(o, p, c0, nch, d, side);
      }
      __syncthreads();
    }
    // the next batch numbers the tile's cells after this one's
    if (threadIdx.x < kLevels) s_base[0][threadIdx.x] += s_cnt1[threadIdx.x];
    __syncthreads();
    k0 = k1;
  }
  if (__ballot(bad) != 0 && lane_id() == 0) atomicOr(status_word, TB_STATUS_INTERNAL);
}

template <bool MIXED>
__global__ __launch_bounds__(kUpperThreads) void k_upper(
    const int32_t *__restrict__ upper, const uint32_t *__restrict__ upper_cnt, int64_t upper_cap,
    const int64_t *__restrict__ n_cells, const int64_t *__restrict__ set_cells, int32_t nsets,
    const double *__restrict__ box, BlockOut o, int dhi, int dlo,
    int32_t *__restrict__ status_word) {
  bool bad = false;
  const int64_t C = *n_cells;
  for (int d = dhi; d >= dlo; --d) {
    const int64_t cnt = min((int64_t)upper_cnt[d], upper_cap);
    for (int64_t k = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; k < cnt;
         k += (int64_t)gridDim.x * blockDim.x) {
      const int64_t p = upper[(int64_t)d * upper_cap + k];
      if (p < 0 || p >= C) {
        bad = true;
        continue;
      }
      // the children: consecutive at depth d + 1, each with key >> 3 == this key
      const uint64_t key = o.cell_key[p];
      const int64_t c0 = o.child_ptr[2 * p];
      int nch = 0;
      while (nch < 8 && c0 >= 0 && c0 + nch < C && (o.cell_key[c0 + nch] >> 3) == key &&
             o.cell_level[c0 + nch] == d + 1)
        ++nch;
      if (nch == 0) {
        bad = true;
        continue;
      }
      const int b = nsets == 1 ? 0 : upper_index(set_cells, nsets + 1, p);
      parent_moments<MIXED>(o, p, c0, nch, d, box[4 * b + 3]);
    }
    // one workgroup runs every depth in one launch; a wider grid gets one launch per depth
    if (gridDim.x == 1) __syncthreads();
  }
  if (__ballot(bad) != 0 && lane_id() == 0) atomicOr(status_word, TB_STATUS_INTERNAL);
}

static BlockOut block_out(const Plan &p, const Work &w, const tb_tree &out) {
  BlockOut o;
  o.cell_key = out.cell_key;
  o.cell_level = out.cell_level;
  o.cell_first = out.cell_first;
  o.cell_count = out.cell_count;
  o.child_ptr = out.child_ptr;
  o.com = out.com;
  o.quad = out.quad;
  o.m_lo = w.m_lo;
  o.upper = w.upper;
  o.upper_cnt = w.counters + kUpperCounter;
  o.upper_cap = p.upper_cap;
  o.c_max = p.c_max;
  o.hilbert = (p.flags & TB_HILBERT) != 0;
  return o;
}

hipError_t launch_blocks(const Plan &p, const Work &w, hipStream_t s) {
  k_blocks<<<(unsigned)p.cell_tiles, kCellThreads, 0, s>>>(sorted_keys(p, w), w.tile_start,
                                                           w.tile_set, w.set_off, p.nsets, w.blk);
  return hipGetLastError();
}

hipError_t launch_block_build(const Plan &p, const Work &w, const tb_tree &out, hipStream_t s) {
  const BlockOut o = block_out(p, w, out);
  auto k = (p.flags & 0xffu) == TB_MIXED ? k_block_build<true> : k_block_build<false>;
  k<<<(unsigned)p.cell_tiles, kCellThreads, 0, s>>>(
      sorted_keys(p, w), w.ad, w.blk, p.n_leaf, w.cell_excl, p.cell_tiles, w.tile_start,
      w.tile_set, w.set_off, p.nsets, w.lvl_off, w.box, w.sorted, o, out.status);
  return hipGetLastError();
}

hipError_t launch_upper(const Plan &p, const Work &w, const tb_tree &out, hipStream_t s) {
  const BlockOut o = block_out(p, w, out);
  auto k = (p.flags & 0xffu) == TB_MIXED ? k_upper<true> : k_upper<false>;
  if (p.nsets == 1) {
    k<<<1, kUpperThreads, 0, s>>>(w.upper, o.upper_cnt, p.upper_cap, out.n_cells, w.set_cells,
                                  p.nsets, w.box, o, kMaxDepth - 1, 0, out.status);
  } else {
    int64_t grid = (p.upper_cap + kUpperThreads - 1) / kUpperThreads;
    if (grid > 256) grid = 256;
    for (int d = kMaxDepth - 1; d >= 0; --d)
      k<<<(unsigned)grid, kUpperThreads, 0, s>>>(w.upper, o.upper_cnt, p.upper_cap, out.n_cells,
                                                 w.set_cells, p.nsets, w.box, o, d, d, out.status);
  }
  return hipGetLastError();
}

}  // namespace tb
