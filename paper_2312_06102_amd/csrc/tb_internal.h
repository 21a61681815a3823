// tb_internal.h -- shared definitions of the gfx950 tree-build kernels.
//
// Internal to the library: kernels, launch wrappers, the workspace plan and a
// few wave64 helpers.  The public C ABI is include/treebuild.h.
//
// Every build is a batch of B >= 1 independent particle sets stored back to
// back (a single build is the batch B = 1).  Set b owns particles
// [set_off[b], set_off[b+1]) in the input and, after the sort, the same range
// of sorted positions; its cells are one contiguous, (depth, key)-ordered block.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include <type_traits>

#include "treebuild.h"

namespace tb {

// ---------------------------------------------------------------------------
// Fixed configuration
// ---------------------------------------------------------------------------
constexpr int kMaxDepth = TB_MAX_DEPTH;         // deepest cell (21 bits per axis)
constexpr int kLevels = kMaxDepth + 1;          // depths 0..21
constexpr int kLevelWords = (kLevels + 1) / 2;  // 16-bit level counters packed in u32

// Cell kernels: one tile of particles (never straddling two sets) per workgroup.
constexpr int kCellThreads = 256;
constexpr int kCellIpt = 8;
constexpr int kCellTile = kCellThreads * kCellIpt;  // 2048 particles


// The chip's eight XCDs each have their own L2, and workgroups of a launch are
// dispatched to them in turn (workgroup b to XCD b mod 8).
// Smallest radix grid whose passes count their tiles rather than look back.
constexpr int64_t kCountedMinTiles = 512;
constexpr uint32_t kXcds = 8;

// Parent kernel: children staged per workgroup step.
constexpr int kParentThreads = 256;
constexpr int kParentChunk = kParentThreads;

// Chunks of at most kBboxChunk particles of one set (the auto box).
constexpr int kBboxChunk = 65536;

// Largest number of sets in one batch.
constexpr int kMaxSetsLds = TB_MAX_SETS;

// counters[kOversizeCounter]: nonzero when a batch set is larger than the
// bound TB_SET_INDEX_BITS gives (set by the setup, read by the reorder)
constexpr int kOversizeCounter = 16;

// counters[kUpperCounter + d]: number of cells above the blocks at depth d
constexpr int kUpperCounter = 32;

// Lookback status word: flag in bits 63:62, value in bits 31:0.
constexpr uint64_t kFlagAggregate = 1ull << 62;
constexpr uint64_t kFlagInclusive = 2ull << 62;
constexpr uint64_t kFlagMask = 3ull << 62;

// Sort configuration chosen for one build (radix digit width and tile shape).
struct SortConfig {
  int bits;     // radix digit width, 8..9
  int ipt;      // keys per thread
  int threads;  // threads per workgroup
  int tile() const { return ipt * threads; }
  int radix() const { return 1 << bits; }
  int passes() const { return (63 + bits - 1) / bits; }  // bit 63 is always 1
};

// What one radix pass reads or writes per element.  The index is the element's
// position before the sort (perm after the last pass); a packed element holds the
// key bits later passes still need above the index bits.
enum SortForm : uint8_t {
  kFormIdx = 0,     // the index alone (the last pass's output)
  kFormKey64 = 2,   // the 64-bit key, with the index in a separate u32 array
  kFormPack64 = 3,  // (key >> consumed bits) << idx_bits | index, in 64 bits
  kFormPack32 = 4,  // the same in 32 bits
};
constexpr int kMaxKeyPasses = 8;
// One radix digit as the counted passes store it between passes.
template <int BITS>
using DigitType = typename std::conditional<(BITS > 8), uint16_t, uint8_t>::type;

// Workspace plan: byte offsets of every scratch array inside the caller's
// workspace, all 256-byte aligned.
struct Plan {
  int64_t n;        // particles in the batch
  int32_t n_leaf;
  uint32_t flags;
  int32_t nsets;    // B
  SortConfig sort;
  int key_passes;   // radix passes over the 63 key bits
  uint32_t counted; // bit k: key pass k takes its tile offsets from a count and a scan
  int idx_bits;     // bits of the largest index, n - 1 (at least 1); in a batch the index
                    // is the position within the set
  int set_index_bits;  // batch: TB_SET_INDEX_BITS (0: none), checked against every set
  uint8_t form[kMaxKeyPasses + 1];  // form[k]: what pass k reads; form[k + 1]: what it writes
  bool seg;         // batch of several sets: every radix pass sorts each set in place
                    // (tiles never straddle a set; each set has its own digit bases)
  int64_t sort_tiles;
  int64_t cell_tiles;   // upper bound of the cell tiles of all sets
  int64_t bbox_chunks;  // upper bound of the bounding-box chunks of all sets
  int64_t c_max;
  int64_t upper_cap;    // cells above the blocks, per depth: at most n / (n_serial + 1) + B
  // offsets
  size_t keys0, keys1;  // u64 [n] ping-pong buffers of keys or packed words
  size_t vals1;         // u32 [n] payload buffer (the other one is out->perm)
  size_t hist;          // u32 [key_passes][radix] global digit counts, then bases (single set)
  size_t hist_part;     // u32 [keygen blocks][key_passes][radix] per-workgroup counts
  size_t status0, status1;  // u64 [sort_tiles][radix] look-back words (alternating passes)
  size_t counters;      // u32 [64] dynamic tile counters
  size_t tile_off;      // u32 [radix][sort_tiles] digit counts of every tile, then their
                        // exclusive prefix over the tiles (counted passes)
  size_t dig;           // u8 (u16 for 9-bit digits) [n] counted passes: the next pass's
                        // digit of every element
  size_t set_off;       // i64 [B + 1] particle offsets of the sets
  size_t box;           // f64 [B][4] the root box of each set
  size_t bbox_part;     // f64 [bbox_chunks][6] per-chunk min/max
  size_t chunk_start;   // i64 [B + 1] first bounding-box chunk of each set
  size_t chunk_set;     // i32 [bbox_chunks] set of each bounding-box chunk
  size_t tile_start;    // i64 [B + 1] first cell tile of each set
  size_t tile_set;      // i32 [cell_tiles] set of each cell tile
  size_t cell_cnt;      // u32 [kLevels][cell_tiles] per-tile cell counts per depth
  size_t cell_excl;     // u32 [kLevels][cell_tiles] prefix over the earlier tiles of the set
  size_t set_tot;       // u32 [B][kLevels] cells of each set and depth
  size_t set_cells;     // i64 [B + 1] first cell of each set; [B] = all cells
  size_t lvl_off;       // i64 [B][kLevels + 1] first cell of each depth of each set
  size_t set_wg;        // i64 [ceil(B / 256)][kLevels] row sums of each set-scan workgroup
  size_t par_start;     // i64 [kLevels][B + 1] parent-pass chunks per depth and set
  size_t seg_tile_start;  // i64 [B + 1] first radix tile of each set (seg)
  size_t seg_tile_set;    // i32 [sort_tiles] set of each radix tile (seg)
  size_t seg_base;        // u32 [B][key_passes][radix] digit counts of each set, then the
                          // position where each digit's run of the set starts (seg)
  size_t packed;        // f32x4 [n] (x, y, z, m) records in original order
  size_t sorted;        // f32x4 [n] the same records in key order
  size_t ad;            // u16 [n] a_i | D_i << 8 of every particle in key order
  size_t head_parent;   // i32 [c_max] parent slot of every first child
  size_t blk;           // u8 [n] root depth of the block a particle starts, or 0xff
  size_t upper;         // i32 [kLevels][upper_cap] slots of the cells above the blocks
  size_t m_lo;          // f32 [c_max] compensation of each cell mass (mixed precision)
  size_t total;
};

int make_plan(int64_t n, int32_t nsets, int32_t n_leaf, uint32_t flags, const SortConfig &sc,
              Plan *p);

// Device views of the workspace
struct Work {
  uint64_t *keys0, *keys1;
  uint32_t *vals1;
  uint32_t *hist;
  uint32_t *hist_part;
  uint64_t *status0, *status1;
  uint32_t *counters;
  uint32_t *tile_off;
  void *dig;
  int64_t *set_off;
  double *box;
  double *bbox_part;
  int64_t *chunk_start;
  int32_t *chunk_set;
  int64_t *tile_start;
  int32_t *tile_set;
  uint32_t *cell_cnt;
  uint32_t *cell_excl;
  uint32_t *set_tot;
  int64_t *set_cells;
  int64_t *lvl_off;
  int64_t *set_wg;
  int64_t *par_start;
  int64_t *seg_tile_start;
  int32_t *seg_tile_set;
  uint32_t *seg_base;
  float4 *packed;
  float4 *sorted;
  uint16_t *ad;
  int32_t *head_parent;
  uint8_t *blk;
  int32_t *upper;
  float *m_lo;
};

Work carve(const Plan &p, void *base);

// Where the set description comes from.
struct BatchIn {
  const int64_t *set_off;  // device [B + 1], or NULL for B == 1 (then {0, n})
  const tb_box *host_box;  // single build: the caller's box (host), or NULL
  const tb_box *dev_boxes; // batch: device [B], or NULL
  bool auto_box;           // derive each set's box from its particles
};

// ---------------------------------------------------------------------------
// Launch wrappers (each defined in the .hip file that holds the kernel)
// ---------------------------------------------------------------------------
// tb_keys.hip
hipError_t launch_init(const Plan &p, const Work &w, const BatchIn &in, const tb_tree &out,
                       hipStream_t s);
hipError_t launch_setup(const Plan &p, const Work &w, const BatchIn &in, int32_t *status,
                        hipStream_t s);
hipError_t launch_bbox(const Plan &p, const Work &w, const float *pos, hipStream_t s);
hipError_t launch_keygen(const Plan &p, const Work &w, const float *pos, const float *mass,
                         const tb_tree &out, hipStream_t s);
hipError_t launch_hist_reduce(const Plan &p, const Work &w, hipStream_t s);
int keygen_blocks(int64_t n);
hipError_t launch_empty(const tb_tree &out, int32_t nsets, const BatchIn &in,
                        int64_t *cell_offsets, hipStream_t s);
// tb_sort.hip
hipError_t launch_sort_pass(const Plan &p, const Work &w, int pass, const tb_tree &out,
                            hipStream_t s);
bool sort_config_supported(const SortConfig &c);
// tb_cells.hip
hipError_t launch_cell_scan(const Plan &p, const Work &w, const tb_tree &out,
                            int64_t *cell_offsets, hipStream_t s);
hipError_t launch_reorder(const Plan &p, const Work &w, const tb_tree &out, hipStream_t s);
size_t cell_lds_limit();
size_t cell_reorder_lds(int nl);
hipError_t launch_cell_emit(const Plan &p, const Work &w, const tb_tree &out, hipStream_t s);
size_t cell_emit_lds(int nl);
// tb_parents.hip
hipError_t launch_parents(const Plan &p, const Work &w, int depth, const tb_tree &out,
                          hipStream_t s);
// tb_blocks.hip
hipError_t launch_blocks(const Plan &p, const Work &w, hipStream_t s);
hipError_t launch_block_build(const Plan &p, const Work &w, const tb_tree &out, hipStream_t s);
hipError_t launch_upper(const Plan &p, const Work &w, const tb_tree &out, hipStream_t s);

// tb_gravity.hip
struct GravIn {
  const float *pos_sorted;  // [n][3] device, key order
  const float *mass_sorted; // [n] device, key order
  int64_t n;
  const tb_tree *tree;      // an FP64 build's outputs (box_out required)
  int64_t c_max;
  double theta, eps;
  int32_t n_crit;
  bool quadrupole;
  bool hilbert;             // the tree was built on Peano-Hilbert keys
  double *acc;              // [n][4] device: ax, ay, az, phi in key order
  int64_t *stats;           // [2] device or NULL: groups, interactions
  void *workspace;          // int32 [c_max] groups + u32 counter
};
hipError_t launch_gravity(const GravIn &in, hipStream_t s);
// tb_sim.hip
hipError_t launch_kick_drift(const int32_t *perm, const double *acc, int64_t n, double dt_kick,
                             double dt_drift, float *pos, float *vel, int32_t *status,
                             hipStream_t s);
hipError_t launch_permute(const int32_t *perm, int64_t n, const void *src, int32_t width,
                          void *dst, int32_t *status, hipStream_t s);
size_t gravity_workspace_bytes(int64_t c_max);

// The sorted keys, recomputed from the sorted particles by the reorder pass (the
// sort passes themselves stop carrying the key once its bits are consumed).
inline uint64_t *sorted_keys(const Plan &, const Work &w) { return w.keys0; }

// ---------------------------------------------------------------------------
// Device helpers
// ---------------------------------------------------------------------------
#if defined(__HIP_DEVICE_COMPILE__) || defined(__HIPCC__)

__device__ __forceinline__ int lane_id() { return __lane_id(); }

// Tile of workgroup b in a grid of nb: XCD x takes a contiguous run of the
// tiles, in order, so that the partial cache lines where consecutive tiles'
// output runs meet are written through one L2.  A bijection of [0, nb).
__device__ __forceinline__ uint32_t xcd_tile(uint32_t b, uint32_t nb) {
  const uint32_t q = nb / kXcds, r = nb % kXcds, x = b % kXcds;
  return x * q + (x < r ? x : r) + b / kXcds;
}

__device__ __forceinline__ uint64_t lanemask_lt() {
  return (uint64_t(1) << lane_id()) - 1u;
}

__device__ __forceinline__ uint64_t atomic_load_agent(const uint64_t *p) {
  return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

__device__ __forceinline__ void atomic_store_agent(uint64_t *p, uint64_t v) {
  __hip_atomic_store(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

// Waits until a look-back word is published.  Predecessor tiles always publish,
// so the wait is short; the bound only turns a broken invariant into an error
// flag (and an exit) instead of a hang.
constexpr uint32_t kSpinLimit = 1u << 25;

__device__ inline uint64_t wait_published(const uint64_t *p, bool &timed_out) {
  uint64_t sw = atomic_load_agent(p);
  uint32_t spins = 0;
  while ((sw & kFlagMask) == 0) {
    if (++spins > kSpinLimit) {
      timed_out = true;
      return kFlagInclusive;
    }
    __builtin_amdgcn_s_sleep(1);
    sw = atomic_load_agent(p);
  }
  return sw;
}

// Exclusive prefix of column `col` over tiles [0, tile) by decoupled look-back:
// every tile publishes its own count (aggregate) as soon as it has it and its
// inclusive prefix once known; a successor sums predecessors' words backwards
// until it meets an inclusive one.  W predecessor words are requested at once,
// so a chain of aggregates costs one memory round trip per W tiles.
template <int W>
__device__ inline uint32_t lookback(const uint64_t *status, int64_t stride, int64_t tile, int col,
                                    bool &timed_out) {
  uint32_t excl = 0;
  int64_t q = tile - 1;
  while (q >= 0) {
    uint64_t sw[W];
#pragma unroll
    for (int k = 0; k < W; ++k)
      sw[k] = (q - k >= 0) ? atomic_load_agent(&status[(q - k) * stride + col]) : kFlagInclusive;
    bool done = false;
#pragma unroll
    for (int k = 0; k < W; ++k) {
      if (!done) {
        uint64_t v = sw[k];
        if ((v & kFlagMask) == 0) v = wait_published(&status[(q - k) * stride + col], timed_out);
        excl += (uint32_t)v;
        done = (v & kFlagMask) == kFlagInclusive;
      }
    }
    if (done) break;
    q -= W;
  }
  return excl;
}

// Spread the low 21 bits of v so that bit b lands on bit 3b.
__device__ __forceinline__ uint64_t spread3(uint64_t v) {
  v &= 0x1fffffull;
  v = (v | (v << 32)) & 0x001f00000000ffffull;
  v = (v | (v << 16)) & 0x001f0000ff0000ffull;
  v = (v | (v << 8)) & 0x100f00f00f00f00full;
  v = (v | (v << 4)) & 0x10c30c30c30c30c3ull;
  v = (v | (v << 2)) & 0x1249249249249249ull;
  return v;
}

// floor(fl64(x - lo) * scale) clamped to [0, 2^21 - 1]; scale = 2^21 / side is a
// power of two, so the multiply is exact and only the subtraction rounds
// (Sec. 2.2: each coordinate becomes a 21-bit integer inside the root cube).
__device__ __forceinline__ uint32_t quantise(float x, double lo, double scale) {
  const double u = __dsub_rn((double)x, lo);
  const double t = __dmul_rn(u, scale);
  if (!(t >= 0.0)) return 0u;
  if (t >= 2097152.0) return 2097151u;
  return (uint32_t)t;  // truncation == floor for t >= 0
}

// 64-bit key: a leading 1, then per depth the octant digit (x, y, z) with x the
// most significant bit (Sec. 2.2).
__device__ __forceinline__ uint64_t morton_key(float x, float y, float z, double lo0,
                                               double lo1, double lo2, double scale) {
  const uint64_t qx = quantise(x, lo0, scale);
  const uint64_t qy = quantise(y, lo1, scale);
  const uint64_t qz = quantise(z, lo2, scale);
  return (1ull << 63) | (spread3(qx) << 2) | (spread3(qy) << 1) | spread3(qz);
}

// Peano-Hilbert variant of the key (footnote of Sec. 2.2): the same layout,
// but the 63 bits below the leading 1 are the cell's index on the 3-D Hilbert
// curve of Skilling's transpose method (AIP Conf. Proc. 707, 381, 2004).  From
// the top level down, an axis whose bit is set inverts the lower bits of x and
// an axis whose bit is clear swaps its lower bits with x's; a Gray-code decode
// along (x, y, z) follows.  Each level's bits of the transposed (x, y, z) are
// that level's 3-bit digit, x the most significant, so the top 3d bits are the
// index of the particle's depth-d cell on the d-level curve.
__device__ __forceinline__ uint64_t hilbert_index21(uint32_t x, uint32_t y, uint32_t z) {
  for (uint32_t bit = 1u << 20; bit > 1u; bit >>= 1) {
    const uint32_t low = bit - 1u;
    if (x & bit) x ^= low;
    if (y & bit) {
      x ^= low;
    } else {
      const uint32_t t = (x ^ y) & low;
      x ^= t;
      y ^= t;
    }
    if (z & bit) {
      x ^= low;
    } else {
      const uint32_t t = (x ^ z) & low;
      x ^= t;
      z ^= t;
    }
  }
  y ^= x;
  z ^= y;
  // bit j of the correction: parity of z's bits above j
  uint32_t t = z >> 1;
  t ^= t >> 1;
  t ^= t >> 2;
  t ^= t >> 4;
  t ^= t >> 8;
  t ^= t >> 16;
  x ^= t;
  y ^= t;
  z ^= t;
  return (spread3(x) << 2) | (spread3(y) << 1) | spread3(z);
}

// Key of a particle: Morton (interleaved coordinates) or Peano-Hilbert, each
// below a leading 1.
__device__ __forceinline__ uint64_t particle_key(float x, float y, float z, double lo0, double lo1,
                                                 double lo2, double scale, bool hilbert) {
  if (!hilbert) return morton_key(x, y, z, lo0, lo1, lo2, scale);
  return (1ull << 63) | hilbert_index21(quantise(x, lo0, scale), quantise(y, lo1, scale),
                                        quantise(z, lo2, scale));
}

// Minimum distinguished depth of two particle keys (Sec. 2.3.1): leading zeros
// of the XOR divided by three, rounded up; identical keys give 22.
__device__ __forceinline__ int min_depth(uint64_t a, uint64_t b) {
  uint64_t x = a ^ b;
  int z = x ? __clzll(static_cast<long long>(x)) : 64;
  return (z + 2) / 3;
}

// Inclusive wave64 scan of a u32 (shuffle-based).
__device__ __forceinline__ uint32_t wave_inclusive_scan(uint32_t v) {
  const int l = lane_id();
#pragma unroll
  for (int o = 1; o < 64; o <<= 1) {
    uint32_t t = __shfl_up(v, o, 64);
    if (l >= o) v += t;
  }
  return v;
}

// Index b of the last entry of the sorted table tab[0..count) with tab[b] <= x
// (the set holding position x when tab holds the set offsets).
template <typename T>
__device__ __forceinline__ int upper_index(const T *tab, int count, int64_t x) {
  int lo = 0, hi = count - 1;  // invariant: tab[lo] <= x
  while (lo < hi) {
    const int mid = (lo + hi + 1) >> 1;
    if ((int64_t)tab[mid] <= x)
      lo = mid;
    else
      hi = mid - 1;
  }
  return lo;
}

#endif

}  // namespace tb
