// tb_api.cpp -- the C ABI of include/treebuild.h: argument checks, workspace
// plan, the fixed launch sequence of a build or a batch of builds, and
// kernel timing.
#include <cfloat>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <map>
#include <mutex>
#include <string>
#include <vector>

#include "tb_internal.h"

namespace tb {

// Table of sort shapes selectable through TB_SORT_CONFIG(k); entry 0 is the default.
static const SortConfig kSortTable[] = {
    {8, 11, 512}, {8, 12, 512}, {8, 10, 512}, {8, 16, 256},
    {9, 16, 256}, {8, 12, 256}, {8, 8, 512},
};
static const int kSortTableSize = (int)(sizeof(kSortTable) / sizeof(kSortTable[0]));

static size_t align256(size_t x) { return (x + 255) & ~size_t(255); }

// Internal plan flag: the root boxes are derived from the data.
constexpr uint32_t kAutoBoxFlag = 0x10000u;

static int64_t max_cells(int64_t n, int32_t n_leaf) {
  if (n <= 0) return 0;
  return n + (int64_t)kMaxDepth * (n / ((int64_t)n_leaf + 1));
}

int make_plan(int64_t n, int32_t nsets, int32_t n_leaf, uint32_t flags, const SortConfig &sc,
              Plan *p) {
  std::memset(p, 0, sizeof(*p));
  p->n = n;
  p->n_leaf = n_leaf;
  p->flags = flags;
  p->nsets = nsets;
  p->sort = sc;
  p->key_passes = sc.passes();
  // A batch sorts every set in place (tiles aligned to the sets, per-set digit
  // bases), so no radix pass over the set id is needed.
  p->seg = nsets > 1;
  // each set starts a tile of its own
  p->sort_tiles = (n + sc.tile() - 1) / sc.tile() + (p->seg ? nsets : 0);
  // Element formats.  The index needs idx_bits bits; once the key bits still to
  // be sorted fit beside it in 64 (or 32) bits, key and index travel as one
  // packed word, so every later pass moves 8 (or 4) bytes an element in and out
  // instead of 12.  With 8-bit digits and N = 2^24 the third pass writes 40 key
  // bits + 24 index bits in 8 bytes, and the seventh 8 + 24 bits in 4.
  p->idx_bits = 1;
  while (p->idx_bits < 32 && (int64_t{1} << p->idx_bits) < n) ++p->idx_bits;
  // a batch sorts its sets in place, so an index within the set suffices: the
  // caller may bound the set size (TB_SET_INDEX_BITS), which k_setup checks
  p->set_index_bits = p->seg ? (int)((flags >> 24) & 0x1fu) : 0;
  if (p->set_index_bits > 0 && p->set_index_bits < p->idx_bits) p->idx_bits = p->set_index_bits;
  // The leading 1 at bit 63 stays in the word (the key kernel's counts of the
  // last 8-bit digit include it), so key >> consumed bits keeps 64 - consumed bits.
  p->form[0] = kFormKey64;
  for (int k = 0; k < p->key_passes; ++k) {
    const int rem = 64 - (k + 1) * sc.bits;  // bits of key >> consumed bits after pass k
    if (k + 1 == p->key_passes)
      p->form[k + 1] = kFormIdx;
    else if (rem + p->idx_bits <= 32)
      p->form[k + 1] = kFormPack32;
    else if (rem + p->idx_bits <= 64)
      p->form[k + 1] = kFormPack64;
    else
      p->form[k + 1] = kFormKey64;
  }
  // The passes of a single set with at least kCountedMinTiles tiles count their
  // tiles' digits first (reduce, then scan) instead of chaining the tiles
  // through the look-back.  The count reads one digit byte an element, which the
  // previous pass (or the key kernel) leaves behind: at N = 2^24 the sort takes
  // 779 us counted against 865 us with look-back, at 2^26 2.99 ms against
  // 3.25 ms; a whole build at 2^22 (745 tiles) 0.636 against 0.649 ms.  Smaller
  // grids look back: a counted pass is three launches where a look-back pass is
  // one (2^21, 373 tiles: 0.443 against 0.419 ms).  A batch looks back too (its
  // 31,180 set-aligned tiles: 7.0 ms against 8.7 ms counted).  TB_SORT_COUNTED
  // counts every pass of any build, a batch's too (there a tile's offsets start
  // again at its set's first tile); TB_SORT_LOOKBACK looks back everywhere.
  p->counted = 0;
  if (!(flags & TB_SORT_LOOKBACK) &&
      ((flags & TB_SORT_COUNTED) || (!p->seg && p->sort_tiles >= kCountedMinTiles)))
    p->counted = (1u << p->key_passes) - 1u;
  // tiles never straddle two sets: at most one partial tile per set
  p->cell_tiles = (n + kCellTile - 1) / kCellTile + nsets;
  // chunks of at most kBboxChunk particles of one set: the auto box works chunk
  // by chunk
  p->bbox_chunks = (flags & kAutoBoxFlag) ? (n + kBboxChunk - 1) / kBboxChunk + nsets : 1;
  // a set of n_b particles has at most n_b + 21 floor(n_b / (n_leaf + 1)) cells,
  // and the sum over the sets is bounded by the same expression of n
  p->c_max = max_cells(n, n_leaf);
  const int P = p->key_passes, R = sc.radix();
  const size_t B1 = (size_t)nsets + 1;
  size_t off = 0;
  auto take = [&](size_t bytes) {
    const size_t o = off;
    off = align256(off + (bytes ? bytes : 1));
    return o;
  };
  p->keys0 = take(8 * (size_t)n);
  p->keys1 = take(8 * (size_t)n);
  p->vals1 = take(4 * (size_t)n);
  p->hist = take(4 * (size_t)P * R);
  p->hist_part = take(4 * (size_t)keygen_blocks(n) * p->key_passes * R);
  p->status0 = take(8 * (size_t)p->sort_tiles * R);
  p->status1 = take(8 * (size_t)p->sort_tiles * R);
  p->counters = take(4 * 64);
  p->tile_off = take(4 * (size_t)p->sort_tiles * R);
  // (rounded to whole 32-bit words: the count kernel reads words)
  p->dig = take(p->counted ? ((size_t)n * (sc.bits > 8 ? 2 : 1) + 3) / 4 * 4 : 0);
  p->set_off = take(8 * B1);
  p->box = take(8 * 4 * (size_t)nsets);
  p->bbox_part = take(8 * 6 * (size_t)p->bbox_chunks);
  p->chunk_start = take(8 * B1);
  p->chunk_set = take(4 * (size_t)p->bbox_chunks);
  p->tile_start = take(8 * B1);
  p->tile_set = take(4 * (size_t)p->cell_tiles);
  p->cell_cnt = take(4 * (size_t)p->cell_tiles * kLevels);
  p->cell_excl = take(4 * (size_t)p->cell_tiles * kLevels);
  p->set_tot = take(4 * (size_t)nsets * kLevels);
  p->set_cells = take(8 * B1);
  p->lvl_off = take(8 * (size_t)nsets * (kLevels + 1));
  p->set_wg = take(8 * (size_t)((nsets + 255) / 256) * kLevels);
  p->par_start = take(8 * (size_t)kLevels * B1);
  p->seg_tile_start = take(p->seg ? 8 * B1 : 0);
  p->seg_tile_set = take(p->seg ? 4 * (size_t)p->sort_tiles : 0);
  p->seg_base = take(p->seg ? 4 * (size_t)nsets * p->key_passes * R : 0);
  p->packed = take(16 * (size_t)n);
  p->sorted = take(16 * (size_t)n);
  p->ad = take(2 * (size_t)n);
  if (flags & TB_SUBTREES) {
    p->blk = take((size_t)n);
    // the cells above the blocks at one depth are disjoint and each holds more
    // than n_serial particles
    p->upper_cap = n / (kCellTile + 1) + nsets;
    p->upper = take(4 * (size_t)kLevels * (size_t)p->upper_cap);
  } else {
    p->head_parent = take(4 * (size_t)p->c_max);
  }
  p->m_lo = take((flags & 0xffu) == TB_MIXED ? 4 * (size_t)p->c_max : 0);
  p->total = off;
  return TB_OK;
}

Work carve(const Plan &p, void *base) {
  unsigned char *b = static_cast<unsigned char *>(base);
  Work w;
  w.keys0 = reinterpret_cast<uint64_t *>(b + p.keys0);
  w.keys1 = reinterpret_cast<uint64_t *>(b + p.keys1);
  w.vals1 = reinterpret_cast<uint32_t *>(b + p.vals1);
  w.hist = reinterpret_cast<uint32_t *>(b + p.hist);
  w.hist_part = reinterpret_cast<uint32_t *>(b + p.hist_part);
  w.status0 = reinterpret_cast<uint64_t *>(b + p.status0);
  w.status1 = reinterpret_cast<uint64_t *>(b + p.status1);
  w.counters = reinterpret_cast<uint32_t *>(b + p.counters);
  w.tile_off = reinterpret_cast<uint32_t *>(b + p.tile_off);
  w.dig = b + p.dig;
  w.set_off = reinterpret_cast<int64_t *>(b + p.set_off);
  w.box = reinterpret_cast<double *>(b + p.box);
  w.bbox_part = reinterpret_cast<double *>(b + p.bbox_part);
  w.chunk_start = reinterpret_cast<int64_t *>(b + p.chunk_start);
  w.chunk_set = reinterpret_cast<int32_t *>(b + p.chunk_set);
  w.tile_start = reinterpret_cast<int64_t *>(b + p.tile_start);
  w.tile_set = reinterpret_cast<int32_t *>(b + p.tile_set);
  w.cell_cnt = reinterpret_cast<uint32_t *>(b + p.cell_cnt);
  w.cell_excl = reinterpret_cast<uint32_t *>(b + p.cell_excl);
  w.set_tot = reinterpret_cast<uint32_t *>(b + p.set_tot);
  w.set_cells = reinterpret_cast<int64_t *>(b + p.set_cells);
  w.lvl_off = reinterpret_cast<int64_t *>(b + p.lvl_off);
  w.set_wg = reinterpret_cast<int64_t *>(b + p.set_wg);
  w.par_start = reinterpret_cast<int64_t *>(b + p.par_start);
  w.seg_tile_start = reinterpret_cast<int64_t *>(b + p.seg_tile_start);
  w.seg_tile_set = reinterpret_cast<int32_t *>(b + p.seg_tile_set);
  w.seg_base = reinterpret_cast<uint32_t *>(b + p.seg_base);
  w.packed = reinterpret_cast<float4 *>(b + p.packed);
  w.sorted = reinterpret_cast<float4 *>(b + p.sorted);
  w.ad = reinterpret_cast<uint16_t *>(b + p.ad);
  w.head_parent = reinterpret_cast<int32_t *>(b + p.head_parent);
  w.blk = b + p.blk;
  w.upper = reinterpret_cast<int32_t *>(b + p.upper);
  w.m_lo = reinterpret_cast<float *>(b + p.m_lo);
  return w;
}

// ---------------------------------------------------------------------------
// kernel timing
// ---------------------------------------------------------------------------
struct TraceRec {
  const char *name;
  hipEvent_t a, b;
};
struct TraceAcc {
  int64_t launches = 0;
  double ms = 0.0;
};
static bool g_trace = false;
static std::vector<TraceRec> g_pending;
static std::map<std::string, TraceAcc> g_acc;

template <class F>
static hipError_t traced(bool on, const char *name, hipStream_t s, F &&f) {
  if (!on) return f();
  TraceRec r{name, nullptr, nullptr};
  if (hipEventCreate(&r.a) != hipSuccess || hipEventCreate(&r.b) != hipSuccess) return hipErrorOutOfMemory;
  (void)hipEventRecord(r.a, s);
  const hipError_t e = f();
  (void)hipEventRecord(r.b, s);
  g_pending.push_back(r);
  return e;
}

static int flush_trace() {
  for (auto &r : g_pending) {
    float ms = 0.f;
    if (hipEventSynchronize(r.b) == hipSuccess && hipEventElapsedTime(&ms, r.a, r.b) == hipSuccess) {
      TraceAcc &acc = g_acc[r.name];
      acc.launches += 1;
      acc.ms += ms;
    }
    (void)hipEventDestroy(r.a);
    (void)hipEventDestroy(r.b);
  }
  g_pending.clear();
  return TB_OK;
}

// ---------------------------------------------------------------------------
// argument checks
// ---------------------------------------------------------------------------
// positive, finite, normal power of two (the same test the device applies to
// boxes it receives)
static bool is_pow2(double side) {
  if (!(side >= DBL_MIN) || !std::isfinite(side)) return false;
  int e;
  return std::frexp(side, &e) == 0.5;
}

static int check_sizes(int64_t n, int32_t n_leaf) {
  if (n < 0 || n > TB_MAX_N) return TB_ERR_ARG;
  if (n_leaf < 1 || n_leaf > TB_MAX_NLEAF) return TB_ERR_ARG;
  if (max_cells(n, n_leaf) > 2147483647LL) return TB_ERR_ARG;  // child_ptr is int32
  return TB_OK;
}

static int config_from_flags(uint32_t flags, SortConfig *sc) {
  const uint32_t prec = flags & 0xffu;
  if (prec != TB_FP64 && prec != TB_MIXED) return TB_ERR_ARG;
  if (flags & ~(0xffffu | TB_SORT_LOOKBACK | TB_SUBTREES | TB_SORT_COUNTED | TB_HILBERT |
                TB_SET_INDEX_BITS(31)))
    return TB_ERR_ARG;
  if ((flags & TB_SORT_LOOKBACK) && (flags & TB_SORT_COUNTED)) return TB_ERR_ARG;
  const int k = (int)((flags >> 8) & 0xffu);
  if (k >= kSortTableSize) return TB_ERR_ARG;
  *sc = kSortTable[k];
  return sort_config_supported(*sc) ? TB_OK : TB_ERR_ARG;
}

static bool box_ok(const tb_box &b) {
  return std::isfinite(b.lo[0]) && std::isfinite(b.lo[1]) && std::isfinite(b.lo[2]) &&
         is_pow2(b.side);
}

// The launch sequence of one batch of nsets sets; a single build is nsets == 1.
static int build_impl(const float *pos, const float *mass, int64_t n, int32_t nsets,
                      int32_t n_leaf, const BatchIn &in, uint32_t flags, void *workspace,
                      size_t ws_bytes, const tb_tree *out, int64_t *cell_offsets,
                      hipStream_t s, bool allow_trace = true) {
  int rc = check_sizes(n, n_leaf);
  if (rc) return rc;
  if (nsets < 1 || nsets > kMaxSetsLds) return TB_ERR_ARG;
  SortConfig sc;
  rc = config_from_flags(flags, &sc);
  if (rc) return rc;
  if (!out || !out->level_offset || !out->n_cells || !out->status) return TB_ERR_ARG;
  if (in.host_box && !box_ok(*in.host_box)) return TB_ERR_BOX;
  // the timing events are host resources a no-allocation caller must not get
  const bool trace = allow_trace && g_trace;
  if (n == 0) {
    return traced(trace, "empty", s,
                  [&] { return launch_empty(*out, nsets, in, cell_offsets, s); }) == hipSuccess
               ? TB_OK
               : TB_ERR_HIP;
  }
  if (!pos || !mass || !out->perm || !out->cell_key || !out->cell_level || !out->cell_first ||
      !out->cell_count || !out->child_ptr || !out->com || !out->quad)
    return TB_ERR_ARG;
  Plan p;
  make_plan(n, nsets, n_leaf, flags | (in.auto_box ? kAutoBoxFlag : 0u), sc, &p);
  if (!workspace || ws_bytes < p.total) return TB_ERR_WORKSPACE;
  // the cell kernels stage a tile plus an n_leaf halo in LDS
  if (cell_emit_lds(n_leaf) > cell_lds_limit()) return TB_ERR_ARG;
  const Work w = carve(p, workspace);

  hipError_t e = hipSuccess;
  auto run = [&](const char *name, auto &&f) {
    if (e == hipSuccess) e = traced(trace, name, s, f);
  };
  run("init", [&] { return launch_init(p, w, in, *out, s); });
  run("setup", [&] { return launch_setup(p, w, in, out->status, s); });
  if (in.auto_box) run("bbox", [&] { return launch_bbox(p, w, pos, s); });
  run("keygen", [&] { return launch_keygen(p, w, pos, mass, *out, s); });
  run("hist_reduce", [&] { return launch_hist_reduce(p, w, s); });
  for (int pass = 0; pass < p.key_passes; ++pass)
    run("sort_pass", [&] { return launch_sort_pass(p, w, pass, *out, s); });
  run("reorder", [&] { return launch_reorder(p, w, *out, s); });
  run("cell_scan", [&] { return launch_cell_scan(p, w, *out, cell_offsets, s); });
  if (flags & TB_SUBTREES) {
    run("blocks", [&] { return launch_blocks(p, w, s); });
    run("block_build", [&] { return launch_block_build(p, w, *out, s); });
    run("upper", [&] { return launch_upper(p, w, *out, s); });
  } else {
    run("cell_emit", [&] { return launch_cell_emit(p, w, *out, s); });
    for (int d = kMaxDepth - 1; d >= 0; --d)
      run("parents", [&] { return launch_parents(p, w, d, *out, s); });
  }
  return e == hipSuccess ? TB_OK : TB_ERR_HIP;
}

// ---------------------------------------------------------------------------
// the build without allocation: workspace in a fixed device array
// ---------------------------------------------------------------------------
// Each GPU the library runs on holds its own copy of this array until the
// process ends.  Host code never uses the array's name as an address: its
// device address comes from hipGetSymbolAddress, once per device.
static __device__ __align__(256) unsigned char scratch[TB_NOALLOC_SCRATCH_BYTES];

constexpr int kMaxDevices = 64;
static std::mutex g_scratch_mu;
static void *g_scratch_ptr[kMaxDevices] = {};

// The current device's address of `scratch`, or NULL if it cannot be had.
static void *scratch_ptr() {
  int dev = -1;
  if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= kMaxDevices) return nullptr;
  std::lock_guard<std::mutex> lock(g_scratch_mu);
  if (!g_scratch_ptr[dev]) {
    void *ptr = nullptr;
    if (hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch)) != hipSuccess || !ptr) return nullptr;
    g_scratch_ptr[dev] = ptr;
  }
  return g_scratch_ptr[dev];
}

static int status_code(int32_t status) {
  if (status & TB_STATUS_NONFINITE) return TB_ERR_NONFINITE;
  if (status & TB_STATUS_MASS) return TB_ERR_MASS;
  if (status & TB_STATUS_SETS) return TB_ERR_ARG;
  if (status & TB_STATUS_BOX) return TB_ERR_BOX;
  if (status & TB_STATUS_INTERNAL) return TB_ERR_INTERNAL;
  return TB_OK;
}

static int wait_status(const tb_tree *out, hipStream_t s) {
  int32_t status = 0;
  if (hipMemcpyAsync(&status, out->status, sizeof(status), hipMemcpyDeviceToHost, s) != hipSuccess)
    return TB_ERR_HIP;
  if (hipStreamSynchronize(s) != hipSuccess) return TB_ERR_HIP;
  return status_code(status);
}

}  // namespace tb

// ---------------------------------------------------------------------------
// C ABI
// ---------------------------------------------------------------------------
extern "C" {

int tb_max_cells(int64_t n, int32_t n_leaf, int64_t *c_max) {
  if (!c_max) return TB_ERR_ARG;
  const int rc = tb::check_sizes(n, n_leaf);
  if (rc) return rc;
  *c_max = tb::max_cells(n, n_leaf);
  return TB_OK;
}

int tb_workspace_bytes_batched(int64_t n_total, int32_t nsets, int32_t n_leaf, uint32_t flags,
                               size_t *bytes) {
  if (!bytes) return TB_ERR_ARG;
  int rc = tb::check_sizes(n_total, n_leaf);
  if (rc) return rc;
  if (nsets < 1 || nsets > tb::kMaxSetsLds) return TB_ERR_ARG;
  tb::SortConfig sc;
  rc = tb::config_from_flags(flags, &sc);
  if (rc) return rc;
  if (n_total == 0) {
    *bytes = 0;
    return TB_OK;
  }
  // The cell kernels' LDS opt-in is a per-device attribute set once, here as
  // well as on the first build, so that a caller who sizes the workspace before
  // capturing a build into a graph makes no attribute call during the capture.
  (void)tb::cell_lds_limit();
  // sized for data-derived boxes, so one workspace serves both kinds of call
  tb::Plan p;
  tb::make_plan(n_total, nsets, n_leaf, flags | tb::kAutoBoxFlag, sc, &p);
  *bytes = p.total;
  return TB_OK;
}

int tb_workspace_bytes(int64_t n, int32_t n_leaf, uint32_t flags, size_t *bytes) {
  return tb_workspace_bytes_batched(n, 1, n_leaf, flags, bytes);
}

int tb_build(const float *pos, const float *mass, int64_t n, int32_t n_leaf, const tb_box *box,
             uint32_t flags, void *workspace, size_t ws_bytes, const tb_tree *out, void *stream) {
  const tb::BatchIn in{nullptr, box, nullptr, box == nullptr};
  return tb::build_impl(pos, mass, n, 1, n_leaf, in, flags, workspace, ws_bytes, out, nullptr,
                        static_cast<hipStream_t>(stream));
}

int tb_build_sync(const float *pos, const float *mass, int64_t n, int32_t n_leaf,
                  const tb_box *box, uint32_t flags, void *workspace, size_t ws_bytes,
                  const tb_tree *out, void *stream) {
  const int rc = tb_build(pos, mass, n, n_leaf, box, flags, workspace, ws_bytes, out, stream);
  if (rc) return rc;
  return tb::wait_status(out, static_cast<hipStream_t>(stream));
}

int tb_build_noalloc(const float *pos, const float *mass, int64_t n, int32_t n_leaf,
                     const tb_box *box, uint32_t flags, const tb_tree *out, void *stream) {
  // sizes first: a build that does not fit the array is refused before any
  // HIP call
  size_t need = 0;
  const int rc = tb_workspace_bytes(n, n_leaf, flags, &need);
  if (rc) return rc;
  if (need > (size_t)TB_NOALLOC_SCRATCH_BYTES) return TB_ERR_SCRATCH;
  void *ws = nullptr;
  if (n > 0) {
    ws = tb::scratch_ptr();
    if (!ws) return TB_ERR_HIP;
  }
  const tb::BatchIn in{nullptr, box, nullptr, box == nullptr};
  return tb::build_impl(pos, mass, n, 1, n_leaf, in, flags, ws, TB_NOALLOC_SCRATCH_BYTES, out,
                        nullptr, static_cast<hipStream_t>(stream), /*traced=*/false);
}

int tb_build_batched(const float *pos, const float *mass, int64_t n_total, int32_t nsets,
                     const int64_t *set_offsets, int32_t n_leaf, const tb_box *boxes,
                     uint32_t flags, void *workspace, size_t ws_bytes, const tb_tree *out,
                     int64_t *cell_offsets, void *stream) {
  if (!set_offsets) return TB_ERR_ARG;
  const tb::BatchIn in{set_offsets, nullptr, boxes, boxes == nullptr};
  return tb::build_impl(pos, mass, n_total, nsets, n_leaf, in, flags, workspace, ws_bytes, out,
                        cell_offsets, static_cast<hipStream_t>(stream));
}

int tb_build_batched_sync(const float *pos, const float *mass, int64_t n_total, int32_t nsets,
                          const int64_t *set_offsets, int32_t n_leaf, const tb_box *boxes,
                          uint32_t flags, void *workspace, size_t ws_bytes, const tb_tree *out,
                          int64_t *cell_offsets, void *stream) {
  const int rc = tb_build_batched(pos, mass, n_total, nsets, set_offsets, n_leaf, boxes, flags,
                                  workspace, ws_bytes, out, cell_offsets, stream);
  if (rc) return rc;
  return tb::wait_status(out, static_cast<hipStream_t>(stream));
}

int tb_gravity_workspace_bytes(int64_t c_max, size_t *bytes) {
  if (!bytes || c_max < 0 || c_max > 2147483647LL) return TB_ERR_ARG;
  *bytes = tb::gravity_workspace_bytes(c_max);
  return TB_OK;
}

int tb_gravity(const float *pos_sorted, const float *mass_sorted, int64_t n, const tb_tree *tree,
               int64_t c_max, double theta, int32_t n_crit, double eps, uint32_t flags,
               double *acc, int64_t *stats, void *workspace, size_t ws_bytes, void *stream) {
  if (n < 0 || n > TB_MAX_N || c_max < 0 || c_max > 2147483647LL || n_crit < 1) return TB_ERR_ARG;
  if (!(theta >= 0.0) || !std::isfinite(theta) || !(eps >= 0.0) || !std::isfinite(eps))
    return TB_ERR_ARG;
  if (flags & ~(TB_GRAV_QUADRUPOLE | TB_HILBERT)) return TB_ERR_ARG;
  if (!tree) return TB_ERR_ARG;
  if (n == 0) return TB_OK;
  if (!pos_sorted || !mass_sorted || !acc || !tree->cell_key || !tree->cell_level ||
      !tree->cell_first || !tree->cell_count || !tree->child_ptr || !tree->com || !tree->quad ||
      !tree->n_cells || !tree->box_out || !tree->status || c_max < 1)
    return TB_ERR_ARG;
  if (!workspace || ws_bytes < tb::gravity_workspace_bytes(c_max)) return TB_ERR_WORKSPACE;
  tb::GravIn in{pos_sorted, mass_sorted, n, tree, c_max, theta, eps, n_crit,
                (flags & TB_GRAV_QUADRUPOLE) != 0, (flags & TB_HILBERT) != 0, acc, stats,
                workspace};
  return tb::launch_gravity(in, static_cast<hipStream_t>(stream)) == hipSuccess ? TB_OK
                                                                               : TB_ERR_HIP;
}

int tb_trace_enable(int on) {
  tb::g_trace = on != 0;
  return TB_OK;
}

int tb_trace_read(tb_trace_entry *out, int cap, int *count) {
  if (!count || (cap > 0 && !out)) return TB_ERR_ARG;
  tb::flush_trace();
  int k = 0;
  for (const auto &kv : tb::g_acc) {
    if (k < cap) {
      std::memset(&out[k], 0, sizeof(out[k]));
      std::snprintf(out[k].name, sizeof(out[k].name), "%s", kv.first.c_str());
      out[k].launches = kv.second.launches;
      out[k].total_ms = kv.second.ms;
    }
    ++k;
  }
  *count = k < cap ? k : cap;
  tb::g_acc.clear();
  return TB_OK;
}

int tb_sort_configs(int32_t *desc, int cap, int *count) {
  if (!count || (cap > 0 && !desc)) return TB_ERR_ARG;
  int k = 0;
  for (; k < tb::kSortTableSize && k < cap; ++k) {
    desc[3 * k + 0] = tb::kSortTable[k].bits;
    desc[3 * k + 1] = tb::kSortTable[k].ipt;
    desc[3 * k + 2] = tb::kSortTable[k].threads;
  }
  *count = cap > 0 ? k : tb::kSortTableSize;
  return TB_OK;
}

const char *tb_version(void) { return "treebuild 0.2 gfx950"; }

}  // extern "C"

extern "C" int tb_kick_drift(const int32_t *perm, const double *acc, int64_t n, double dt_kick,
                             double dt_drift, float *pos, float *vel, int32_t *status,
                             void *stream) {
  if (n < 0 || n > TB_MAX_N || !std::isfinite(dt_kick) || !std::isfinite(dt_drift))
    return TB_ERR_ARG;
  if (n == 0) return TB_OK;
  if (!acc || !pos || !vel) return TB_ERR_ARG;
  return tb::launch_kick_drift(perm, acc, n, dt_kick, dt_drift, pos, vel, status,
                               static_cast<hipStream_t>(stream)) == hipSuccess
             ? TB_OK
             : TB_ERR_HIP;
}

extern "C" int tb_permute(const int32_t *perm, int64_t n, const void *src, int32_t width,
                          void *dst, int32_t *status, void *stream) {
  if (n < 0 || n > TB_MAX_N || width < 1 || width > 64) return TB_ERR_ARG;
  if (n == 0) return TB_OK;
  if (!perm || !src || !dst || src == dst) return TB_ERR_ARG;
  return tb::launch_permute(perm, n, src, width, dst, status, static_cast<hipStream_t>(stream)) ==
                 hipSuccess
             ? TB_OK
             : TB_ERR_HIP;
}
