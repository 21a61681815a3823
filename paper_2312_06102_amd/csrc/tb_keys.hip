// tb_keys.hip -- build set-up, root boxes and Morton keys (Sec. 2.2; Sec. 2.3 step i).
//
// k_init        clears the counters and look-back words one build needs (plain
//               fill kernels, so a captured graph holds no memset node) and
//               copies the set offsets and caller-given root boxes into the
//               workspace.
// k_setup       checks the set offsets and caller-given boxes, then builds the
//               per-set tables: first cell tile, bounding-box chunk and radix
//               tile of each set, and the set of every tile and chunk.
// k_bbox_*      FP64 min/max over each set's positions -> root box with a
//               power-of-two side (only when no box is given).
// k_keygen      FP64 quantisation of each coordinate to 21 bits, bit interleave
//               below a leading 1, plus per-workgroup digit histograms of every
//               radix pass (so the sort never re-reads the keys to count them)
//               and the packed (x, y, z, m) record of every particle.
// k_hist_reduce column sums of those per-workgroup histograms.
// k_keygen_sets the same for a batch, chunk by chunk of one set, with each set's
//               digit counts added up per set;
// k_set_base    each set's digit counts -> the start of every digit's run (a
//               single set's global counts too).
#include "tb_internal.h"

namespace tb {

constexpr int kInitThreads = 256;
constexpr int kKeygenThreads = 512;
constexpr int kKeygenMaxBlocks = 512;
constexpr int kKeygenIpt = 4;
constexpr int kSetupThreads = 1024;

// ---------------------------------------------------------------------------
// init
// ---------------------------------------------------------------------------
__global__ __launch_bounds__(kInitThreads) void k_init(
    uint64_t *__restrict__ status0, int64_t n_status0, uint32_t *__restrict__ counters,
    int32_t *__restrict__ status_word, int64_t n, int32_t nsets,
    const int64_t *__restrict__ set_off_in, int64_t *__restrict__ set_off,
    const tb_box *__restrict__ boxes_in, double *__restrict__ box, int host_box, double lo0,
    double lo1, double lo2, double side, int single, int with_chunks,
    int64_t *__restrict__ tile_start,
    int32_t *__restrict__ tile_set, int64_t *__restrict__ chunk_start,
    int32_t *__restrict__ chunk_set) {
  const int64_t tid = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  const int64_t stride = (int64_t)gridDim.x * blockDim.x;
  for (int64_t i = tid; i < n_status0; i += stride) status0[i] = 0;
  if (single) {
    // one set given by the host: its tables need no validation or scan (the
    // chunk table exists only when the box comes from the data)
    const int64_t nt = (n + kCellTile - 1) / kCellTile;
    const int64_t nc = with_chunks ? (n + kBboxChunk - 1) / kBboxChunk : 0;
    for (int64_t t = tid; t < nt; t += stride) tile_set[t] = 0;
    for (int64_t c = tid; c < nc; c += stride) chunk_set[c] = 0;
    if (tid == 0) {
      tile_start[0] = 0;
      tile_start[1] = nt;
      if (with_chunks) {
        chunk_start[0] = 0;
        chunk_start[1] = nc;
      }
    }
  }
  if (tid < 64) counters[tid] = 0;
  for (int64_t b = tid; b <= nsets; b += stride)
    set_off[b] = set_off_in ? set_off_in[b] : (b == 0 ? 0 : n);
  if (boxes_in) {
    for (int64_t b = tid; b < nsets; b += stride) {
      box[4 * b + 0] = boxes_in[b].lo[0];
      box[4 * b + 1] = boxes_in[b].lo[1];
      box[4 * b + 2] = boxes_in[b].lo[2];
      box[4 * b + 3] = boxes_in[b].side;
    }
  }
  if (tid == 0) {
    *status_word = 0;
    if (host_box) {
      box[0] = lo0;
      box[1] = lo1;
      box[2] = lo2;
      box[3] = side;
    }
  }
}

// A single set described by the host (tb_build): k_init writes its tables and
// k_setup is skipped.
static bool single_set(const Plan &p, const BatchIn &in) {
  return p.nsets == 1 && !in.set_off && !in.dev_boxes;
}

hipError_t launch_init(const Plan &p, const Work &w, const BatchIn &in, const tb_tree &out,
                       hipStream_t s) {
  const int64_t n0 = p.sort_tiles * (int64_t)p.sort.radix();
  int64_t work = n0 > p.nsets ? n0 : p.nsets;
  int blocks = (int)((work + kInitThreads - 1) / kInitThreads);
  if (blocks > 1024) blocks = 1024;
  if (blocks < 1) blocks = 1;
  const tb_box *hb = in.host_box;
  k_init<<<blocks, kInitThreads, 0, s>>>(w.status0, n0, w.counters, out.status, p.n, p.nsets,
                                         in.set_off, w.set_off, in.dev_boxes, w.box, hb ? 1 : 0,
                                         hb ? hb->lo[0] : 0.0, hb ? hb->lo[1] : 0.0,
                                         hb ? hb->lo[2] : 0.0, hb ? hb->side : 1.0,
                                         single_set(p, in) ? 1 : 0, in.auto_box ? 1 : 0,
                                         w.tile_start, w.tile_set,
                                         w.chunk_start, w.chunk_set);
  return hipGetLastError();
}

// ---------------------------------------------------------------------------
// per-set tables (one workgroup)
// ---------------------------------------------------------------------------
// lo finite and side a positive, finite, normal power of two
__device__ __forceinline__ bool box_valid(const double *b) {
  const uint64_t bits = (uint64_t)__double_as_longlong(b[3]);
  const uint32_t ex = (uint32_t)(bits >> 52) & 0x7ffu;
  return isfinite(b[0]) && isfinite(b[1]) && isfinite(b[2]) && (bits >> 63) == 0 &&
         (bits & ((1ull << 52) - 1)) == 0 && ex != 0 && ex != 0x7ffu;
}

__global__ __launch_bounds__(kSetupThreads) void k_setup(
    int64_t *__restrict__ set_off, int32_t nsets, int64_t n, int64_t *__restrict__ tile_start,
    int64_t *__restrict__ chunk_start, int64_t *__restrict__ sort_tile_start, int sort_tile_keys,
    int with_chunks, double *__restrict__ box, int check_boxes, int max_set_bits,
    uint32_t *__restrict__ oversize, int32_t *__restrict__ status_word) {
  __shared__ uint32_t s_w[3][kSetupThreads / 64];
  __shared__ uint64_t s_carry[3];
  __shared__ int s_bad;
  // The offsets must start at 0, end at n and never decrease.  Anything else is
  // reported and replaced by {0, ..., 0, n}, so no kernel indexes outside [0, n).
  if (threadIdx.x == 0) s_bad = (set_off[0] != 0 || set_off[nsets] != n) ? 1 : 0;
  __syncthreads();
  for (int b = threadIdx.x; b < nsets; b += kSetupThreads)
    if (set_off[b] > set_off[b + 1] || set_off[b] < 0) s_bad = 1;
  __syncthreads();
  if (s_bad) {
    for (int b = threadIdx.x; b <= nsets; b += kSetupThreads) set_off[b] = b == nsets ? n : 0;
    if (threadIdx.x == 0) atomicOr(status_word, TB_STATUS_SETS);
  }
  if (max_set_bits > 0) {
    // A set larger than the caller's bound (checked on the offsets as they now
    // stand): its indices do not fit in the sort's index bits, so its order and
    // the keys the cell stages would read from it are not consistent.  It is
    // reported, and the flag makes the reorder give every particle the same key,
    // which turns each set into coincident points: a tree every kernel handles
    // and C_max bounds.
    __syncthreads();
    bool big = false;
    for (int b = threadIdx.x; b < nsets; b += kSetupThreads)
      big |= set_off[b + 1] - set_off[b] > (int64_t{1} << max_set_bits);
    if (big) {
      atomicOr(status_word, TB_STATUS_SETS);
      *oversize = 1u;
    }
  }
  // a caller-given box that is not usable is reported and replaced by the unit
  // cube, so that the key arithmetic stays finite
  if (check_boxes) {
    bool bad_box = false;
    for (int b = threadIdx.x; b < nsets; b += kSetupThreads) {
      if (!box_valid(box + 4 * b)) {
        bad_box = true;
        box[4 * b + 0] = box[4 * b + 1] = box[4 * b + 2] = 0.0;
        box[4 * b + 3] = 1.0;
      }
    }
    if (bad_box) atomicOr(status_word, TB_STATUS_BOX);
  }
  // exclusive scans over sets of the tile and chunk counts, in rounds
  if (threadIdx.x == 0) s_carry[0] = s_carry[1] = s_carry[2] = 0;
  __syncthreads();
  const int wv = threadIdx.x / 64;
  for (int r0 = 0; r0 < nsets; r0 += kSetupThreads) {
    const int b = r0 + threadIdx.x;
    int64_t nb = 0;
    if (b < nsets) nb = set_off[b + 1] - set_off[b];
    const uint32_t nt = (uint32_t)((nb + kCellTile - 1) / kCellTile);
    const uint32_t nc = with_chunks ? (uint32_t)((nb + kBboxChunk - 1) / kBboxChunk) : 0u;
    const uint32_t ns = sort_tile_start ? (uint32_t)((nb + sort_tile_keys - 1) / sort_tile_keys)
                                        : 0u;
    const uint32_t it = wave_inclusive_scan(nt), ic = wave_inclusive_scan(nc),
                   is = wave_inclusive_scan(ns);
    if (lane_id() == 63) {
      s_w[0][wv] = it;
      s_w[1][wv] = ic;
      s_w[2][wv] = is;
    }
    __syncthreads();
    uint64_t ot = s_carry[0], oc = s_carry[1], os = s_carry[2], tt = 0, tc = 0, ts = 0;
    for (int q = 0; q < kSetupThreads / 64; ++q) {
      if (q < wv) {
        ot += s_w[0][q];
        oc += s_w[1][q];
        os += s_w[2][q];
      }
      tt += s_w[0][q];
      tc += s_w[1][q];
      ts += s_w[2][q];
    }
    ot += it - nt;
    oc += ic - nc;
    os += is - ns;
    if (b < nsets) {
      tile_start[b] = (int64_t)ot;
      if (with_chunks) chunk_start[b] = (int64_t)oc;
      if (sort_tile_start) sort_tile_start[b] = (int64_t)os;
    }
    __syncthreads();
    if (threadIdx.x == 0) {
      s_carry[0] += tt;
      s_carry[1] += tc;
      s_carry[2] += ts;
    }
    __syncthreads();
  }
  if (threadIdx.x == 0) {
    tile_start[nsets] = (int64_t)s_carry[0];
    if (with_chunks) chunk_start[nsets] = (int64_t)s_carry[1];
    if (sort_tile_start) sort_tile_start[nsets] = (int64_t)s_carry[2];
  }
}

// The set of every cell tile, bounding-box chunk and radix tile: one thread per
// entry, binary search over the first-tile / first-chunk tables; the threads
// past them clear a batch's per-set digit counts.
__global__ __launch_bounds__(256) void k_tile_map(
    const int64_t *__restrict__ tile_start, int32_t *__restrict__ tile_set, int64_t cell_tiles,
    const int64_t *__restrict__ chunk_start, int32_t *__restrict__ chunk_set, int64_t bbox_chunks,
    int with_chunks, const int64_t *__restrict__ sort_tile_start,
    int32_t *__restrict__ sort_tile_set, int64_t sort_tiles, uint32_t *__restrict__ set_counts,
    int64_t n_counts, int32_t nsets) {
  const int64_t stride = (int64_t)gridDim.x * blockDim.x;
  const int64_t nc = with_chunks ? bbox_chunks : 0, ns = sort_tile_set ? sort_tiles : 0;
  const int64_t total = cell_tiles + nc + ns + n_counts;
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < total; i += stride) {
    if (i < cell_tiles) {
      if (i < tile_start[nsets]) tile_set[i] = upper_index(tile_start, nsets + 1, i);
    } else if (i < cell_tiles + nc) {
      const int64_t c = i - cell_tiles;
      if (c < chunk_start[nsets]) chunk_set[c] = upper_index(chunk_start, nsets + 1, c);
    } else if (i < cell_tiles + nc + ns) {
      const int64_t t = i - cell_tiles - nc;
      if (t < sort_tile_start[nsets]) sort_tile_set[t] = upper_index(sort_tile_start, nsets + 1, t);
    } else {
      set_counts[i - cell_tiles - nc - ns] = 0u;
    }
  }
}

hipError_t launch_setup(const Plan &p, const Work &w, const BatchIn &in, int32_t *status,
                        hipStream_t s) {
  if (single_set(p, in)) return hipSuccess;  // written by k_init
  const bool with_chunks = in.auto_box;
  k_setup<<<1, kSetupThreads, 0, s>>>(w.set_off, p.nsets, p.n, w.tile_start, w.chunk_start,
                                      p.seg ? w.seg_tile_start : nullptr, p.sort.tile(),
                                      with_chunks ? 1 : 0, w.box, in.dev_boxes ? 1 : 0,
                                      p.set_index_bits, w.counters + kOversizeCounter, status);
  const int64_t n_counts = p.seg ? (int64_t)p.nsets * p.key_passes * p.sort.radix() : 0;
  const int64_t entries = p.cell_tiles + (with_chunks ? p.bbox_chunks : 0) +
                          (p.seg ? p.sort_tiles : 0) + n_counts;
  int64_t grid = (entries + 255) / 256;
  if (grid > 4096) grid = 4096;
  k_tile_map<<<(unsigned)grid, 256, 0, s>>>(
      w.tile_start, w.tile_set, p.cell_tiles, w.chunk_start, w.chunk_set, p.bbox_chunks,
      with_chunks ? 1 : 0, p.seg ? w.seg_tile_start : nullptr, p.seg ? w.seg_tile_set : nullptr,
      p.sort_tiles, w.seg_base, n_counts, p.nsets);
  return hipGetLastError();
}

// ---------------------------------------------------------------------------
// root boxes (FP64 min / max per set, then the power-of-two side)
// ---------------------------------------------------------------------------
constexpr int kBboxThreads = 256;

__global__ __launch_bounds__(kBboxThreads) void k_bbox_partial(
    const float *__restrict__ pos, const int64_t *__restrict__ set_off,
    const int64_t *__restrict__ chunk_start, const int32_t *__restrict__ chunk_set,
    int32_t nsets, double *__restrict__ part) {
  __shared__ double red[6][kBboxThreads / 64];
  const int64_t c = blockIdx.x;
  if (c >= chunk_start[nsets]) return;
  const int b = chunk_set[c];
  const int64_t i0 = set_off[b] + (c - chunk_start[b]) * (int64_t)kBboxChunk;
  const int64_t i1 = min(i0 + (int64_t)kBboxChunk, set_off[b + 1]);
  double mn[3] = {INFINITY, INFINITY, INFINITY};
  double mx[3] = {-INFINITY, -INFINITY, -INFINITY};
  for (int64_t i = i0 + threadIdx.x; i < i1; i += kBboxThreads) {
#pragma unroll
    for (int a = 0; a < 3; ++a) {
      double v = (double)pos[3 * i + a];
      mn[a] = fmin(mn[a], v);
      mx[a] = fmax(mx[a], v);
    }
  }
#pragma unroll
  for (int a = 0; a < 3; ++a) {
    for (int o = 32; o > 0; o >>= 1) {
      mn[a] = fmin(mn[a], __shfl_xor(mn[a], o, 64));
      mx[a] = fmax(mx[a], __shfl_xor(mx[a], o, 64));
    }
  }
  const int wv = threadIdx.x / 64;
  if (lane_id() == 0) {
#pragma unroll
    for (int a = 0; a < 3; ++a) {
      red[a][wv] = mn[a];
      red[3 + a][wv] = mx[a];
    }
  }
  __syncthreads();
  if (threadIdx.x < 6) {
    const int k = threadIdx.x;
    double r = red[k][0];
    for (int q = 1; q < kBboxThreads / 64; ++q) r = (k < 3) ? fmin(r, red[k][q]) : fmax(r, red[k][q]);
    part[c * 6 + k] = r;
  }
}

__global__ __launch_bounds__(64) void k_bbox_final(const double *__restrict__ part,
                                                   const int64_t *__restrict__ chunk_start,
                                                   int32_t nsets, double *__restrict__ box) {
  for (int b = blockIdx.x; b < nsets; b += gridDim.x) {
    double mn[3] = {INFINITY, INFINITY, INFINITY};
    double mx[3] = {-INFINITY, -INFINITY, -INFINITY};
    for (int64_t c = chunk_start[b] + threadIdx.x; c < chunk_start[b + 1]; c += 64) {
#pragma unroll
      for (int a = 0; a < 3; ++a) {
        mn[a] = fmin(mn[a], part[c * 6 + a]);
        mx[a] = fmax(mx[a], part[c * 6 + 3 + a]);
      }
    }
#pragma unroll
    for (int a = 0; a < 3; ++a) {
      for (int o = 32; o > 0; o >>= 1) {
        mn[a] = fmin(mn[a], __shfl_xor(mn[a], o, 64));
        mx[a] = fmax(mx[a], __shfl_xor(mx[a], o, 64));
      }
    }
    if (threadIdx.x == 0) {
      double ext = 0.0;
#pragma unroll
      for (int a = 0; a < 3; ++a) {
        const double e = mx[a] - mn[a];
        ext = e > ext ? e : ext;
      }
      // smallest power of two strictly above ext: ext = f * 2^e with f in [0.5, 1)
      double side = 1.0;
      if (ext > 0.0 && isfinite(ext)) {
        int e;
        (void)frexp(ext, &e);
        side = ldexp(1.0, e);
      }
      box[4 * b + 0] = isfinite(mn[0]) ? mn[0] : 0.0;
      box[4 * b + 1] = isfinite(mn[1]) ? mn[1] : 0.0;
      box[4 * b + 2] = isfinite(mn[2]) ? mn[2] : 0.0;
      box[4 * b + 3] = side;
    }
  }
}

hipError_t launch_bbox(const Plan &p, const Work &w, const float *pos, hipStream_t s) {
  k_bbox_partial<<<(unsigned)p.bbox_chunks, kBboxThreads, 0, s>>>(
      pos, w.set_off, w.chunk_start, w.chunk_set, p.nsets, w.bbox_part);
  const int blocks = p.nsets < 4096 ? p.nsets : 4096;
  k_bbox_final<<<blocks, 64, 0, s>>>(w.bbox_part, w.chunk_start, p.nsets, w.box);
  return hipGetLastError();
}

// ---------------------------------------------------------------------------
// Morton keys
// ---------------------------------------------------------------------------

// One particle's key and record, and its digit of every radix pass counted in
// the LDS histograms h; a wave whose lanes all share a digit adds once (the upper
// digits of clustered data are mostly uniform).
template <int BITS>
__device__ __forceinline__ void key_one(float x, float y, float z, float m, bool valid,
                                        int64_t i, double lo0, double lo1, double lo2,
                                        double scale, bool hilbert, uint64_t *__restrict__ keys,
                                        float4 *__restrict__ packed, void *__restrict__ dig0,
                                        uint32_t *h, bool &bad) {
  constexpr int R = 1 << BITS;
  constexpr int MAXP = (63 + BITS - 1) / BITS;
  bad |= valid && !(isfinite(x) && isfinite(y) && isfinite(z));
  const uint64_t key = particle_key(x, y, z, lo0, lo1, lo2, scale, hilbert);
  if (valid) {
    keys[i] = key;
    // (x, y, z, m) in one 16-byte record: the reorder step gathers one line each
    packed[i] = make_float4(x, y, z, m);
    // the first radix pass's digit, for its tile counts (counted passes)
    if (dig0) static_cast<DigitType<BITS> *>(dig0)[i] = (DigitType<BITS>)(key & (R - 1));
  }
  const uint64_t active = __ballot(valid);
  if (valid) {
#pragma unroll
    for (int p = 0; p < MAXP; ++p) {
      const uint32_t d = (uint32_t)(key >> (p * BITS)) & (R - 1);
      const uint32_t d0 = __builtin_amdgcn_readfirstlane(d);
      if (__ballot(d == d0) == active) {
        if (lane_id() == __ffsll((long long)active) - 1)
          atomicAdd(&h[p * R + d0], (uint32_t)__popcll(active));
      } else {
        atomicAdd(&h[p * R + d], 1u);
      }
    }
  }
}

// A single set: a grid-stride loop, one histogram per workgroup.
template <int BITS>
__global__ __launch_bounds__(kKeygenThreads) void k_keygen(
    const float *__restrict__ pos, const float *__restrict__ mass, int64_t n,
    const double *__restrict__ box, uint64_t *__restrict__ keys, float4 *__restrict__ packed,
    void *__restrict__ dig0, uint32_t *__restrict__ hist_part, int passes, int hilbert,
    int32_t *__restrict__ status_word) {
  constexpr int R = 1 << BITS;
  constexpr int MAXP = (63 + BITS - 1) / BITS;
  __shared__ uint32_t h[MAXP * R];
  for (int i = threadIdx.x; i < passes * R; i += blockDim.x) h[i] = 0;
  __syncthreads();
  bool bad = false;
  const double lo0 = box[0], lo1 = box[1], lo2 = box[2];
  const double scale = 2097152.0 / box[3];
  // each step a thread handles kKeygenIpt particles whose loads are all issued
  // before any is used (indices past the end are clamped and masked)
  const int64_t step = (int64_t)gridDim.x * blockDim.x * kKeygenIpt;
  for (int64_t i0 = (int64_t)blockIdx.x * blockDim.x * kKeygenIpt + threadIdx.x; i0 < n;
       i0 += step) {
    float x[kKeygenIpt], y[kKeygenIpt], z[kKeygenIpt], m[kKeygenIpt];
#pragma unroll
    for (int r = 0; r < kKeygenIpt; ++r) {
      const int64_t i = min(i0 + (int64_t)r * blockDim.x, n - 1);
      x[r] = pos[3 * i + 0];
      y[r] = pos[3 * i + 1];
      z[r] = pos[3 * i + 2];
      m[r] = mass[i];
    }
#pragma unroll
    for (int r = 0; r < kKeygenIpt; ++r) {
      const int64_t i = i0 + (int64_t)r * blockDim.x;
      key_one<BITS>(x[r], y[r], z[r], m[r], i < n, i, lo0, lo1, lo2, scale, hilbert != 0, keys,
                    packed, dig0, h, bad);
    }
  }
  if (__ballot(bad) != 0 && lane_id() == 0) atomicOr(status_word, TB_STATUS_NONFINITE);
  __syncthreads();
  uint32_t *dst = hist_part + (int64_t)blockIdx.x * passes * R;
  for (int i = threadIdx.x; i < passes * R; i += blockDim.x) dst[i] = h[i];
}

// A batch: workgroup g takes the particles [g N / G, (g + 1) N / G) of the whole
// batch, which may span several sets (or part of one).  Its histogram is added
// to the set's counts, set_counts[b][p][d], each time its range leaves a set, so
// every workgroup has the same number of particles whatever the set sizes.
template <int BITS>
__global__ __launch_bounds__(kKeygenThreads) void k_keygen_sets(
    const float *__restrict__ pos, const float *__restrict__ mass, int64_t n,
    const int64_t *__restrict__ set_off, int32_t nsets, const double *__restrict__ box,
    uint64_t *__restrict__ keys, float4 *__restrict__ packed, void *__restrict__ dig0,
    uint32_t *__restrict__ set_counts, int passes, int hilbert, int32_t *__restrict__ status_word) {
  constexpr int R = 1 << BITS;
  constexpr int MAXP = (63 + BITS - 1) / BITS;
  constexpr int64_t kStep = (int64_t)kKeygenThreads * kKeygenIpt;
  __shared__ uint32_t h[MAXP * R];
  __shared__ int s_b;
  const int64_t per = (n + gridDim.x - 1) / gridDim.x;
  const int64_t g_lo = (int64_t)blockIdx.x * per;
  const int64_t g_hi = min(n, g_lo + per);
  if (g_lo >= g_hi) return;  // the same for the whole workgroup
  // the set holding g_lo: the last b with set_off[b] <= g_lo (the offsets start
  // at 0, end at n and never decrease)
  if (threadIdx.x == 0) {
    int lo = 0, hi = nsets;
    while (hi - lo > 1) {
      const int mid = (lo + hi) >> 1;
      if (set_off[mid] <= g_lo) lo = mid; else hi = mid;
    }
    s_b = lo;
  }
  for (int i = threadIdx.x; i < passes * R; i += blockDim.x) h[i] = 0;
  __syncthreads();
  int b = s_b;
  bool bad = false;
  for (int64_t s0 = g_lo; s0 < g_hi;) {
    while (b + 1 < nsets && set_off[b + 1] <= s0) ++b;  // past empty sets
    const int64_t s1 = min(g_hi, max(s0 + 1, set_off[b + 1]));
    const double lo0 = box[4 * b + 0], lo1 = box[4 * b + 1], lo2 = box[4 * b + 2];
    const double scale = 2097152.0 / box[4 * b + 3];
    for (int64_t base = s0; base < s1; base += kStep) {
      float x[kKeygenIpt], y[kKeygenIpt], z[kKeygenIpt], m[kKeygenIpt];
#pragma unroll
      for (int r = 0; r < kKeygenIpt; ++r) {
        const int64_t i = min(base + r * kKeygenThreads + threadIdx.x, s1 - 1);
        x[r] = pos[3 * i + 0];
        y[r] = pos[3 * i + 1];
        z[r] = pos[3 * i + 2];
        m[r] = mass[i];
      }
#pragma unroll
      for (int r = 0; r < kKeygenIpt; ++r) {
        const int64_t i = base + r * kKeygenThreads + threadIdx.x;
        key_one<BITS>(x[r], y[r], z[r], m[r], i < s1, i, lo0, lo1, lo2, scale, hilbert != 0,
                      keys, packed, dig0, h, bad);
      }
    }
    __syncthreads();
    uint32_t *dst = set_counts + (int64_t)b * passes * R;
    for (int i = threadIdx.x; i < passes * R; i += blockDim.x) {
      const uint32_t c = h[i];
      if (c) {
        atomicAdd(&dst[i], c);
        h[i] = 0;  // cleared for the next set
      }
    }
    __syncthreads();
    s0 = s1;
  }
  if (__ballot(bad) != 0 && lane_id() == 0) atomicOr(status_word, TB_STATUS_NONFINITE);
}

// Each set's digit counts of every pass -> the position where each digit's run
// of the set starts (the set's first position plus the counts of the smaller
// digits).  One workgroup per (set, pass) (blockIdx.y: the pass), one thread
// per digit.
template <int BITS>
__global__ __launch_bounds__(1 << BITS) void k_set_base(const int64_t *__restrict__ set_off,
                                                        uint32_t *__restrict__ set_counts,
                                                        int passes, int32_t nsets) {
  constexpr int R = 1 << BITS;
  __shared__ uint32_t s_w[R / 64];
  const int p = blockIdx.y;
  for (int b = blockIdx.x; b < nsets; b += gridDim.x) {
    uint32_t *row = set_counts + ((int64_t)b * passes + p) * R;
    const uint32_t v = row[threadIdx.x];
    const uint32_t inc = wave_inclusive_scan(v);
    if (lane_id() == 63) s_w[threadIdx.x / 64] = inc;
    __syncthreads();
    uint32_t off = 0;
    for (int q = 0; q < (int)threadIdx.x / 64; ++q) off += s_w[q];
    row[threadIdx.x] = (uint32_t)set_off[b] + off + inc - v;
    __syncthreads();
  }
}

// hist[c] = sum over rows b of part[b][c], for c < cols.  16 columns per
// workgroup, 16 row groups per column, so each thread sums only rows/16 values.
__global__ __launch_bounds__(256) void k_hist_reduce(const uint32_t *__restrict__ part, int rows,
                                                     int cols, uint32_t *__restrict__ hist) {
  __shared__ uint32_t red[16][17];
  const int col = threadIdx.x & 15;
  const int g = threadIdx.x >> 4;
  const int c = blockIdx.x * 16 + col;
  uint32_t s = 0;
  if (c < cols) {
#pragma unroll 8
    for (int b = g; b < rows; b += 16) s += part[(int64_t)b * cols + c];
  }
  red[g][col] = s;
  __syncthreads();
  if (threadIdx.x < 16 && c < cols) {
    uint32_t t = 0;
#pragma unroll
    for (int k = 0; k < 16; ++k) t += red[k][col];
    hist[c] = t;
  }
}

int keygen_blocks(int64_t n) {
  // at least four keys per thread; enough workgroups to fill every CU
  int64_t b = (n + 4 * kKeygenThreads - 1) / (4 * kKeygenThreads);
  if (b > kKeygenMaxBlocks) b = kKeygenMaxBlocks;
  if (b < 1) b = 1;
  return (int)b;
}

hipError_t launch_keygen(const Plan &p, const Work &w, const float *pos, const float *mass,
                         const tb_tree &out, hipStream_t s) {
  const int passes = p.key_passes;
  const int hil = (p.flags & TB_HILBERT) ? 1 : 0;
  if (!p.seg) {
    const int blocks = keygen_blocks(p.n);
#define TB_KEYGEN(B)                                                                           \
  k_keygen<B><<<blocks, kKeygenThreads, 0, s>>>(pos, mass, p.n, w.box, w.keys0, w.packed,      \
                                                (p.counted & 1u) ? w.dig : nullptr, w.hist_part, passes, \
                                                hil, out.status)
    switch (p.sort.bits) {
      case 8: TB_KEYGEN(8); break;
      case 9: TB_KEYGEN(9); break;
      default: return hipErrorInvalidValue;
    }
#undef TB_KEYGEN
  } else {
    // as many particles per workgroup as the single-set kernel at its largest grid
    const int blocks = 2 * keygen_blocks(p.n);
#define TB_KEYGEN_SETS(B)                                                                      \
  k_keygen_sets<B><<<(unsigned)blocks, kKeygenThreads, 0, s>>>(                                \
      pos, mass, p.n, w.set_off, p.nsets, w.box, w.keys0, w.packed,                            \
      (p.counted & 1u) ? w.dig : nullptr, w.seg_base, passes, hil, out.status)
    switch (p.sort.bits) {
      case 8: TB_KEYGEN_SETS(8); break;
      case 9: TB_KEYGEN_SETS(9); break;
      default: return hipErrorInvalidValue;
    }
#undef TB_KEYGEN_SETS
  }
  return hipGetLastError();
}

hipError_t launch_hist_reduce(const Plan &p, const Work &w, hipStream_t s) {
  // each set's digit counts become its digit bases (a single set: once, rather
  // than in every tile of a pass)
  uint32_t *counts = w.seg_base;
  if (!p.seg) {
    const int cols = p.key_passes * p.sort.radix();
    k_hist_reduce<<<(cols + 15) / 16, 256, 0, s>>>(w.hist_part, keygen_blocks(p.n), cols, w.hist);
    counts = w.hist;
  }
  const dim3 grid((unsigned)(p.nsets < 65535 ? p.nsets : 65535), (unsigned)p.key_passes);
  if (p.sort.bits == 8)
    k_set_base<8><<<grid, 256, 0, s>>>(w.set_off, counts, p.key_passes, p.nsets);
  else if (p.sort.bits == 9)
    k_set_base<9><<<grid, 512, 0, s>>>(w.set_off, counts, p.key_passes, p.nsets);
  else
    return hipErrorInvalidValue;
  return hipGetLastError();
}

// ---------------------------------------------------------------------------
// N == 0: only the scalar outputs are written
// ---------------------------------------------------------------------------
__global__ void k_empty(int64_t *level_offset, int32_t nsets, int64_t *n_cells,
                        int64_t *cell_offsets, int32_t *status_word, double *box_out,
                        const tb_box *boxes_in, int host_box, double lo0, double lo1, double lo2,
                        double side) {
  for (int64_t i = threadIdx.x; i < (int64_t)nsets * (kLevels + 1); i += blockDim.x)
    level_offset[i] = 0;
  if (cell_offsets)
    for (int64_t i = threadIdx.x; i <= nsets; i += blockDim.x) cell_offsets[i] = 0;
  if (box_out) {
    for (int64_t b = threadIdx.x; b < nsets; b += blockDim.x) {
      box_out[4 * b + 0] = boxes_in ? boxes_in[b].lo[0] : (host_box ? lo0 : 0.0);
      box_out[4 * b + 1] = boxes_in ? boxes_in[b].lo[1] : (host_box ? lo1 : 0.0);
      box_out[4 * b + 2] = boxes_in ? boxes_in[b].lo[2] : (host_box ? lo2 : 0.0);
      box_out[4 * b + 3] = boxes_in ? boxes_in[b].side : (host_box ? side : 1.0);
    }
  }
  if (threadIdx.x == 0) {
    *n_cells = 0;
    *status_word = 0;
  }
}

hipError_t launch_empty(const tb_tree &out, int32_t nsets, const BatchIn &in,
                        int64_t *cell_offsets, hipStream_t s) {
  const tb_box *hb = in.host_box;
  k_empty<<<1, 256, 0, s>>>(out.level_offset, nsets, out.n_cells, cell_offsets, out.status,
                            out.box_out, in.dev_boxes, hb ? 1 : 0, hb ? hb->lo[0] : 0.0,
                            hb ? hb->lo[1] : 0.0, hb ? hb->lo[2] : 0.0, hb ? hb->side : 1.0);
  return hipGetLastError();
}

}  // namespace tb
