// tb_keys.hip -- build set-up, root box and Morton keys (Sec. 2.2; Sec. 2.3 step i).
//
// k_init        clears the counters and lookback words one build needs (a plain
//               fill kernel, so a captured graph holds no memset node) and
//               stores a caller-given root box on the device.
// k_bbox_*      FP64 min/max over the positions -> root box with a power-of-two
//               side (only when the caller gives no box).
// k_keygen      FP64 quantisation of each coordinate to 21 bits, bit interleave
//               below a leading 1, plus per-workgroup digit histograms of every
//               radix pass (so the sort never re-reads the keys to count them).
// k_hist_reduce column sums of those per-workgroup histograms.
#include "tb_internal.h"

namespace tb {

constexpr int kInitThreads = 256;
constexpr int kKeygenThreads = 512;
constexpr int kKeygenMaxBlocks = 512;
constexpr int kKeygenIpt = 4;

// ---------------------------------------------------------------------------
// init
// ---------------------------------------------------------------------------
__global__ __launch_bounds__(kInitThreads) void k_init(
    uint64_t *__restrict__ status0, int64_t n_status0, uint32_t *__restrict__ counters,
    int32_t *__restrict__ status_word,
    double *__restrict__ box, int box_given, double lo0, double lo1, double lo2, double side) {
  const int64_t tid = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  const int64_t stride = (int64_t)gridDim.x * blockDim.x;
  for (int64_t i = tid; i < n_status0; i += stride) status0[i] = 0;
  if (tid < 64) counters[tid] = 0;
  if (tid == 0) {
    *status_word = 0;
    if (box_given) {
      box[0] = lo0;
      box[1] = lo1;
      box[2] = lo2;
      box[3] = side;
    }
  }
}

hipError_t launch_init(const Plan &p, const Work &w, const tb_box *box, const tb_tree &out,
                       hipStream_t s) {
  const int64_t n0 = p.sort_tiles * (int64_t)p.sort.radix();
  int blocks = (int)((n0 + kInitThreads - 1) / kInitThreads);
  if (blocks > 1024) blocks = 1024;
  if (blocks < 1) blocks = 1;
  k_init<<<blocks, kInitThreads, 0, s>>>(w.status0, n0, w.counters, out.status, w.box, box ? 1 : 0, box ? box->lo[0] : 0.0,
                                         box ? box->lo[1] : 0.0, box ? box->lo[2] : 0.0,
                                         box ? box->side : 1.0);
  return hipGetLastError();
}

// ---------------------------------------------------------------------------
// root box (FP64 min / max, then the power-of-two side)
// ---------------------------------------------------------------------------
__global__ __launch_bounds__(kBboxThreads) void k_bbox_partial(const float *__restrict__ pos,
                                                               int64_t n,
                                                               double *__restrict__ part) {
  __shared__ double red[6][kBboxThreads / 64];
  double mn[3] = {INFINITY, INFINITY, INFINITY};
  double mx[3] = {-INFINITY, -INFINITY, -INFINITY};
  const int64_t stride = (int64_t)gridDim.x * blockDim.x;
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n; i += stride) {
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
    const int c = threadIdx.x;
    double r = red[c][0];
    for (int k = 1; k < kBboxThreads / 64; ++k) r = (c < 3) ? fmin(r, red[c][k]) : fmax(r, red[c][k]);
    part[blockIdx.x * 6 + c] = r;
  }
}

__global__ __launch_bounds__(64) void k_bbox_final(const double *__restrict__ part, int nblocks,
                                                   double *__restrict__ box) {
  double mn[3] = {INFINITY, INFINITY, INFINITY};
  double mx[3] = {-INFINITY, -INFINITY, -INFINITY};
  for (int b = threadIdx.x; b < nblocks; b += 64) {
#pragma unroll
    for (int a = 0; a < 3; ++a) {
      mn[a] = fmin(mn[a], part[b * 6 + a]);
      mx[a] = fmax(mx[a], part[b * 6 + 3 + a]);
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
    box[0] = isfinite(mn[0]) ? mn[0] : 0.0;
    box[1] = isfinite(mn[1]) ? mn[1] : 0.0;
    box[2] = isfinite(mn[2]) ? mn[2] : 0.0;
    box[3] = side;
  }
}

hipError_t launch_bbox(const Plan &p, const Work &w, const float *pos, hipStream_t s) {
  int blocks = (int)((p.n + kBboxThreads - 1) / kBboxThreads);
  if (blocks > kBboxBlocks) blocks = kBboxBlocks;
  if (blocks < 1) blocks = 1;
  k_bbox_partial<<<blocks, kBboxThreads, 0, s>>>(pos, p.n, w.bbox_part);
  k_bbox_final<<<1, 64, 0, s>>>(w.bbox_part, blocks, w.box);
  return hipGetLastError();
}

// ---------------------------------------------------------------------------
// Morton keys
// ---------------------------------------------------------------------------

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
// power of two, so the multiply is exact and only the subtraction rounds.
__device__ __forceinline__ uint32_t quantise(float x, double lo, double scale) {
  const double u = __dsub_rn((double)x, lo);
  const double t = __dmul_rn(u, scale);
  if (!(t >= 0.0)) return 0u;
  if (t >= 2097152.0) return 2097151u;
  return (uint32_t)t;  // truncation == floor for t >= 0
}

template <int BITS>
__global__ __launch_bounds__(kKeygenThreads) void k_keygen(
    const float *__restrict__ pos, int64_t n, const double *__restrict__ box,
    uint64_t *__restrict__ keys, uint32_t *__restrict__ hist_part, int passes,
    int32_t *__restrict__ status_word) {
  constexpr int R = 1 << BITS;
  constexpr int MAXP = (63 + BITS - 1) / BITS;
  __shared__ uint32_t h[MAXP * R];
  for (int i = threadIdx.x; i < passes * R; i += blockDim.x) h[i] = 0;
  __syncthreads();

  const double lo0 = box[0], lo1 = box[1], lo2 = box[2];
  const double scale = 2097152.0 / box[3];
  bool bad = false;
  // each step a thread handles kKeygenIpt particles whose loads are all issued
  // before any is used (indices past the end are clamped and masked)
  const int64_t step = (int64_t)gridDim.x * blockDim.x * kKeygenIpt;
  for (int64_t i0 = (int64_t)blockIdx.x * blockDim.x * kKeygenIpt + threadIdx.x; i0 < n;
       i0 += step) {
    float x[kKeygenIpt], y[kKeygenIpt], z[kKeygenIpt];
#pragma unroll
    for (int r = 0; r < kKeygenIpt; ++r) {
      const int64_t i = min(i0 + (int64_t)r * blockDim.x, n - 1);
      x[r] = pos[3 * i + 0];
      y[r] = pos[3 * i + 1];
      z[r] = pos[3 * i + 2];
    }
#pragma unroll
    for (int r = 0; r < kKeygenIpt; ++r) {
      const int64_t i = i0 + (int64_t)r * blockDim.x;
      const bool valid = i < n;
      bad |= valid && !(isfinite(x[r]) && isfinite(y[r]) && isfinite(z[r]));
      const uint64_t qx = quantise(x[r], lo0, scale);
      const uint64_t qy = quantise(y[r], lo1, scale);
      const uint64_t qz = quantise(z[r], lo2, scale);
      const uint64_t key = (1ull << 63) | (spread3(qx) << 2) | (spread3(qy) << 1) | spread3(qz);
      if (valid) keys[i] = key;
      // digit histograms of every radix pass; a wave whose lanes all share the
      // digit adds once (the upper digits of clustered data are mostly uniform)
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
  }
  if (__ballot(bad) != 0 && lane_id() == 0) atomicOr(status_word, TB_STATUS_NONFINITE);
  __syncthreads();
  uint32_t *dst = hist_part + (int64_t)blockIdx.x * passes * R;
  for (int i = threadIdx.x; i < passes * R; i += blockDim.x) dst[i] = h[i];
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

hipError_t launch_keygen(const Plan &p, const Work &w, const float *pos, const tb_tree &out,
                         hipStream_t s) {
  const int blocks = keygen_blocks(p.n);
  const int passes = p.sort.passes();
  switch (p.sort.bits) {
    case 8: k_keygen<8><<<blocks, kKeygenThreads, 0, s>>>(pos, p.n, w.box, w.keys0, w.hist_part, passes, out.status); break;
    case 9: k_keygen<9><<<blocks, kKeygenThreads, 0, s>>>(pos, p.n, w.box, w.keys0, w.hist_part, passes, out.status); break;
    case 10: k_keygen<10><<<blocks, kKeygenThreads, 0, s>>>(pos, p.n, w.box, w.keys0, w.hist_part, passes, out.status); break;
    case 11: k_keygen<11><<<blocks, kKeygenThreads, 0, s>>>(pos, p.n, w.box, w.keys0, w.hist_part, passes, out.status); break;
    default: return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

hipError_t launch_hist_reduce(const Plan &p, const Work &w, hipStream_t s) {
  const int cols = p.sort.passes() * p.sort.radix();
  k_hist_reduce<<<(cols + 15) / 16, 256, 0, s>>>(w.hist_part, keygen_blocks(p.n), cols, w.hist);
  return hipGetLastError();
}

// ---------------------------------------------------------------------------
// N == 0: only the scalar outputs are written
// ---------------------------------------------------------------------------
__global__ void k_empty(int64_t *level_offset, int64_t *n_cells, int32_t *status_word,
                        double *box_out, int box_given, double lo0, double lo1, double lo2,
                        double side) {
  const int t = threadIdx.x;
  if (t < kLevels + 1) level_offset[t] = 0;
  if (t == 0) {
    *n_cells = 0;
    *status_word = 0;
    if (box_out) {
      box_out[0] = box_given ? lo0 : 0.0;
      box_out[1] = box_given ? lo1 : 0.0;
      box_out[2] = box_given ? lo2 : 0.0;
      box_out[3] = box_given ? side : 1.0;
    }
  }
}

hipError_t launch_empty(const tb_tree &out, const tb_box *box, hipStream_t s) {
  k_empty<<<1, 64, 0, s>>>(out.level_offset, out.n_cells, out.status, out.box_out, box ? 1 : 0,
                           box ? box->lo[0] : 0.0, box ? box->lo[1] : 0.0,
                           box ? box->lo[2] : 0.0, box ? box->side : 1.0);
  return hipGetLastError();
}

}  // namespace tb
