// tb_parents.hip -- parents one depth at a time, deepest first (Sec. 2.3.2,
// Algorithm 2), with their counts, child links and moments.
//
// Algorithm 2 scans the depth-(d+1) cells in key order and hangs each one on
// the parent whose key is its own key shifted right by three bits, opening a
// new parent whenever that key changes; a parent's centre of mass (and, the
// paper notes, any higher multipole) is computed from its children once they
// are all registered.  In the (depth, key)-ordered array the children of a
// depth-d cell are one contiguous run at depth d+1, and the cell placement pass
// already recorded each internal cell's first child and, for that first child,
// the slot of its parent.  One launch per depth: the depth-(d+1) cells (and the
// parent slots of their first children) are staged through LDS in key order; a
// child whose key, shifted right by three, differs from its predecessor's --
// the boundary test of Algorithm 2 -- opens the run of its siblings.  The
// openers of a chunk are packed to the low threads, each of which combines its
// run into the parent:
//
//   M   = sum M_c
//   com = sum M_c (com_c + s_c) / M
//   Q   = sum [Q_c + M_c (3 d_a d_b - |d|^2 delta_ab)],  d = com_c + s_c - com
//
// where s_c = +-l/4 per axis is the child centre relative to the parent centre
// (l the parent side; the octant bit picks the sign), so every quantity stays
// in a cell-relative frame.
#include "tb_internal.h"
#include "tb_moments.h"

namespace tb {

constexpr int kChunk = kParentThreads;  // children staged per workgroup step
static_assert(kChunk == kParentThreads, "one staged child (and parent slot) per thread");
constexpr int kHalo = 7;                 // a parent has at most 8 children

// A set's parents [P0, P1) and children [P1, L2) at one depth, the first parent
// chunk of the set (row_b) and the side of its root box.
struct SetBounds {
  int64_t P0, P1, L2, row_b;
  double side;
};

__device__ inline SetBounds set_bounds(int b, int depth, const int64_t *row,
                                       const int64_t *level_offset, const double *box) {
  const int64_t *lo_b = level_offset + b * (kLevels + 1);
  return {lo_b[depth], lo_b[depth + 1], lo_b[depth + 2], row[b], box[4 * b + 3]};
}

// Packs the chunk positions of the run openers (a child at or past L1 whose
// key >> 3 differs from the previous child's) into s_open and returns their
// number.  s_key holds the keys of [base - 1, base + kChunk + kHalo); zero
// outside [L1, L2).  Both barriers are block-wide.
__device__ inline int pack_openers(const uint64_t *s_key, int64_t base, int64_t L1, int64_t L2,
                                   int *s_wop, uint16_t *s_open) {
  const int t = threadIdx.x;
  const int64_t c = base + t;
  const bool op = c < L2 && (c == L1 || (s_key[t] >> 3) != (s_key[t + 1] >> 3));
  const uint64_t bal = __ballot(op);
  if (lane_id() == 0) s_wop[t >> 6] = __popcll(bal);
  __syncthreads();
  int before = 0, total = 0;
#pragma unroll
  for (int w = 0; w < kParentThreads / 64; ++w) {
    const int v = s_wop[w];
    before += w < (t >> 6) ? v : 0;
    total += v;
  }
  if (op) s_open[before + __popcll(bal & lanemask_lt())] = (uint16_t)t;
  __syncthreads();
  return total;
}

__global__ __launch_bounds__(kParentThreads) void k_parents_fp64(
    int depth, const int64_t *__restrict__ level_offset, const uint64_t *__restrict__ cell_key,
    int32_t *__restrict__ cell_count, int32_t *__restrict__ child_ptr,
    double *__restrict__ com, double *__restrict__ quad, const int32_t *__restrict__ head_parent,
    const double *__restrict__ box, int32_t *__restrict__ status_word, int32_t nsets,
    const int64_t *__restrict__ par_start, int hilbert) {
  __shared__ uint64_t s_key[kChunk + kHalo + 1];  // keys of [base - 1, base + kChunk + kHalo)
  __shared__ int32_t s_cnt[kChunk + kHalo];
  __shared__ int32_t s_hp[kChunk];  // parent slot of each staged first child
  __shared__ int s_wop[kParentThreads / 64];
  __shared__ uint16_t s_open[kChunk];
  __shared__ __align__(16) double s_com[(kChunk + kHalo) * 4];
  __shared__ __align__(16) double s_quad[(kChunk + kHalo) * 6];

  __shared__ int s_set;
  const int64_t *row = par_start + depth * (nsets + 1);
  const int64_t n_chunks = row[nsets];
  bool internal = false;
  // the chunk's set and its bounds: loaded once for a single set (they are the
  // same for every chunk), per chunk in a batch
  SetBounds sb = {0, 0, 0, 0, 1.0};
  if (nsets == 1) sb = set_bounds(0, depth, row, level_offset, box);
  for (int64_t ch = blockIdx.x; ch < n_chunks; ch += gridDim.x) {
    if (nsets > 1) {
      if (threadIdx.x == 0) s_set = upper_index(row, nsets + 1, ch);
      __syncthreads();
      sb = set_bounds(s_set, depth, row, level_offset, box);
    }
    const int64_t P0 = sb.P0, P1 = sb.P1;
    const int64_t L1 = P1, L2 = sb.L2;
    const double q = ldexp(sb.side, -(depth + 2));  // a quarter of the parent side
    const int64_t base = L1 + (ch - sb.row_b) * (int64_t)kChunk;
    // stage the chunk: every load is issued before the first LDS store
    const int64_t lim = min((int64_t)(kChunk + kHalo), L2 - base);
    constexpr int KN = (kChunk + kHalo + 1 + kParentThreads - 1) / kParentThreads;
    constexpr int CN = (kChunk + kHalo + kParentThreads - 1) / kParentThreads;
    constexpr int MN = ((kChunk + kHalo) * 2 + kParentThreads - 1) / kParentThreads;
    constexpr int QN = ((kChunk + kHalo) * 3 + kParentThreads - 1) / kParentThreads;
    uint64_t kv[KN];
    int32_t cv[CN];
    double2 mv[MN], qv[QN];
    const int32_t hv = base + threadIdx.x < L2 ? head_parent[base + threadIdx.x] : -1;
    const double2 *com2 = reinterpret_cast<const double2 *>(com) + 2 * base;
    const double2 *quad2 = reinterpret_cast<const double2 *>(quad) + 3 * base;
#pragma unroll
    for (int r = 0; r < KN; ++r) {
      const int x = r * kParentThreads + threadIdx.x;
      const int64_t c = base - 1 + x;
      kv[r] = (x < kChunk + kHalo + 1 && c >= L1 && c < L2) ? cell_key[c] : 0ull;
    }
#pragma unroll
    for (int r = 0; r < CN; ++r) {
      const int x = r * kParentThreads + threadIdx.x;
      cv[r] = x < lim ? cell_count[base + x] : 0;
    }
#pragma unroll
    for (int r = 0; r < MN; ++r) {
      const int x = r * kParentThreads + threadIdx.x;
      mv[r] = x < 2 * lim ? com2[x] : make_double2(0.0, 0.0);
    }
#pragma unroll
    for (int r = 0; r < QN; ++r) {
      const int x = r * kParentThreads + threadIdx.x;
      qv[r] = x < 3 * lim ? quad2[x] : make_double2(0.0, 0.0);
    }
#pragma unroll
    for (int r = 0; r < KN; ++r) {
      const int x = r * kParentThreads + threadIdx.x;
      if (x < kChunk + kHalo + 1) s_key[x] = kv[r];  // 0 never matches a parent key
    }
#pragma unroll
    for (int r = 0; r < CN; ++r) {
      const int x = r * kParentThreads + threadIdx.x;
      if (x < lim) s_cnt[x] = cv[r];
    }
    s_hp[threadIdx.x] = hv;
#pragma unroll
    for (int r = 0; r < MN; ++r) {
      const int x = r * kParentThreads + threadIdx.x;
      if (x < 2 * lim) reinterpret_cast<double2 *>(s_com)[x] = mv[r];
    }
#pragma unroll
    for (int r = 0; r < QN; ++r) {
      const int x = r * kParentThreads + threadIdx.x;
      if (x < 3 * lim) reinterpret_cast<double2 *>(s_quad)[x] = qv[r];
    }
    __syncthreads();

    const int n_open = pack_openers(s_key, base, L1, L2, s_wop, s_open);
    if ((int)threadIdx.x < n_open) {
      const int t = s_open[threadIdx.x];
      const uint64_t kp = s_key[t + 1] >> 3;
      const int64_t pc = s_hp[t];
      int nch = 0;
      while (nch < 8 && t + nch < lim && (s_key[t + nch + 1] >> 3) == kp) ++nch;
      if (pc < P0 || pc >= P1) {
        internal = true;
      } else {
        double M = 0.0, S0 = 0.0, S1 = 0.0, S2 = 0.0;
        int64_t cnt = 0;
        uint32_t octs = 0;  // 3 bits per child
        for (int k = 0; k < nch; ++k) {
          const int x = t + k;
          const uint32_t o = child_octant(s_key[x + 1], depth + 1, hilbert != 0);
          octs |= o << (3 * k);
          const double mc = s_com[4 * x + 3];
          M += mc;
          S0 += mc * (s_com[4 * x + 0] + ((o & 4u) ? q : -q));
          S1 += mc * (s_com[4 * x + 1] + ((o & 2u) ? q : -q));
          S2 += mc * (s_com[4 * x + 2] + ((o & 1u) ? q : -q));
          cnt += s_cnt[x];
        }
        const double cx = S0 / M, cy = S1 / M, cz = S2 / M;
        double Q[6] = {0, 0, 0, 0, 0, 0};
        for (int k = 0; k < nch; ++k) {
          const int x = t + k;
          const uint32_t o = (octs >> (3 * k)) & 7u;
          const double mc = s_com[4 * x + 3];
          const double d0 = s_com[4 * x + 0] + ((o & 4u) ? q : -q) - cx;
          const double d1 = s_com[4 * x + 1] + ((o & 2u) ? q : -q) - cy;
          const double d2 = s_com[4 * x + 2] + ((o & 1u) ? q : -q) - cz;
          const double dd = d0 * d0 + d1 * d1 + d2 * d2;
          Q[0] += s_quad[6 * x + 0] + mc * (3.0 * d0 * d0 - dd);
          Q[1] += s_quad[6 * x + 1] + mc * (3.0 * d0 * d1);
          Q[2] += s_quad[6 * x + 2] + mc * (3.0 * d0 * d2);
          Q[3] += s_quad[6 * x + 3] + mc * (3.0 * d1 * d1 - dd);
          Q[4] += s_quad[6 * x + 4] + mc * (3.0 * d1 * d2);
          Q[5] += s_quad[6 * x + 5] + mc * (3.0 * d2 * d2 - dd);
        }
        cell_count[pc] = (int32_t)cnt;
        child_ptr[2 * pc + 1] = nch;
        double2 *cd = reinterpret_cast<double2 *>(com + 4 * pc);
        cd[0] = make_double2(cx, cy);
        cd[1] = make_double2(cz, M);
        double2 *qd = reinterpret_cast<double2 *>(quad + 6 * pc);
        qd[0] = make_double2(Q[0], Q[1]);
        qd[1] = make_double2(Q[2], Q[3]);
        qd[2] = make_double2(Q[4], Q[5]);
      }
    }
    __syncthreads();
  }
  if (__ballot(internal) != 0 && lane_id() == 0) atomicOr(status_word, TB_STATUS_INTERNAL);
}

// Mixed precision: the same combination in FP32 with Kahan-compensated sums,
// in units of the parent side (a child's frame maps to the parent's by an
// exact halving and a shift of +-1/4).  The stored moments are in absolute
// units; converting by powers of two is exact.  Each cell's mass also carries
// its compensation term (m_lo) so that the mass stays correctly rounded at
// every depth.
__device__ __forceinline__ void kahan_add_p(float &sum, float &comp, float x) {
  const float y = x - comp;
  const float t = sum + y;
  comp = (t - sum) - y;
  sum = t;
}

__global__ __launch_bounds__(kParentThreads) void k_parents_mixed(
    int depth, const int64_t *__restrict__ level_offset, const uint64_t *__restrict__ cell_key,
    int32_t *__restrict__ cell_count, int32_t *__restrict__ child_ptr,
    float *__restrict__ com, float *__restrict__ quad, float *__restrict__ m_lo,
    const int32_t *__restrict__ head_parent, const double *__restrict__ box,
    int32_t *__restrict__ status_word, int32_t nsets, const int64_t *__restrict__ par_start,
    int hilbert) {
  __shared__ uint64_t s_key[kChunk + kHalo + 1];
  __shared__ int32_t s_cnt[kChunk + kHalo];
  __shared__ int32_t s_hp[kChunk];
  __shared__ int s_wop[kParentThreads / 64];
  __shared__ uint16_t s_open[kChunk];
  __shared__ float4 s_com[kChunk + kHalo];
  __shared__ __align__(16) float s_quad[(kChunk + kHalo) * 6];
  __shared__ float s_mlo[kChunk + kHalo];

  __shared__ int s_set;
  const int64_t *row = par_start + depth * (nsets + 1);
  const int64_t n_chunks = row[nsets];
  bool internal = false;
  SetBounds sb = {0, 0, 0, 0, 1.0};
  if (nsets == 1) sb = set_bounds(0, depth, row, level_offset, box);
  for (int64_t ch = blockIdx.x; ch < n_chunks; ch += gridDim.x) {
    if (nsets > 1) {
      if (threadIdx.x == 0) s_set = upper_index(row, nsets + 1, ch);
      __syncthreads();
      sb = set_bounds(s_set, depth, row, level_offset, box);
    }
    const int64_t P0 = sb.P0, P1 = sb.P1;
    const int64_t L1 = P1, L2 = sb.L2;
    const float lc = ldexpf((float)sb.side, -(depth + 1));  // child side
    const float lp = 2.0f * lc;                             // parent side
    const float inv_lc = 1.0f / lc, inv_lc2 = inv_lc * inv_lc;
    const int64_t base = L1 + (ch - sb.row_b) * (int64_t)kChunk;
    const int64_t lim = min((int64_t)(kChunk + kHalo), L2 - base);
    constexpr int KN = (kChunk + kHalo + 1 + kParentThreads - 1) / kParentThreads;
    constexpr int CN = (kChunk + kHalo + kParentThreads - 1) / kParentThreads;
    constexpr int QN = ((kChunk + kHalo) * 3 + kParentThreads - 1) / kParentThreads;
    uint64_t kv[KN];
    int32_t cv[CN];
    const int32_t hv = base + threadIdx.x < L2 ? head_parent[base + threadIdx.x] : -1;
    float4 mv[CN];
    float lv[CN];
    float2 qv[QN];
    const float2 *quad2 = reinterpret_cast<const float2 *>(quad) + 3 * base;
#pragma unroll
    for (int r = 0; r < KN; ++r) {
      const int x = r * kParentThreads + threadIdx.x;
      const int64_t c = base - 1 + x;
      kv[r] = (x < kChunk + kHalo + 1 && c >= L1 && c < L2) ? cell_key[c] : 0ull;
    }
#pragma unroll
    for (int r = 0; r < CN; ++r) {
      const int x = r * kParentThreads + threadIdx.x;
      const int64_t c = base + (x < lim ? x : lim - 1);
      cv[r] = cell_count[c];
      mv[r] = reinterpret_cast<const float4 *>(com)[c];
      lv[r] = m_lo[c];
    }
#pragma unroll
    for (int r = 0; r < QN; ++r) {
      const int x = r * kParentThreads + threadIdx.x;
      qv[r] = quad2[x < 3 * lim ? x : 3 * lim - 1];
    }
#pragma unroll
    for (int r = 0; r < KN; ++r) {
      const int x = r * kParentThreads + threadIdx.x;
      if (x < kChunk + kHalo + 1) s_key[x] = kv[r];
    }
#pragma unroll
    for (int r = 0; r < CN; ++r) {
      const int x = r * kParentThreads + threadIdx.x;
      if (x < lim) {
        s_cnt[x] = cv[r];
        s_com[x] = mv[r];
        s_mlo[x] = lv[r];
      }
    }
    s_hp[threadIdx.x] = hv;
#pragma unroll
    for (int r = 0; r < QN; ++r) {
      const int x = r * kParentThreads + threadIdx.x;
      if (x < 3 * lim) reinterpret_cast<float2 *>(s_quad)[x] = qv[r];
    }
    __syncthreads();

    const int n_open = pack_openers(s_key, base, L1, L2, s_wop, s_open);
    if ((int)threadIdx.x < n_open) {
      const int t = s_open[threadIdx.x];
      const uint64_t kp = s_key[t + 1] >> 3;
      const int64_t pc = s_hp[t];
      int nch = 0;
      while (nch < 8 && t + nch < lim && (s_key[t + nch + 1] >> 3) == kp) ++nch;
      if (pc < P0 || pc >= P1) {
        internal = true;
      } else {
        float M = 0.f, Mc = 0.f, S[3] = {0.f, 0.f, 0.f}, Sc[3] = {0.f, 0.f, 0.f};
        int64_t cnt = 0;
        uint32_t octs = 0;  // 3 bits per child
        for (int k = 0; k < nch; ++k) {
          const int x = t + k;
          const uint32_t o = child_octant(s_key[x + 1], depth + 1, hilbert != 0);
          octs |= o << (3 * k);
          const float4 cm = s_com[x];
          const float up[3] = {0.5f * (cm.x * inv_lc) + ((o & 4u) ? 0.25f : -0.25f),
                               0.5f * (cm.y * inv_lc) + ((o & 2u) ? 0.25f : -0.25f),
                               0.5f * (cm.z * inv_lc) + ((o & 1u) ? 0.25f : -0.25f)};
          kahan_add_p(M, Mc, cm.w);
          kahan_add_p(M, Mc, s_mlo[x]);
#pragma unroll
          for (int a = 0; a < 3; ++a) kahan_add_p(S[a], Sc[a], cm.w * up[a]);
          cnt += s_cnt[x];
        }
        const float cx = S[0] / M, cy = S[1] / M, cz = S[2] / M;
        float Q[6] = {0, 0, 0, 0, 0, 0}, Qc[6] = {0, 0, 0, 0, 0, 0};
        for (int k = 0; k < nch; ++k) {
          const int x = t + k;
          const uint32_t o = (octs >> (3 * k)) & 7u;
          const float4 cm = s_com[x];
          const float mc = cm.w;
          const float d0 = 0.5f * (cm.x * inv_lc) + ((o & 4u) ? 0.25f : -0.25f) - cx;
          const float d1 = 0.5f * (cm.y * inv_lc) + ((o & 2u) ? 0.25f : -0.25f) - cy;
          const float d2 = 0.5f * (cm.z * inv_lc) + ((o & 1u) ? 0.25f : -0.25f) - cz;
          const float dd = d0 * d0 + d1 * d1 + d2 * d2;
          const float qs = 0.25f * inv_lc2;  // child units -> parent units
          kahan_add_p(Q[0], Qc[0], s_quad[6 * x + 0] * qs + mc * (3.0f * d0 * d0 - dd));
          kahan_add_p(Q[1], Qc[1], s_quad[6 * x + 1] * qs + mc * (3.0f * d0 * d1));
          kahan_add_p(Q[2], Qc[2], s_quad[6 * x + 2] * qs + mc * (3.0f * d0 * d2));
          kahan_add_p(Q[3], Qc[3], s_quad[6 * x + 3] * qs + mc * (3.0f * d1 * d1 - dd));
          kahan_add_p(Q[4], Qc[4], s_quad[6 * x + 4] * qs + mc * (3.0f * d1 * d2));
          kahan_add_p(Q[5], Qc[5], s_quad[6 * x + 5] * qs + mc * (3.0f * d2 * d2 - dd));
        }
        cell_count[pc] = (int32_t)cnt;
        child_ptr[2 * pc + 1] = nch;
        reinterpret_cast<float4 *>(com)[pc] = make_float4(cx * lp, cy * lp, cz * lp, M);
        const float lp2 = lp * lp;
        float2 *qd = reinterpret_cast<float2 *>(quad + 6 * pc);
        qd[0] = make_float2(Q[0] * lp2, Q[1] * lp2);
        qd[1] = make_float2(Q[2] * lp2, Q[3] * lp2);
        qd[2] = make_float2(Q[4] * lp2, Q[5] * lp2);
        m_lo[pc] = -Mc;
      }
    }
    __syncthreads();
  }
  if (__ballot(internal) != 0 && lane_id() == 0) atomicOr(status_word, TB_STATUS_INTERNAL);
}

hipError_t launch_parents(const Plan &p, const Work &w, int depth, const tb_tree &out,
                          hipStream_t s) {
  // at most 8^(depth+1) children per set one depth down, in chunks of kChunk
  int64_t bound = p.c_max;
  if (depth + 1 < 10) {
    const int64_t b8 = (int64_t(1) << (3 * (depth + 1))) * p.nsets;
    if (b8 < bound) bound = b8;
  }
  int64_t blocks = (bound + kChunk - 1) / kChunk + p.nsets;
  if (blocks > 1024) blocks = 1024;
  if (blocks < 1) blocks = 1;
  if ((p.flags & 0xffu) == TB_MIXED)
    k_parents_mixed<<<(unsigned)blocks, kParentThreads, 0, s>>>(
        depth, w.lvl_off, out.cell_key, out.cell_count, out.child_ptr,
        static_cast<float *>(out.com), static_cast<float *>(out.quad), w.m_lo, w.head_parent,
        w.box, out.status, p.nsets, w.par_start, (p.flags & TB_HILBERT) ? 1 : 0);
  else
    k_parents_fp64<<<(unsigned)blocks, kParentThreads, 0, s>>>(
        depth, w.lvl_off, out.cell_key, out.cell_count, out.child_ptr,
        static_cast<double *>(out.com), static_cast<double *>(out.quad), w.head_parent, w.box,
        out.status, p.nsets, w.par_start, (p.flags & TB_HILBERT) ? 1 : 0);
  return hipGetLastError();
}

}  // namespace tb
