// tb_moments.h -- monopole, centre of mass and traceless quadrupole of cells
// (Sec. 2.3.2 and its footnotes), shared by the kernels that build leaves,
// block subtrees and the cells above the blocks.
//
// Frames.  A leaf sums over its particles relative to its own geometric
// centre.  A parent combines its children in its own frame: a child's centre
// sits at +-l/4 per axis from the parent centre (l the parent side; the child's
// octant bit picks the sign), so every quantity stays cell-relative:
//   M   = sum M_c
//   com = sum M_c (com_c + s_c) / M
//   Q   = sum [Q_c + M_c (3 d_a d_b - |d|^2 delta_ab)],  d = com_c + s_c - com.
// FP64: plain sums.  Mixed precision: FP32 with Kahan-compensated sums in units
// of the cell side; each cell also keeps the compensation of its mass (m_lo).
#pragma once

#include "tb_internal.h"

namespace tb {

#if defined(__HIP_DEVICE_COMPILE__) || defined(__HIPCC__)

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

// Cell coordinates (i, j, k) at depth d of the cell whose key is `ckey` (its
// leading 1 at bit 3d).  Morton keys interleave them directly; a Peano-Hilbert
// key is decoded with the inverse of the encoding of tb_internal.h: the Gray
// code undone, then the levels' inversions and swaps undone bottom-up.
__device__ __forceinline__ void cell_coords(uint64_t ckey, int d, bool hilbert, uint32_t c[3]) {
  const uint64_t idx = ckey & ((1ull << (3 * d)) - 1ull);
  uint32_t x = compact3(idx >> 2), y = compact3(idx >> 1), z = compact3(idx);
  if (hilbert && d > 0) {
    const uint32_t t = z >> 1;
    z ^= y;
    y ^= x;
    x ^= t;
    const uint32_t top = 1u << d;
    for (uint32_t bit = 2u; bit != top; bit <<= 1) {
      const uint32_t low = bit - 1u;
      if (z & bit) {
        x ^= low;
      } else {
        const uint32_t u = (x ^ z) & low;
        x ^= u;
        z ^= u;
      }
      if (y & bit) {
        x ^= low;
      } else {
        const uint32_t u = (x ^ y) & low;
        x ^= u;
        y ^= u;
      }
      if (x & bit) x ^= low;
    }
  }
  c[0] = x;
  c[1] = y;
  c[2] = z;
}

// Octant (x, y, z bits, x the most significant) of a depth-d cell inside its
// parent; for Morton keys simply the key's last digit.
__device__ __forceinline__ uint32_t child_octant(uint64_t ckey, int d, bool hilbert) {
  if (!hilbert) return (uint32_t)(ckey & 7u);
  uint32_t c[3];
  cell_coords(ckey, d, true, c);
  return ((c[0] & 1u) << 2) | ((c[1] & 1u) << 1) | (c[2] & 1u);
}

// ---- FP64 leaves: one pass of m, m r, m r r relative to the leaf centre ----
struct LeafSums {
  double s0, s1[3], s2[6];
};

__device__ __forceinline__ void leaf_zero(LeafSums &a) {
  a.s0 = 0.0;
#pragma unroll
  for (int k = 0; k < 3; ++k) a.s1[k] = 0.0;
#pragma unroll
  for (int k = 0; k < 6; ++k) a.s2[k] = 0.0;
}

__device__ __forceinline__ void leaf_add(LeafSums &a, float4 rec, const double lo[3],
                                         const double off[3]) {
  const double m = (double)rec.w;
  const double r0 = __dsub_rn(__dsub_rn((double)rec.x, lo[0]), off[0]);
  const double r1 = __dsub_rn(__dsub_rn((double)rec.y, lo[1]), off[1]);
  const double r2 = __dsub_rn(__dsub_rn((double)rec.z, lo[2]), off[2]);
  a.s0 += m;
  a.s1[0] += m * r0;
  a.s1[1] += m * r1;
  a.s1[2] += m * r2;
  a.s2[0] += m * r0 * r0;
  a.s2[1] += m * r0 * r1;
  a.s2[2] += m * r0 * r2;
  a.s2[3] += m * r1 * r1;
  a.s2[4] += m * r1 * r2;
  a.s2[5] += m * r2 * r2;
}

__device__ __forceinline__ void leaf_finish(const LeafSums &a, double com[4], double quad[6]) {
  const double M = a.s0;
  const double c0 = a.s1[0] / M, c1 = a.s1[1] / M, c2 = a.s1[2] / M;
  const double xx = a.s2[0] - M * c0 * c0, xy = a.s2[1] - M * c0 * c1, xz = a.s2[2] - M * c0 * c2;
  const double yy = a.s2[3] - M * c1 * c1, yz = a.s2[4] - M * c1 * c2, zz = a.s2[5] - M * c2 * c2;
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
}

__device__ __forceinline__ void store_moments_fp64(double *com, double *quad, int64_t c,
                                                   const double cm[4], const double qd[6]) {
  double2 *cd = reinterpret_cast<double2 *>(com + 4 * c);
  cd[0] = make_double2(cm[0], cm[1]);
  cd[1] = make_double2(cm[2], cm[3]);
  double2 *qq = reinterpret_cast<double2 *>(quad + 6 * c);
  qq[0] = make_double2(qd[0], qd[1]);
  qq[1] = make_double2(qd[2], qd[3]);
  qq[2] = make_double2(qd[4], qd[5]);
}

// ---- mixed precision: FP32 sums with Kahan compensation, in cell units ----
__device__ __forceinline__ void kahan_add(float &sum, float &comp, float x) {
  const float y = x - comp;
  const float t = sum + y;
  comp = (t - sum) - y;
  sum = t;
}

struct LeafSumsF {
  float s[10], c[10];  // m, m u (3), m u u (6): sums and Kahan compensations
};

__device__ __forceinline__ void leaf_zero(LeafSumsF &a) {
#pragma unroll
  for (int k = 0; k < 10; ++k) a.s[k] = a.c[k] = 0.0f;
}

// One particle's contribution in units of the leaf side.  The offset from the
// leaf centre is formed from the particle's quantised coordinate: FP64 only
// recomputes t = fl64(x - lo) * 2^21 / side exactly as the key does; then
// (q - base - half) is exact in FP32 and adding the fraction t - q rounds once.
__device__ __forceinline__ void leaf_add_f(LeafSumsF &a, float4 rec, const double lo[3],
                                           double scale, const uint32_t base[3], float half,
                                           int dl) {
  const float m = rec.w;
  const float xv[3] = {rec.x, rec.y, rec.z};
  float u[3];
#pragma unroll
  for (int k = 0; k < 3; ++k) {
    const double t = __dmul_rn(__dsub_rn((double)xv[k], lo[k]), scale);
    double qd = floor(t);
    if (!(qd >= 0.0)) qd = 0.0;  // also a NaN position (flagged by the key pass)
    if (qd > 2097151.0) qd = 2097151.0;
    const int32_t q = (int32_t)qd;
    const float frac = (float)(t - qd);
    const float r = ((float)(q - (int32_t)base[k]) - half) + frac;  // grid units
    u[k] = ldexpf(r, dl - kMaxDepth);                                 // leaf units
  }
  kahan_add(a.s[0], a.c[0], m);
  kahan_add(a.s[1], a.c[1], m * u[0]);
  kahan_add(a.s[2], a.c[2], m * u[1]);
  kahan_add(a.s[3], a.c[3], m * u[2]);
  kahan_add(a.s[4], a.c[4], m * u[0] * u[0]);
  kahan_add(a.s[5], a.c[5], m * u[0] * u[1]);
  kahan_add(a.s[6], a.c[6], m * u[0] * u[2]);
  kahan_add(a.s[7], a.c[7], m * u[1] * u[1]);
  kahan_add(a.s[8], a.c[8], m * u[1] * u[2]);
  kahan_add(a.s[9], a.c[9], m * u[2] * u[2]);
}

// com (in cell units), M, its compensation, and Q (cell units).
__device__ __forceinline__ void leaf_finish_f(const LeafSumsF &a, float com[4], float &m_lo,
                                              float quad[6]) {
  const float M = a.s[0];
  const float c0 = a.s[1] / M, c1 = a.s[2] / M, c2 = a.s[3] / M;
  const float xx = a.s[4] - M * c0 * c0, xy = a.s[5] - M * c0 * c1, xz = a.s[6] - M * c0 * c2;
  const float yy = a.s[7] - M * c1 * c1, yz = a.s[8] - M * c1 * c2, zz = a.s[9] - M * c2 * c2;
  const float tr = xx + yy + zz;
  com[0] = c0;
  com[1] = c1;
  com[2] = c2;
  com[3] = M;
  m_lo = -a.c[0];
  quad[0] = 3.0f * xx - tr;
  quad[1] = 3.0f * xy;
  quad[2] = 3.0f * xz;
  quad[3] = 3.0f * yy - tr;
  quad[4] = 3.0f * yz;
  quad[5] = 3.0f * zz - tr;
}

// Mixed leaf results are stored in absolute units: scaling by the side (a power
// of two) is exact.
__device__ __forceinline__ void store_moments_mixed(float *com, float *quad, float *m_lo,
                                                    int64_t c, const float cm[4], float mlo,
                                                    const float qd[6], float l) {
  reinterpret_cast<float4 *>(com)[c] = make_float4(cm[0] * l, cm[1] * l, cm[2] * l, cm[3]);
  const float l2 = l * l;
  float2 *qq = reinterpret_cast<float2 *>(quad + 6 * c);
  qq[0] = make_float2(qd[0] * l2, qd[1] * l2);
  qq[1] = make_float2(qd[2] * l2, qd[3] * l2);
  qq[2] = make_float2(qd[4] * l2, qd[5] * l2);
  m_lo[c] = mlo;
}

// ---- parents from their children (children: nch consecutive cells from c0) ----
// dp is the parent's depth, side the root box side.  The children's count,
// centre of mass and quadrupole must be final; the parent's count, number of
// children and moments are written.
__device__ inline void parent_from_children_fp64(int64_t pc, int64_t c0, int nch, int dp,
                                                 double side, const uint64_t *cell_key,
                                                 int32_t *cell_count, int32_t *child_ptr,
                                                 double *com, double *quad, bool hilbert) {
  const double q = ldexp(side, -(dp + 2));  // a quarter of the parent side
  double M = 0.0, S0 = 0.0, S1 = 0.0, S2 = 0.0;
  int64_t cnt = 0;
  uint32_t octs = 0;  // 3 bits per child
  for (int k = 0; k < nch; ++k) {
    const int64_t x = c0 + k;
    const uint32_t o = child_octant(cell_key[x], dp + 1, hilbert);
    octs |= o << (3 * k);
    const double4 cm = *reinterpret_cast<const double4 *>(com + 4 * x);
    M += cm.w;
    S0 += cm.w * (cm.x + ((o & 4u) ? q : -q));
    S1 += cm.w * (cm.y + ((o & 2u) ? q : -q));
    S2 += cm.w * (cm.z + ((o & 1u) ? q : -q));
    cnt += cell_count[x];
  }
  const double cx = S0 / M, cy = S1 / M, cz = S2 / M;
  double Q[6] = {0, 0, 0, 0, 0, 0};
  for (int k = 0; k < nch; ++k) {
    const int64_t x = c0 + k;
    const uint32_t o = (octs >> (3 * k)) & 7u;
    const double4 cm = *reinterpret_cast<const double4 *>(com + 4 * x);
    const double *qc = quad + 6 * x;
    const double d0 = cm.x + ((o & 4u) ? q : -q) - cx;
    const double d1 = cm.y + ((o & 2u) ? q : -q) - cy;
    const double d2 = cm.z + ((o & 1u) ? q : -q) - cz;
    const double dd = d0 * d0 + d1 * d1 + d2 * d2;
    Q[0] += qc[0] + cm.w * (3.0 * d0 * d0 - dd);
    Q[1] += qc[1] + cm.w * (3.0 * d0 * d1);
    Q[2] += qc[2] + cm.w * (3.0 * d0 * d2);
    Q[3] += qc[3] + cm.w * (3.0 * d1 * d1 - dd);
    Q[4] += qc[4] + cm.w * (3.0 * d1 * d2);
    Q[5] += qc[5] + cm.w * (3.0 * d2 * d2 - dd);
  }
  cell_count[pc] = (int32_t)cnt;
  child_ptr[2 * pc + 1] = nch;
  const double cm[4] = {cx, cy, cz, M};
  store_moments_fp64(com, quad, pc, cm, Q);
}

__device__ inline void parent_from_children_mixed(int64_t pc, int64_t c0, int nch, int dp,
                                                  double side, const uint64_t *cell_key,
                                                  int32_t *cell_count, int32_t *child_ptr,
                                                  float *com, float *quad, float *m_lo,
                                                  bool hilbert) {
  const float lc = ldexpf((float)side, -(dp + 1));  // child side
  const float lp = 2.0f * lc;                       // parent side
  const float inv_lc = 1.0f / lc, inv_lc2 = inv_lc * inv_lc;
  float M = 0.f, Mc = 0.f, S[3] = {0.f, 0.f, 0.f}, Sc[3] = {0.f, 0.f, 0.f};
  int64_t cnt = 0;
  uint32_t octs = 0;  // 3 bits per child
  for (int k = 0; k < nch; ++k) {
    const int64_t x = c0 + k;
    const uint32_t o = child_octant(cell_key[x], dp + 1, hilbert);
    octs |= o << (3 * k);
    const float4 cm = reinterpret_cast<const float4 *>(com)[x];
    const float up[3] = {0.5f * (cm.x * inv_lc) + ((o & 4u) ? 0.25f : -0.25f),
                         0.5f * (cm.y * inv_lc) + ((o & 2u) ? 0.25f : -0.25f),
                         0.5f * (cm.z * inv_lc) + ((o & 1u) ? 0.25f : -0.25f)};
    kahan_add(M, Mc, cm.w);
    kahan_add(M, Mc, m_lo[x]);
#pragma unroll
    for (int a = 0; a < 3; ++a) kahan_add(S[a], Sc[a], cm.w * up[a]);
    cnt += cell_count[x];
  }
  const float cx = S[0] / M, cy = S[1] / M, cz = S[2] / M;
  float Q[6] = {0, 0, 0, 0, 0, 0}, Qc[6] = {0, 0, 0, 0, 0, 0};
  const float qs = 0.25f * inv_lc2;  // child units -> parent units
  for (int k = 0; k < nch; ++k) {
    const int64_t x = c0 + k;
    const uint32_t o = (octs >> (3 * k)) & 7u;
    const float4 cm = reinterpret_cast<const float4 *>(com)[x];
    const float *qc = quad + 6 * x;
    const float mc = cm.w;
    const float d0 = 0.5f * (cm.x * inv_lc) + ((o & 4u) ? 0.25f : -0.25f) - cx;
    const float d1 = 0.5f * (cm.y * inv_lc) + ((o & 2u) ? 0.25f : -0.25f) - cy;
    const float d2 = 0.5f * (cm.z * inv_lc) + ((o & 1u) ? 0.25f : -0.25f) - cz;
    const float dd = d0 * d0 + d1 * d1 + d2 * d2;
    kahan_add(Q[0], Qc[0], qc[0] * qs + mc * (3.0f * d0 * d0 - dd));
    kahan_add(Q[1], Qc[1], qc[1] * qs + mc * (3.0f * d0 * d1));
    kahan_add(Q[2], Qc[2], qc[2] * qs + mc * (3.0f * d0 * d2));
    kahan_add(Q[3], Qc[3], qc[3] * qs + mc * (3.0f * d1 * d1 - dd));
    kahan_add(Q[4], Qc[4], qc[4] * qs + mc * (3.0f * d1 * d2));
    kahan_add(Q[5], Qc[5], qc[5] * qs + mc * (3.0f * d2 * d2 - dd));
  }
  cell_count[pc] = (int32_t)cnt;
  child_ptr[2 * pc + 1] = nch;
  const float cm[4] = {cx, cy, cz, M};
  store_moments_mixed(com, quad, m_lo, pc, cm, -Mc, Q, lp);
}

#endif

}  // namespace tb
