// tb_parents.hip -- parents one depth at a time, deepest first (Sec. 2.3.2,
// Algorithm 2), with their counts, child links and moments.
//
// Algorithm 2 scans the depth-(d+1) cells in key order and hangs each one on
// the parent whose key is its own key shifted right by three bits, opening a
// new parent whenever that key changes; a parent's centre of mass (and, the
// paper notes, any higher multipole) is computed from its children once they
// are all registered.  In the (depth, key)-ordered array the children of a
// depth-d cell are one contiguous run at depth d+1, and the cell placement pass
// already recorded each internal cell's first child.  One launch per depth:
// every internal depth-d cell walks forward from its first child while the
// child key, shifted right by three, equals its own key -- the same boundary
// test Algorithm 2 applies -- and combines the children:
//
//   M   = sum M_c
//   com = sum M_c (com_c + s_c) / M
//   Q   = sum [Q_c + M_c (3 d_a d_b - |d|^2 delta_ab)],  d = com_c + s_c - com
//
// where s_c = +-l/4 per axis is the child centre relative to the parent centre
// (l the parent side; the octant bit picks the sign), so every quantity stays
// in a cell-relative frame.
#include "tb_internal.h"

namespace tb {

__global__ __launch_bounds__(kParentThreads) void k_parents_fp64(
    int depth, const int64_t *__restrict__ level_offset, const uint64_t *__restrict__ cell_key,
    int32_t *__restrict__ cell_count, int32_t *__restrict__ child_ptr,
    double *__restrict__ com, double *__restrict__ quad, const double *__restrict__ box) {
  const int64_t L0 = level_offset[depth], L1 = level_offset[depth + 1];
  const int64_t L2 = level_offset[depth + 2];
  const double q = ldexp(box[3], -(depth + 2));  // a quarter of the parent side
  const int64_t stride = (int64_t)gridDim.x * blockDim.x;
  for (int64_t pc = L0 + blockIdx.x * (int64_t)blockDim.x + threadIdx.x; pc < L1; pc += stride) {
    const int32_t fc = child_ptr[2 * pc];
    if (fc < 0) continue;  // leaf
    const uint64_t kp = cell_key[pc];
    int64_t c1 = fc;
    double M = 0, S[3] = {0, 0, 0};
    int64_t cnt = 0;
    while (c1 < L2 && c1 < fc + 8 && (cell_key[c1] >> 3) == kp) {
      const uint32_t o = (uint32_t)(cell_key[c1] & 7u);
      const double mc = com[4 * c1 + 3];
      const double r0 = com[4 * c1 + 0] + ((o & 4u) ? q : -q);
      const double r1 = com[4 * c1 + 1] + ((o & 2u) ? q : -q);
      const double r2 = com[4 * c1 + 2] + ((o & 1u) ? q : -q);
      M += mc;
      S[0] += mc * r0;
      S[1] += mc * r1;
      S[2] += mc * r2;
      cnt += cell_count[c1];
      ++c1;
    }
    const double c0 = S[0] / M, cy = S[1] / M, cz = S[2] / M;
    double Q[6] = {0, 0, 0, 0, 0, 0};
    for (int64_t c = fc; c < c1; ++c) {
      const uint32_t o = (uint32_t)(cell_key[c] & 7u);
      const double mc = com[4 * c + 3];
      const double d0 = com[4 * c + 0] + ((o & 4u) ? q : -q) - c0;
      const double d1 = com[4 * c + 1] + ((o & 2u) ? q : -q) - cy;
      const double d2 = com[4 * c + 2] + ((o & 1u) ? q : -q) - cz;
      const double dd = d0 * d0 + d1 * d1 + d2 * d2;
      Q[0] += quad[6 * c + 0] + mc * (3.0 * d0 * d0 - dd);
      Q[1] += quad[6 * c + 1] + mc * (3.0 * d0 * d1);
      Q[2] += quad[6 * c + 2] + mc * (3.0 * d0 * d2);
      Q[3] += quad[6 * c + 3] + mc * (3.0 * d1 * d1 - dd);
      Q[4] += quad[6 * c + 4] + mc * (3.0 * d1 * d2);
      Q[5] += quad[6 * c + 5] + mc * (3.0 * d2 * d2 - dd);
    }
    cell_count[pc] = (int32_t)cnt;
    child_ptr[2 * pc + 1] = (int32_t)(c1 - fc);
    com[4 * pc + 0] = c0;
    com[4 * pc + 1] = cy;
    com[4 * pc + 2] = cz;
    com[4 * pc + 3] = M;
#pragma unroll
    for (int k = 0; k < 6; ++k) quad[6 * pc + k] = Q[k];
  }
}

hipError_t launch_parents(const Plan &p, const Work &w, int depth, const tb_tree &out,
                          hipStream_t s) {
  (void)w;
  // at most 8^depth cells at this depth
  int64_t bound = p.c_max;
  if (depth < 10) {
    const int64_t b8 = int64_t(1) << (3 * depth);
    if (b8 < bound) bound = b8;
  }
  int64_t blocks = (bound + kParentThreads - 1) / kParentThreads;
  if (blocks > 2048) blocks = 2048;
  if (blocks < 1) blocks = 1;
  k_parents_fp64<<<(unsigned)blocks, kParentThreads, 0, s>>>(
      depth, out.level_offset, out.cell_key, out.cell_count, out.child_ptr,
      static_cast<double *>(out.com), static_cast<double *>(out.quad), w.box);
  return hipGetLastError();
}

}  // namespace tb
