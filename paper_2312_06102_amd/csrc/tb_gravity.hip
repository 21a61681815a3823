// tb_gravity.hip -- the gravity calculation that consumes the tree (Sec. 2.1).
//
// Barnes-Hut with Barnes' shared interaction lists: the particles of a group
// (the first cell on each path down from the root that holds at most n_crit
// particles, or is a leaf) share one list, built by one workgroup walking the
// tree from the root.  A cell C is accepted for group G when it is neither G
// nor one of its ancestors and l_C < theta * d, d the distance from C's centre
// of mass to the closest point of G's cube (eq. 1, l/d < theta, then holds for
// every particle of G).  A cell that is not accepted is opened: a leaf gives
// its particles (direct, softened terms), an internal cell its children.
//
// k_find_groups  : every internal cell holding more than n_crit particles
//                  lists those of its children that are groups (the root
//                  itself when it is one).
// k_walk         : one workgroup per group.  The cells still to visit sit on an
//                  LDS stack; each round pops up to one cell per thread, tests
//                  it, appends accepted cells, opened leaves and the children
//                  of opened cells at positions given by block-wide prefix
//                  sums (so lists and sums come out in the same order on every
//                  run), then every thread adds the round's cell and particle
//                  terms to its own group particles.  FP64 throughout.
#include "tb_internal.h"
#include "tb_moments.h"

namespace tb {

constexpr int kWalkThreads = 256;
constexpr int kWalkPpt = 4;                               // group particles per thread per pass
constexpr int kWalkPass = kWalkThreads * kWalkPpt;        // group particles per pass
constexpr int kStackCap = 4096;                           // cells waiting in LDS
constexpr int kPartBatch = 256;                           // source particles staged at once
constexpr int kCellBatch = kWalkThreads / 2;              // accepted cells staged at once

struct GravArgs {
  const uint64_t *key;
  const uint8_t *level;
  const int32_t *first, *count, *child;
  const double *com, *quad;
  const double *box;
  const float *pos;   // sorted positions [n][3]
  const float *mass;  // sorted masses [n]
  double theta2, eps2;
  int quad_on;
  int hilbert;  // the cell keys are Peano-Hilbert keys
};

// Geometric centre (absolute) and side of cell c.
__device__ inline void cell_centre(const GravArgs &g, int64_t c, double cen[3], double &l) {
  const int d = g.level[c];
  uint32_t ijk[3];
  cell_coords(g.key[c], d, g.hilbert != 0, ijk);
  l = ldexp(g.box[3], -d);
#pragma unroll
  for (int a = 0; a < 3; ++a) cen[a] = g.box[a] + ((double)ijk[a] + 0.5) * l;
}

__global__ void k_grav_init(uint32_t *__restrict__ n_groups, unsigned long long *__restrict__ stats) {
  if (threadIdx.x == 0) *n_groups = 0;
  if (stats && threadIdx.x < 2) stats[threadIdx.x] = 0;
}

__global__ __launch_bounds__(256) void k_find_groups(
    const int64_t *__restrict__ n_cells, const int32_t *__restrict__ count,
    const int32_t *__restrict__ child, int32_t n_crit, int32_t *__restrict__ groups,
    uint32_t *__restrict__ n_groups) {
  const int64_t C = *n_cells;
  for (int64_t c = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; c < C;
       c += (int64_t)gridDim.x * blockDim.x) {
    const bool leaf = child[2 * c] < 0;
    if (c == 0 && (leaf || count[0] <= n_crit)) groups[atomicAdd(n_groups, 1u)] = 0;
    if (leaf || count[c] <= n_crit) continue;
    const int32_t f = child[2 * c], nch = child[2 * c + 1];
    for (int k = 0; k < nch; ++k) {
      const int32_t ch = f + k;
      if (child[2 * ch] < 0 || count[ch] <= n_crit) groups[atomicAdd(n_groups, 1u)] = ch;
    }
  }
}

// Block-wide exclusive prefix of v (256 threads); *total receives the sum.
__device__ inline int block_excl(int v, int *s_w, int *total) {
  const int wv = threadIdx.x >> 6;
  const uint32_t inc = wave_inclusive_scan((uint32_t)v);
  if (lane_id() == 63) s_w[wv] = (int)inc;
  __syncthreads();
  int off = 0, tot = 0;
#pragma unroll
  for (int q = 0; q < kWalkThreads / 64; ++q) {
    const int t = s_w[q];
    off += q < wv ? t : 0;
    tot += t;
  }
  __syncthreads();
  *total = tot;
  return off + (int)inc - v;
}

// Four workgroups a CU: 38.9 KB of LDS each (the cells and particles of a
// round are staged in halves), and registers held to four waves a SIMD
// (128 VGPRs, no spill).
__global__ __launch_bounds__(kWalkThreads, 4) void k_walk(
    GravArgs g, const int32_t *__restrict__ groups, const uint32_t *__restrict__ n_groups,
    double *__restrict__ acc, unsigned long long *__restrict__ stats,
    int32_t *__restrict__ status_word) {
  __shared__ int32_t s_stack[kStackCap];
  __shared__ int32_t s_cells[kWalkThreads];   // accepted cells of the round
  __shared__ int32_t s_leaves[kWalkThreads];  // opened leaves of the round
  __shared__ int32_t s_lstart[kWalkThreads + 1];
  __shared__ double s_cdat[kCellBatch][10];   // com (abs) x y z, M, Q[6]
  __shared__ double s_part[kPartBatch][4];     // x y z m of staged source particles
  __shared__ int32_t s_pidx[kPartBatch];
  __shared__ int s_w[kWalkThreads / 64];
  __shared__ int s_top, s_over;

  const uint32_t G = *n_groups;
  for (uint32_t gi = blockIdx.x; gi < G; gi += gridDim.x) {
    const int32_t grp = groups[gi];
    double gc[3], gl;
    cell_centre(g, grp, gc, gl);
    const double gh = 0.5 * gl;
    const int gd = g.level[grp];
    const uint64_t gkey = g.key[grp];
    const int64_t gf = g.first[grp], gn = g.count[grp];
    unsigned long long my_cells = 0, my_pairs = 0;
    // groups larger than one pass (saturated depth-21 leaves, n_crit > kWalkPass)
    // walk the tree once per pass
    for (int64_t p0 = 0; p0 < gn; p0 += kWalkPass) {
      double xi[kWalkPpt][3], ai[kWalkPpt][4];
      int64_t si[kWalkPpt];
#pragma unroll
      for (int u = 0; u < kWalkPpt; ++u) {
        const int64_t k = p0 + u * kWalkThreads + threadIdx.x;
        si[u] = k < gn ? gf + k : -1;
        const int64_t s = si[u] >= 0 ? si[u] : gf;
#pragma unroll
        for (int a = 0; a < 3; ++a) xi[u][a] = (double)g.pos[3 * s + a];
#pragma unroll
        for (int a = 0; a < 4; ++a) ai[u][a] = 0.0;
      }
      if (threadIdx.x == 0) {
        s_stack[0] = 0;  // the root
        s_top = 1;
        s_over = 0;
      }
      __syncthreads();
      // Every round pops at least one cell and every cell is pushed at most once,
      // so the loop ends.  The pop count shrinks as the stack fills, so that the
      // children of the popped cells (at most 8 each) always fit; a stack that
      // still cannot take them is reported and the group's walk stops.
      for (;;) {
        const int top = s_top;
        if (top == 0 || s_over) break;
        const int npop = min(min(top, kWalkThreads), max(1, (kStackCap - top) / 8));
        int c = -1;
        if ((int)threadIdx.x < npop) c = s_stack[top - npop + threadIdx.x];
        __syncthreads();  // everyone has read its cell before the stack is rewritten
        // the test
        int accept = 0, leaf = 0, nch = 0, fch = 0;
        if (c >= 0) {
          const int cd = g.level[c];
          const bool contains = cd <= gd && (gkey >> (3 * (gd - cd))) == g.key[c];
          if (!contains) {
            double cen[3], l, d2 = 0.0;
            cell_centre(g, c, cen, l);
#pragma unroll
            for (int a = 0; a < 3; ++a) {
              const double t = fabs(cen[a] + g.com[4 * (int64_t)c + a] - gc[a]) - gh;
              if (t > 0.0) d2 += t * t;
            }
            accept = l * l < g.theta2 * d2;
          }
          if (!accept) {
            fch = g.child[2 * (int64_t)c];
            if (fch < 0)
              leaf = 1;
            else
              nch = g.child[2 * (int64_t)c + 1];
          }
        }
        int tot_c, tot_l, tot_p;
        const int pc = block_excl(accept, s_w, &tot_c);
        const int pl = block_excl(leaf, s_w, &tot_l);
        const int pp = block_excl(nch, s_w, &tot_p);
        const int base = top - npop;
        if (base + tot_p > kStackCap) {
          if (threadIdx.x == 0) s_over = 1;
        } else {
          for (int k = 0; k < nch; ++k) s_stack[base + pp + k] = fch + k;
        }
        if (accept) s_cells[pc] = c;
        if (leaf) s_leaves[pl] = c;
        if (threadIdx.x == 0) s_top = base + tot_p;
        __syncthreads();
        if (s_over) break;
        // particle ranges of the opened leaves
        int lc = 0;
        if ((int)threadIdx.x < tot_l) lc = g.count[s_leaves[threadIdx.x]];
        int tot_pairs;
        const int lp = block_excl(lc, s_w, &tot_pairs);
        if ((int)threadIdx.x < tot_l) s_lstart[threadIdx.x] = lp;
        if (threadIdx.x == 0) s_lstart[tot_l] = tot_pairs;
        __syncthreads();
        if (p0 == 0) {  // the lists are the same on every pass
          my_cells += (unsigned long long)tot_c;
          my_pairs += (unsigned long long)tot_pairs;
        }
        // cell terms, the accepted cells staged kCellBatch at a time (absolute
        // centre of mass, mass, quadrupole); each particle sums them in order
        for (int c0 = 0; c0 < tot_c; c0 += kCellBatch) {
          const int nc = min(kCellBatch, tot_c - c0);
          __syncthreads();  // the previous batch is consumed
          if ((int)threadIdx.x < nc) {
            const int64_t cc = s_cells[c0 + threadIdx.x];
            double cen[3], l;
            cell_centre(g, cc, cen, l);
#pragma unroll
            for (int a = 0; a < 3; ++a) s_cdat[threadIdx.x][a] = cen[a] + g.com[4 * cc + a];
            s_cdat[threadIdx.x][3] = g.com[4 * cc + 3];
#pragma unroll
            for (int q = 0; q < 6; ++q) s_cdat[threadIdx.x][4 + q] = g.quad[6 * cc + q];
          }
          __syncthreads();
#pragma unroll
          for (int u = 0; u < kWalkPpt; ++u) {
            if (si[u] < 0) continue;
            for (int k = 0; k < nc; ++k) {
              const double r0 = xi[u][0] - s_cdat[k][0];
              const double r1 = xi[u][1] - s_cdat[k][1];
              const double r2v = xi[u][2] - s_cdat[k][2];
              const double M = s_cdat[k][3];
              const double rr = r0 * r0 + r1 * r1 + r2v * r2v;
              const double rinv = 1.0 / sqrt(rr);
              const double rinv2 = rinv * rinv, rinv3 = rinv * rinv2;
              double t0 = -M * r0 * rinv3, t1 = -M * r1 * rinv3, t2 = -M * r2v * rinv3;
              double phi = -M * rinv;
              if (g.quad_on) {
                const double *Q = &s_cdat[k][4];
                const double q0 = Q[0] * r0 + Q[1] * r1 + Q[2] * r2v;
                const double q1 = Q[1] * r0 + Q[3] * r1 + Q[4] * r2v;
                const double q2 = Q[2] * r0 + Q[4] * r1 + Q[5] * r2v;
                const double rqr = r0 * q0 + r1 * q1 + r2v * q2;
                const double rinv5 = rinv3 * rinv2, rinv7 = rinv5 * rinv2;
                t0 += q0 * rinv5 - 2.5 * rqr * r0 * rinv7;
                t1 += q1 * rinv5 - 2.5 * rqr * r1 * rinv7;
                t2 += q2 * rinv5 - 2.5 * rqr * r2v * rinv7;
                phi -= 0.5 * rqr * rinv5;
              }
              ai[u][0] += t0;
              ai[u][1] += t1;
              ai[u][2] += t2;
              ai[u][3] += phi;
            }
          }
        }
        // particle terms, staged kPartBatch at a time
        for (int q0 = 0; q0 < tot_pairs; q0 += kPartBatch) {
          const int nb = min(kPartBatch, tot_pairs - q0);
          __syncthreads();
          for (int x = threadIdx.x; x < nb; x += kWalkThreads) {
            const int q = q0 + x;
            // the leaf holding pair slot q
            int lo = 0, hi = tot_l - 1;
            while (lo < hi) {
              const int mid = (lo + hi + 1) >> 1;
              if (s_lstart[mid] <= q)
                lo = mid;
              else
                hi = mid - 1;
            }
            const int64_t s = (int64_t)g.first[s_leaves[lo]] + (q - s_lstart[lo]);
            s_pidx[x] = (int32_t)s;
            s_part[x][0] = (double)g.pos[3 * s + 0];
            s_part[x][1] = (double)g.pos[3 * s + 1];
            s_part[x][2] = (double)g.pos[3 * s + 2];
            s_part[x][3] = (double)g.mass[s];
          }
          __syncthreads();
#pragma unroll
          for (int u = 0; u < kWalkPpt; ++u) {
            if (si[u] < 0) continue;
            for (int k = 0; k < nb; ++k) {
              if (s_pidx[k] == si[u]) continue;  // no self term
              const double r0 = xi[u][0] - s_part[k][0];
              const double r1 = xi[u][1] - s_part[k][1];
              const double r2v = xi[u][2] - s_part[k][2];
              const double rr = r0 * r0 + r1 * r1 + r2v * r2v + g.eps2;
              const double rinv = 1.0 / sqrt(rr);
              const double mr3 = s_part[k][3] * rinv * rinv * rinv;
              ai[u][0] -= mr3 * r0;
              ai[u][1] -= mr3 * r1;
              ai[u][2] -= mr3 * r2v;
              ai[u][3] -= s_part[k][3] * rinv;
            }
          }
        }
        __syncthreads();  // the round's LDS data is consumed before the next pop
      }
      if (s_over) {
        if (threadIdx.x == 0) atomicOr(status_word, TB_STATUS_INTERNAL);
      }
#pragma unroll
      for (int u = 0; u < kWalkPpt; ++u) {
        if (si[u] < 0) continue;
        double2 *o = reinterpret_cast<double2 *>(acc + 4 * si[u]);
        o[0] = make_double2(ai[u][0], ai[u][1]);
        o[1] = make_double2(ai[u][2], ai[u][3]);
      }
      __syncthreads();
    }
    if (threadIdx.x == 0 && stats) {
      // every group particle meets every listed cell and every listed particle
      // but itself
      atomicAdd(&stats[0], 1ull);
      atomicAdd(&stats[1], (unsigned long long)gn * (my_cells + my_pairs - 1ull));
    }
  }
}

size_t gravity_workspace_bytes(int64_t c_max) { return 4 * (size_t)c_max + 256; }

hipError_t launch_gravity(const GravIn &in, hipStream_t s) {
  GravArgs g;
  g.key = in.tree->cell_key;
  g.level = in.tree->cell_level;
  g.first = in.tree->cell_first;
  g.count = in.tree->cell_count;
  g.child = in.tree->child_ptr;
  g.com = static_cast<const double *>(in.tree->com);
  g.quad = static_cast<const double *>(in.tree->quad);
  g.box = in.tree->box_out;
  g.pos = in.pos_sorted;
  g.mass = in.mass_sorted;
  g.theta2 = in.theta * in.theta;
  g.eps2 = in.eps * in.eps;
  g.quad_on = in.quadrupole ? 1 : 0;
  g.hilbert = in.hilbert ? 1 : 0;
  int32_t *groups = static_cast<int32_t *>(in.workspace);
  uint32_t *n_groups = reinterpret_cast<uint32_t *>(groups + in.c_max);
  k_grav_init<<<1, 64, 0, s>>>(n_groups, reinterpret_cast<unsigned long long *>(in.stats));
  int64_t blocks = (in.c_max + 255) / 256;
  if (blocks > 4096) blocks = 4096;
  k_find_groups<<<(unsigned)blocks, 256, 0, s>>>(in.tree->n_cells, g.count, g.child, in.n_crit,
                                                 groups, n_groups);
  // a fixed grid of workgroups takes the groups in turn
  int64_t wg = in.n / 64 + 1;
  if (wg > 4096) wg = 4096;
  k_walk<<<(unsigned)wg, kWalkThreads, 0, s>>>(g, groups, n_groups, in.acc,
                                               reinterpret_cast<unsigned long long *>(in.stats),
                                               in.tree->status);
  return hipGetLastError();
}

}  // namespace tb
