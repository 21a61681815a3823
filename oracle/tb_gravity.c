/*
 * tb_gravity.c -- TEST INFRASTRUCTURE ONLY.
 *
 * CPU references for the gravity calculation that consumes the tree
 * (Sec. 2.1): a plain O(N^2) direct summation, and a sequential Barnes-Hut
 * walk with the opening criterion l/d < theta (eq. 1) and Barnes' shared
 * interaction lists for groups of at most n_crit particles.  Only the test
 * suite may load them; they share no code with the HIP implementation.
 *
 * Units G = 1.  Particle-particle terms use Plummer softening eps:
 *   a_i += -m_j (x_i - x_j) / (|x_i - x_j|^2 + eps^2)^(3/2)
 *   phi_i += -m_j / (|x_i - x_j|^2 + eps^2)^(1/2),     j != i.
 * An accepted cell C with mass M, centre of mass x_C and traceless quadrupole
 * Q = sum m (3 y y - |y|^2 I) about x_C acts through its expansion (unsoftened),
 * with r = x_i - x_C:
 *   phi += -M / r - (r.Q.r) / (2 r^5)
 *   a   += -M r / r^3 + (Q r) / r^5 - (5/2) (r.Q.r) r / r^7
 * (the quadrupole terms only when requested).
 *
 * Walk (readings where the paper is silent):
 *   - groups: going down from the root, the first cell on each path that holds
 *     at most n_crit particles, or is a leaf, is a group; its particles share
 *     one interaction list;
 *   - a cell C is accepted for group G when it is neither G nor an ancestor of
 *     G and l_C < theta * d, with d the distance from C's centre of mass to
 *     the closest point of G's cube (so l_C / d < theta holds for every
 *     particle of G); cells containing the group are always opened;
 *   - a cell that is not accepted is opened: a leaf gives its particles
 *     (direct terms), an internal cell its children, in key order.
 * Everything is FP64; the lists are summed in the order the depth-first walk
 * produces them.  Each particle also gets the sum of the magnitudes of its
 * acceleration terms, the scale against which summation error is measured.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>

#define TBG_OK 0
#define TBG_ERR_ARG (-1)
#define TBG_ERR_NOMEM (-7)

/* All-pairs direct summation: acc [n][4] = (ax, ay, az, phi) in input order. */
int tbg_direct(const float *pos, const float *mass, int64_t n, double eps, double *acc) {
  int64_t i, j;
  if (n < 0 || (n > 0 && (!pos || !mass || !acc))) return TBG_ERR_ARG;
  for (i = 0; i < n; ++i) {
    double xi = pos[3 * i], yi = pos[3 * i + 1], zi = pos[3 * i + 2];
    double ax = 0.0, ay = 0.0, az = 0.0, phi = 0.0;
    for (j = 0; j < n; ++j) {
      double dx, dy, dz, r2, rinv, rinv3;
      if (j == i) continue;
      dx = xi - (double)pos[3 * j];
      dy = yi - (double)pos[3 * j + 1];
      dz = zi - (double)pos[3 * j + 2];
      r2 = dx * dx + dy * dy + dz * dz + eps * eps;
      rinv = 1.0 / sqrt(r2);
      rinv3 = rinv * rinv * rinv;
      ax -= (double)mass[j] * dx * rinv3;
      ay -= (double)mass[j] * dy * rinv3;
      az -= (double)mass[j] * dz * rinv3;
      phi -= (double)mass[j] * rinv;
    }
    acc[4 * i + 0] = ax;
    acc[4 * i + 1] = ay;
    acc[4 * i + 2] = az;
    acc[4 * i + 3] = phi;
  }
  return TBG_OK;
}

/* Direct summation for the m particles idx[0..m) only (acc [m][4], same terms),
 * so that single outputs of very large sets can be checked one by one. */
int tbg_direct_subset(const float *pos, const float *mass, int64_t n, double eps,
                      const int64_t *idx, int64_t m, double *acc) {
  int64_t k, j;
  if (n < 0 || m < 0 || (m > 0 && (!pos || !mass || !idx || !acc))) return TBG_ERR_ARG;
  for (k = 0; k < m; ++k) {
    int64_t i = idx[k];
    double xi, yi, zi, ax = 0.0, ay = 0.0, az = 0.0, phi = 0.0;
    if (i < 0 || i >= n) return TBG_ERR_ARG;
    xi = pos[3 * i];
    yi = pos[3 * i + 1];
    zi = pos[3 * i + 2];
    for (j = 0; j < n; ++j) {
      double dx, dy, dz, r2, rinv, rinv3;
      if (j == i) continue;
      dx = xi - (double)pos[3 * j];
      dy = yi - (double)pos[3 * j + 1];
      dz = zi - (double)pos[3 * j + 2];
      r2 = dx * dx + dy * dy + dz * dz + eps * eps;
      rinv = 1.0 / sqrt(r2);
      rinv3 = rinv * rinv * rinv;
      ax -= (double)mass[j] * dx * rinv3;
      ay -= (double)mass[j] * dy * rinv3;
      az -= (double)mass[j] * dz * rinv3;
      phi -= (double)mass[j] * rinv;
    }
    acc[4 * k + 0] = ax;
    acc[4 * k + 1] = ay;
    acc[4 * k + 2] = az;
    acc[4 * k + 3] = phi;
  }
  return TBG_OK;
}

/* tb_oracle.c: cell coordinates of a Peano-Hilbert index */
void tbo_hilbert_decode(const uint64_t *h, int64_t n, int bits, uint32_t *q);

typedef struct {
  int curve; /* 0: Morton keys, 1: Peano-Hilbert keys */
  const uint64_t *key;
  const uint8_t *level;
  const int32_t *first, *count, *child;
  const double *com, *quad;
  const double *lo;
  double side;
  const double *x;  /* [n][3] sorted positions, FP64 */
  const double *m;  /* [n] sorted masses */
  double theta, eps;
  int quad_on;
  int64_t interactions; /* cell terms plus particle pairs, over all particles */
  /* the current group's interaction lists */
  int64_t *cells, ncells, cap_cells;
  int64_t *leaves, nleaves, cap_leaves;
  int failed;
} tbg_walk;

/* Geometric centre of cell c (box frame plus the box corner) and its side. */
static void cell_geometry(const tbg_walk *w, int64_t c, double cen[3], double *l) {
  uint32_t ijk[3] = {0u, 0u, 0u};
  int d = w->level[c], k, a;
  uint64_t key = w->key[c];
  double h = ldexp(w->side, -d);
  if (w->curve) {
    const uint64_t idx = key & (((uint64_t)1 << (3 * d)) - 1u);
    tbo_hilbert_decode(&idx, 1, d, ijk);
  } else {
    for (k = d - 1; k >= 0; --k) {
      uint32_t oct = (uint32_t)((key >> (3 * k)) & 7u);
      ijk[0] = (ijk[0] << 1) | ((oct >> 2) & 1u);
      ijk[1] = (ijk[1] << 1) | ((oct >> 1) & 1u);
      ijk[2] = (ijk[2] << 1) | (oct & 1u);
    }
  }
  for (a = 0; a < 3; ++a) cen[a] = w->lo[a] + ((double)ijk[a] + 0.5) * h;
  *l = h;
}

static int push(int64_t **v, int64_t *n, int64_t *cap, int64_t x) {
  if (*n == *cap) {
    int64_t nc = *cap ? 2 * *cap : 256;
    int64_t *nv = (int64_t *)realloc(*v, (size_t)nc * sizeof(int64_t));
    if (!nv) return -1;
    *v = nv;
    *cap = nc;
  }
  (*v)[(*n)++] = x;
  return 0;
}

/* Is cell c the group g or one of its ancestors? */
static int contains_group(const tbg_walk *w, int64_t c, int64_t g) {
  int dc = w->level[c], dg = w->level[g];
  if (dc > dg) return 0;
  return (w->key[g] >> (3 * (dg - dc))) == w->key[c];
}

/* Depth-first walk from cell c for group g (centre gc, half side gh). */
static void walk_cell(tbg_walk *w, int64_t c, int64_t g, const double gc[3], double gh) {
  int k;
  if (w->failed) return;
  if (!contains_group(w, c, g)) {
    double cen[3], l, d2 = 0.0;
    int a;
    cell_geometry(w, c, cen, &l);
    for (a = 0; a < 3; ++a) {
      double x = cen[a] + w->com[4 * c + a];
      double t = fabs(x - gc[a]) - gh;
      if (t > 0.0) d2 += t * t;
    }
    if (l * l < w->theta * w->theta * d2) {
      if (push(&w->cells, &w->ncells, &w->cap_cells, c)) w->failed = 1;
      return;
    }
  }
  if (w->child[2 * c] < 0) {
    if (push(&w->leaves, &w->nleaves, &w->cap_leaves, c)) w->failed = 1;
    return;
  }
  for (k = 0; k < w->child[2 * c + 1]; ++k) walk_cell(w, w->child[2 * c] + k, g, gc, gh);
}

/* The forces on the particles of group g from its interaction lists. */
static void group_forces(tbg_walk *w, int64_t g, double *acc) {
  int64_t s, k, j, pairs = 0;
  for (k = 0; k < w->nleaves; ++k) pairs += w->count[w->leaves[k]];
  /* every particle meets each listed cell and every listed particle but itself */
  w->interactions += (int64_t)w->count[g] * (w->ncells + pairs - 1);
  for (s = w->first[g]; s < w->first[g] + w->count[g]; ++s) {
    const double *xi = &w->x[3 * s];
    double a[3] = {0.0, 0.0, 0.0}, phi = 0.0, mag = 0.0;
    for (k = 0; k < w->ncells; ++k) {
      int64_t c = w->cells[k];
      double cen[3], l, r[3], r2, rinv, rinv2, rinv3, M = w->com[4 * c + 3], t[3];
      int q;
      cell_geometry(w, c, cen, &l);
      for (q = 0; q < 3; ++q) r[q] = xi[q] - (cen[q] + w->com[4 * c + q]);
      r2 = r[0] * r[0] + r[1] * r[1] + r[2] * r[2];
      rinv = 1.0 / sqrt(r2);
      rinv2 = rinv * rinv;
      rinv3 = rinv * rinv2;
      for (q = 0; q < 3; ++q) t[q] = -M * r[q] * rinv3;
      phi -= M * rinv;
      if (w->quad_on) {
        const double *Q = &w->quad[6 * c];
        double Qr[3], rQr, rinv5, rinv7;
        Qr[0] = Q[0] * r[0] + Q[1] * r[1] + Q[2] * r[2];
        Qr[1] = Q[1] * r[0] + Q[3] * r[1] + Q[4] * r[2];
        Qr[2] = Q[2] * r[0] + Q[4] * r[1] + Q[5] * r[2];
        rQr = r[0] * Qr[0] + r[1] * Qr[1] + r[2] * Qr[2];
        rinv5 = rinv3 * rinv2;
        rinv7 = rinv5 * rinv2;
        for (q = 0; q < 3; ++q) t[q] += Qr[q] * rinv5 - 2.5 * rQr * r[q] * rinv7;
        phi -= 0.5 * rQr * rinv5;
      }
      for (q = 0; q < 3; ++q) a[q] += t[q];
      mag += sqrt(t[0] * t[0] + t[1] * t[1] + t[2] * t[2]);
    }
    for (k = 0; k < w->nleaves; ++k) {
      int64_t c = w->leaves[k];
      for (j = w->first[c]; j < w->first[c] + w->count[c]; ++j) {
        double r[3], r2, rinv, rinv3, t[3];
        int q;
        if (j == s) continue;
        for (q = 0; q < 3; ++q) r[q] = xi[q] - w->x[3 * j + q];
        r2 = r[0] * r[0] + r[1] * r[1] + r[2] * r[2] + w->eps * w->eps;
        rinv = 1.0 / sqrt(r2);
        rinv3 = rinv * rinv * rinv;
        for (q = 0; q < 3; ++q) t[q] = -w->m[j] * r[q] * rinv3;
        phi -= w->m[j] * rinv;
        for (q = 0; q < 3; ++q) a[q] += t[q];
        mag += sqrt(t[0] * t[0] + t[1] * t[1] + t[2] * t[2]);
      }
    }
    acc[5 * s + 0] = a[0];
    acc[5 * s + 1] = a[1];
    acc[5 * s + 2] = a[2];
    acc[5 * s + 3] = phi;
    acc[5 * s + 4] = mag;
  }
}

/* Walks every group below cell c. */
static void walk_groups(tbg_walk *w, int64_t c, int32_t n_crit, double *acc, int64_t *ngroups) {
  int k;
  if (w->failed) return;
  if (w->count[c] <= n_crit || w->child[2 * c] < 0) {
    double gc[3], l;
    cell_geometry(w, c, gc, &l);
    w->ncells = w->nleaves = 0;
    walk_cell(w, 0, c, gc, 0.5 * l);
    if (!w->failed) group_forces(w, c, acc);
    *ngroups += 1;
    return;
  }
  for (k = 0; k < w->child[2 * c + 1]; ++k) walk_groups(w, w->child[2 * c] + k, n_crit, acc,
                                                        ngroups);
}

/*
 * Tree walk over a tree in the layout of tbo_build (cells by (depth, key), com
 * relative to the cell centre, quad, child_ptr {first, n}).
 *   pos, mass       original particle arrays; perm maps sorted -> original
 *   acc [n][5]      out: (ax, ay, az, phi, sum of |term|) in sorted order
 *   stats [2]       out (may be NULL): groups, and interactions (cells +
 *                   particle pairs) summed over particles
 *   curve           0: the cell keys are Morton keys, 1: Peano-Hilbert keys
 */
int tbg_walk_tree_curve(const float *pos, const float *mass, const int32_t *perm, int64_t n,
                        const uint64_t *cell_key, const uint8_t *cell_level,
                        const int32_t *cell_first, const int32_t *cell_count,
                        const int32_t *child_ptr, const double *com, const double *quad,
                        const double lo[3], double side, double theta, int32_t n_crit,
                        double eps, int quad_on, int curve, double *acc, int64_t *stats) {
  tbg_walk w;
  double *x = NULL, *m = NULL;
  int64_t s, groups = 0;
  if (n < 0 || n_crit < 1 || !(theta >= 0.0) || !(eps >= 0.0) || curve < 0 || curve > 1)
    return TBG_ERR_ARG;
  if (n == 0) return TBG_OK;
  if (!pos || !mass || !perm || !cell_key || !cell_level || !cell_first || !cell_count ||
      !child_ptr || !com || !quad || !lo || !acc)
    return TBG_ERR_ARG;
  x = (double *)malloc((size_t)n * 3 * sizeof(double));
  m = (double *)malloc((size_t)n * sizeof(double));
  if (!x || !m) {
    free(x);
    free(m);
    return TBG_ERR_NOMEM;
  }
  for (s = 0; s < n; ++s) {
    int32_t p = perm[s];
    x[3 * s + 0] = pos[3 * (int64_t)p + 0];
    x[3 * s + 1] = pos[3 * (int64_t)p + 1];
    x[3 * s + 2] = pos[3 * (int64_t)p + 2];
    m[s] = mass[p];
  }
  w.curve = curve;
  w.key = cell_key;
  w.level = cell_level;
  w.first = cell_first;
  w.count = cell_count;
  w.child = child_ptr;
  w.com = com;
  w.quad = quad;
  w.lo = lo;
  w.side = side;
  w.x = x;
  w.m = m;
  w.theta = theta;
  w.eps = eps;
  w.quad_on = quad_on;
  w.cells = w.leaves = NULL;
  w.ncells = w.nleaves = w.cap_cells = w.cap_leaves = 0;
  w.failed = 0;
  w.interactions = 0;
  walk_groups(&w, 0, n_crit, acc, &groups);
  if (stats) {
    stats[0] = groups;
    stats[1] = w.interactions;
  }
  free(w.cells);
  free(w.leaves);
  free(x);
  free(m);
  return w.failed ? TBG_ERR_NOMEM : TBG_OK;
}

int tbg_walk_tree(const float *pos, const float *mass, const int32_t *perm, int64_t n,
                  const uint64_t *cell_key, const uint8_t *cell_level, const int32_t *cell_first,
                  const int32_t *cell_count, const int32_t *child_ptr, const double *com,
                  const double *quad, const double lo[3], double side, double theta,
                  int32_t n_crit, double eps, int quad_on, double *acc, int64_t *stats) {
  return tbg_walk_tree_curve(pos, mass, perm, n, cell_key, cell_level, cell_first, cell_count,
                             child_ptr, com, quad, lo, side, theta, n_crit, eps, quad_on, 0, acc,
                             stats);
}
